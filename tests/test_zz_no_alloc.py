"""The allocation-free network evaluation (mlp_forward_noalloc, whose work
area is a fixed device array) against mlp_forward on the same rows: two calls
in a row, the second with fewer rows, equal bit for bit (same kernels, same
per-row arithmetic; only the work buffers differ)."""
import numpy as np
import pytest
import torch

from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_13264_amd as nm
    return nm


@pytest.mark.parametrize("n_in,width,n_out,rows", [(8, 256, 1, (50000, 3000)),
                                                  (5, 96, 3, (20000, 77)),
                                                  (40, 64, 2, (70000, 1000)),
                                                  (8, 300, 1, (30000, 65))])
def test_noalloc_forward_equals_forward(nm, n_in, width, n_out, rows):
    say(f"[no-alloc] net {n_in}-{width}-{n_out}, rows {rows}")
    net = nm.MLP(n_in, width, n_out, seed=11)
    rng = np.random.default_rng(width)
    for n in rows:
        X = torch.as_tensor(rng.normal(size=(n, n_in)), dtype=torch.float32, device="cuda")
        Y_ref = torch.full((n, n_out), np.nan, dtype=torch.float32, device="cuda")
        Y = torch.full((n, n_out), np.nan, dtype=torch.float32, device="cuda")
        net.forward(X, Y_ref)
        net.forward_noalloc(X, Y)
        torch.cuda.synchronize()
        assert torch.isfinite(Y).all()
        assert torch.equal(Y, Y_ref)
    net.close()
