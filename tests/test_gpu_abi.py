"""GPU: the C ABI's error behaviour, forced from the host (call order, bad
arguments, iteration caps, non-finite inputs); every kernel still runs to
completion and the context stays usable where the header says so."""
import numpy as np
import pytest
import torch

import synth

from gpu_helpers import T, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_13264_amd as nm
    return nm


def _system(o=2, v=4, naux=18):
    return synth.make_system(o, v, naux, synth.exact_check_seed(o, v))


def test_call_order_is_enforced(nm):
    say("[abi] call order")
    sysd = _system()
    ctx = nm.Context(2, 4, 18, T(sysd["eps"]), T(sysd["B"]))
    with pytest.raises(nm.CCError) as e:
        ctx.eom(nm.CC_BOTH, 2)
    assert e.value.code == -2
    with pytest.raises(nm.CCError) as e:
        ctx.multipliers([(1, 2)])
    assert e.value.code == -2
    ctx.ground()
    with pytest.raises(nm.CCError) as e:
        ctx.multipliers([(1, 2)])           # needs both EOM sides
    assert e.value.code == -2
    ctx.eom(nm.CC_RIGHT, 2)
    with pytest.raises(nm.CCError) as e:
        ctx.multipliers([(1, 2)])           # left states still missing
    assert e.value.code == -2
    ctx.eom(nm.CC_LEFT, 2)
    with pytest.raises(nm.CCError) as e:
        ctx.densities(1, 2)
    assert e.value.code == -2
    with pytest.raises(nm.CCError) as e:
        ctx.nacme(1, 2, T(np.zeros((1, 6, 6))), T(np.zeros((1, 18, 6, 6))))
    assert e.value.code == -2
    # the context is still usable: the full chain now succeeds
    ctx.multipliers([(1, 2)])
    ctx.densities(1, 2)
    F = ctx.nacme(1, 2, T(np.zeros((1, 6, 6))), T(np.zeros((1, 18, 6, 6))))
    assert F[0] == 0.0
    ctx.close()


def test_bad_arguments_are_rejected(nm):
    say("[abi] bad arguments")
    sysd = _system()
    with pytest.raises(nm.CCError) as e:
        nm.Context(0, 4, 18, T(sysd["eps"]), T(sysd["B"]))
    assert e.value.code == -1
    eps = sysd["eps"].copy()
    eps[1] = np.nan
    with pytest.raises(nm.CCError) as e:
        nm.Context(2, 4, 18, T(eps), T(sysd["B"]))
    assert e.value.code == -1
    with pytest.raises(nm.CCError) as e:
        nm.Context(2, 4, 18, T(sysd["eps"]), T(sysd["B"]), nm.default_opts(precision=7))
    assert e.value.code == -1
    ctx = nm.Context(2, 4, 18, T(sysd["eps"]), T(sysd["B"]))
    ctx.ground()
    with pytest.raises(nm.CCError) as e:
        ctx.eom(4, 2)                   # no such side
    assert e.value.code == -1
    ctx.eom(nm.CC_BOTH, 2)
    for pl in [[(3, 1)], [(0, 3)], [(1, -1)], [(1, 2), (2, 1), (1, 2)], []]:
        with pytest.raises(nm.CCError) as e:
            ctx.multipliers(pl)
        assert e.value.code == -1
    ctx.close()


def test_iteration_cap_reports_not_converged(nm):
    say("[abi] maxit")
    sysd = _system()
    ctx = nm.Context(2, 4, 18, T(sysd["eps"]), T(sysd["B"]), nm.default_opts(maxit=2))
    e, it, rc = ctx.ground()
    assert rc == 1 and it == 2 and np.isfinite(e)
    ctx.close()
    ctx = nm.Context(2, 4, 18, T(sysd["eps"]), T(sysd["B"]))
    e_ref, _, rc = ctx.ground()
    assert rc == 0
    ctx.close()
    ctx = nm.Context(2, 4, 18, T(sysd["eps"]), T(sysd["B"]), nm.default_opts(maxit=2))
    ctx.set_guess(nm._lib.CC_T, 0, torch.zeros(8 + 64, dtype=torch.float64, device="cuda"))
    e2, it2, rc2 = ctx.ground()
    assert rc2 == 1 and abs(e2 - e_ref) > 0.0
    ctx.close()


def test_non_finite_integrals_are_reported(nm):
    say("[abi] non-finite integrals")
    sysd = _system()
    B = sysd["B"].copy()
    B[0, 2, 3] = B[0, 3, 2] = np.inf
    ctx = nm.Context(2, 4, 18, T(sysd["eps"]), T(B))
    with pytest.raises(nm.CCError) as e:
        ctx.ground()
    assert e.value.code == -5
    ctx.close()
