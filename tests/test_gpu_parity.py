"""GPU parity: the library (through its C ABI) against the fp64 oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import ccsd
from oracle import response as rs

from gpu_helpers import T, oracle_state, say, to_full, to_packed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_13264_amd as nm
    return nm


CONTRACTIONS = [
    ("ijcd,acbd->ijab", [(3, 5, 7, 9), (13, 7, 11, 9)], (3, 5, 13, 11)),       # ladder
    ("pP,PQRS->pQRS", [(7, 7), (7, 6, 5, 4)], (7, 6, 5, 4)),                  # index transform
    ("qQ,pQRS->pqRS", [(6, 6), (5, 6, 4, 3)], (5, 6, 4, 3)),                  # batched (promoted)
    ("pqrS,sS->pqrs", [(4, 5, 6, 7), (3, 7)], (4, 5, 6, 3)),                  # transposed B
    ("kicd,adkc->ia", [(3, 4, 5, 6), (7, 6, 3, 5)], (4, 7)),                  # split-K shaped
    ("ia,jb->ijab", [(3, 5), (4, 6)], (3, 4, 5, 6)),                          # outer product
    ("ijab,iajb->", [(3, 4, 5, 6), (3, 5, 4, 6)], ()),                        # full contraction
    ("iiaa,ia->ia", [(3, 3, 5, 5), (3, 5)], (3, 5)),                          # diagonal + batch
    ("zik,zkj->zij", [(5, 33, 17), (5, 17, 70)], (5, 33, 70)),               # explicit batch
    ("ak,kx->ax", [(70, 4100), (4100, 3)], (70, 3)),                         # long K, split
    ("ik,kj->ij", [(300, 70), (70, 260)], (300, 260)),                       # 128-tile, ragged
    ("ki,kj->ij", [(70, 300), (70, 260)], (300, 260)),                       # 128-tile, A^T
    ("ik,jk->ij", [(300, 70), (260, 70)], (300, 260)),                       # 128-tile, B^T
    ("ki,jk->ij", [(70, 300), (260, 70)], (300, 260)),                       # 128-tile, both
    ("zik,zkj->zij", [(3, 130, 41), (3, 41, 140)], (3, 130, 140)),           # 128-tile, batch
    ("ijcd,cdab->ijab", [(4, 33, 13, 11), (13, 11, 12, 15)], (4, 33, 12, 15)),  # ladder, 128-tile
    ("ik,kj->ij", [(256, 64), (64, 1024)], (256, 1024)),                     # 8-divisible grid
    # short contracted range, large operand with no GEMM-shaped layout (the
    # short-K kernels): lanes along an x label, along an f label, two k labels
    ("ikab,zkj->zijab", [(8, 33, 64, 64), (2, 33, 9)], (2, 8, 9, 64, 64)),
    ("ijal,zlb->zijab", [(16, 16, 128, 33), (2, 33, 48)], (2, 16, 16, 128, 48)),
    ("aikbc,kc->iab", [(48, 8, 4, 48, 15), (4, 15)], (8, 48, 48)),
]


@pytest.mark.parametrize("spec,shapes,oshape", CONTRACTIONS)
def test_contract_matches_torch(nm, spec, shapes, oshape):
    say(f"[contract] {spec}")
    rng = np.random.default_rng(len(spec))
    A = T(rng.normal(size=shapes[0]))
    B = T(rng.normal(size=shapes[1]))
    C0 = rng.normal(size=oshape) if oshape else rng.normal(size=(1,))
    C = T(C0.reshape(oshape) if oshape else C0)
    la, rest = spec.split(",")
    lb, lc = rest.split("->")
    Ac, Bc = A.cpu(), B.cpu()
    if la == "iiaa":
        Ac = torch.einsum("iiaa->ia", Ac)
        ref = torch.einsum("ia,ia->ia", Ac, Bc)
    else:
        ref = torch.einsum(spec, Ac, Bc)
    ref = 0.7 * ref + 0.3 * torch.as_tensor(C0.reshape(oshape) if oshape else C0[0])
    nm.contract(spec, 0.7, A, B, 0.3, C)
    torch.cuda.synchronize()
    err = (C.cpu().reshape(ref.shape) - ref).abs().max().item()
    assert err < 1e-11 * max(1.0, ref.abs().max().item())


@pytest.mark.parametrize("o,v", [(1, 4), (2, 3), (3, 5), (4, 12)])
def test_residual_matches_oracle(nm, o, v):
    say(f"[residual] o={o} v={v}")
    naux = 3 * (o + v)
    sysd = synth.make_system(o, v, naux, synth.exact_check_seed(o, v))
    h, g = rs.system_hamiltonian(sysd["eps"], sysd["B"], o)
    t1, t2 = synth.random_amplitudes(o, v, seed=5, scale=0.1)
    om1, om2 = ccsd.residual(torch.as_tensor(t1), torch.as_tensor(t2), h, g)
    ref = np.concatenate([om1.numpy().ravel(), om2.numpy().ravel()])
    ctx = nm.Context(o, v, naux, T(sysd["eps"]), T(sysd["B"]))
    out = torch.zeros(ref.size, dtype=torch.float64, device="cuda")
    ctx.residual(T(np.concatenate([t1.ravel(), t2.ravel()])), out)
    torch.cuda.synchronize()
    assert np.abs(out.cpu().numpy() - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
    ctx.close()


@pytest.mark.parametrize("o,v", [(2, 3), (3, 5)])
def test_jacobian_transforms_match_oracle(nm, o, v):
    say(f"[jacobian] o={o} v={v}")
    naux = 3 * (o + v)
    st = oracle_state(o, v, naux, synth.exact_check_seed(o, v), 2)
    sysd = st["sys"]
    ctx = nm.Context(o, v, naux, T(sysd["eps"]), T(sysd["B"]))
    ctx.ground()
    x = np.random.default_rng(3).normal(size=st["x"].numel())
    y = torch.zeros(o * v + (o * v) ** 2, dtype=torch.float64, device="cuda")
    ctx.apply_jacobian(nm.CC_RIGHT, T(to_full(x, o, v)), y)
    ref = rs.right_transform(st["x"], torch.as_tensor(x), st["h"], st["g"], o, v).numpy()
    assert np.abs(to_packed(y.cpu().numpy(), o, v) - ref).max() < 1e-9
    ctx.apply_jacobian(nm.CC_LEFT, T(to_full(x, o, v)), y)
    ref = rs.left_transform(st["x"], torch.as_tensor(x), st["h"], st["g"], o, v).numpy()
    assert np.abs(to_packed(y.cpu().numpy(), o, v) - ref).max() < 1e-9
    ctx.close()


@pytest.mark.parametrize("o,v,naux,seed", [(1, 5, 18, None), (2, 4, 18, None), (4, 12, 48, 2301)])
def test_pipeline_matches_oracle(nm, o, v, naux, seed):
    say(f"[pipeline] o={o} v={v} naux={naux}")
    seed = synth.exact_check_seed(o, v) if seed is None else seed
    nroots = 2
    st = oracle_state(o, v, naux, seed, nroots)
    sysd = st["sys"]
    n = o + v
    dirs = synth.make_directions(n, naux, seed + 17, 2)
    ctx = nm.Context(o, v, naux, T(sysd["eps"]), T(sysd["B"]))
    e, it, rc = ctx.ground()
    assert rc == 0
    e_hf_ref = float(ccsd.energy(torch.zeros(o, v, dtype=torch.float64),
                                 torch.zeros(o, o, v, v, dtype=torch.float64), st["h"], st["g"]))
    assert abs((e + e_hf_ref) - st["E0"]) < 1e-9
    w, _, rc = ctx.eom(nm.CC_BOTH, nroots)
    assert rc == 0
    assert np.abs(np.array(w) - st["omega"].numpy()).max() < 1e-9
    Nf = o * v + (o * v) ** 2
    buf = torch.zeros(Nf, dtype=torch.float64, device="cuda")
    for k in range(nroots):
        R = to_packed(ctx.export(nm._lib.CC_R, k + 1, 0, buf).cpu().numpy(), o, v)
        L = to_packed(ctx.export(nm._lib.CC_L, k + 1, 0, buf).cpu().numpy(), o, v)
        assert np.abs(R - st["R"][k].numpy()).max() < 1e-7
        assert np.abs(L - st["L"][k].numpy()).max() < 1e-7
        assert abs(ctx.export_r0(k + 1) - float(st["R0"][k])) < 1e-8
    # both ordered pairs in one call: their zeta equations share the block solver
    its, rc = ctx.multipliers([(1, 2), (2, 1)])
    assert rc == 0 and all(z > 0 for z, _ in its)
    for (i, j) in [(0, 1), (1, 0)]:
        m = rs.multipliers(st, i, j, relaxed=True)
        eta = to_packed(ctx.export(nm._lib.CC_ETA_T, i + 1, j + 1, buf).cpu().numpy(), o, v)
        assert np.abs(eta - m["eta_t"].numpy()).max() < 1e-7
        zeta = to_packed(ctx.export(nm._lib.CC_ZETA, i + 1, j + 1, buf).cpu().numpy(), o, v)
        assert np.abs(zeta - m["zeta"].numpy()).max() < 1e-7
        kb = torch.zeros(o * v, dtype=torch.float64, device="cuda")
        ek = ctx.export(nm._lib.CC_ETA_K, i + 1, j + 1, kb).cpu().numpy().reshape(o, v)
        assert np.abs(ek - m["eta_kappa"].numpy()).max() < 1e-7
        kb = ctx.export(nm._lib.CC_KAPPA, i + 1, j + 1, kb).cpu().numpy().reshape(o, v)
        assert np.abs(kb - m["kappa_bar"].numpy()).max() < 1e-7
        D1 = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        ctx.densities(i + 1, j + 1, D1)
        Dref, dref = rs.effective_densities(st, m, j)
        Dg = D1.cpu().numpy()
        assert np.abs(0.5 * (Dg + Dg.T) - Dref.numpy()).max() < 1e-7
        F = ctx.nacme(i + 1, j + 1, T(dirs["dh"]), T(dirs["dB"]))
        for q in range(2):
            dg = np.einsum("Ppq,Prs->pqrs", dirs["dB"][q], dirs["dB"][q])
            Fo = rs.coupling_direct(st, m, j, dirs["dh"][q], dg)
            assert abs(F[q] - Fo) < 1e-7 * max(1.0, abs(Fo))
    ctx.close()


@pytest.mark.parametrize("o,v,naux,seed", [(1, 5, 18, None), (2, 4, 18, None), (4, 12, 48, 2301)])
def test_ground_pair_couplings_match_oracle(nm, o, v, naux, seed):
    """F_i0: excited left state i, CC ground state on the right (j = 0)."""
    say(f"[ground pair] o={o} v={v}")
    seed = synth.exact_check_seed(o, v) if seed is None else seed
    st = oracle_state(o, v, naux, seed, 2)
    sysd = st["sys"]
    n = o + v
    dirs = synth.make_directions(n, naux, seed + 17, 2)
    ctx = nm.Context(o, v, naux, T(sysd["eps"]), T(sysd["B"]))
    ctx.ground()
    ctx.eom(nm.CC_BOTH, 2)
    Nf = o * v + (o * v) ** 2
    buf = torch.zeros(Nf, dtype=torch.float64, device="cuda")
    for i in range(2):
        m = rs.multipliers(st, i, rs.GROUND, relaxed=True)
        ctx.multipliers([(i + 1, 0)])
        zeta = to_packed(ctx.export(nm._lib.CC_ZETA, i + 1, 0, buf).cpu().numpy(), o, v)
        assert np.abs(zeta - m["zeta"].numpy()).max() < 1e-7
        kb = torch.zeros(o * v, dtype=torch.float64, device="cuda")
        ek = ctx.export(nm._lib.CC_ETA_K, i + 1, 0, kb).cpu().numpy().reshape(o, v)
        assert np.abs(ek - m["eta_kappa"].numpy()).max() < 1e-7
        kb = ctx.export(nm._lib.CC_KAPPA, i + 1, 0, kb).cpu().numpy().reshape(o, v)
        assert np.abs(kb - m["kappa_bar"].numpy()).max() < 1e-7
        D1 = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        ctx.densities(i + 1, 0, D1)
        Dref, _ = rs.effective_densities(st, m, rs.GROUND)
        Dg = D1.cpu().numpy()
        assert np.abs(0.5 * (Dg + Dg.T) - Dref.numpy()).max() < 1e-7
        F = ctx.nacme(i + 1, 0, T(dirs["dh"]), T(dirs["dB"]))
        for q in range(2):
            dg = np.einsum("Ppq,Prs->pqrs", dirs["dB"][q], dirs["dB"][q])
            Fo = rs.coupling_direct(st, m, rs.GROUND, dirs["dh"][q], dg)
            assert abs(F[q] - Fo) < 1e-7 * max(1.0, abs(Fo))
    ctx.close()


@pytest.mark.parametrize("o,v,naux,seed", [(1, 5, 18, None), (2, 4, 18, None), (4, 12, 48, 2301)])
def test_ground_bra_couplings_match_oracle(nm, o, v, naux, seed):
    """F_0j: the ground-state left state <HF|(1 + Lambda) exp(-T) on the left,
    excited right state j; both pairs (0, 1), (0, 2) in one multipliers call
    (Lambda solved once), with an excited pair beside them."""
    say(f"[ground bra] o={o} v={v}")
    seed = synth.exact_check_seed(o, v) if seed is None else seed
    st = oracle_state(o, v, naux, seed, 2)
    sysd = st["sys"]
    n = o + v
    dirs = synth.make_directions(n, naux, seed + 17, 2)
    ctx = nm.Context(o, v, naux, T(sysd["eps"]), T(sysd["B"]))
    ctx.ground()
    ctx.eom(nm.CC_BOTH, 2)
    Nf = o * v + (o * v) ** 2
    buf = torch.zeros(Nf, dtype=torch.float64, device="cuda")
    its, rc = ctx.multipliers([(0, 1), (1, 2), (0, 2)])
    assert rc == 0
    for j in range(2):
        m = rs.multipliers(st, rs.GROUND, j, relaxed=True)
        eta = to_packed(ctx.export(nm._lib.CC_ETA_T, 0, j + 1, buf).cpu().numpy(), o, v)
        assert np.abs(eta - m["eta_t"].numpy()).max() < 1e-7 * max(1.0, float(m["eta_t"].abs().max()))
        zeta = to_packed(ctx.export(nm._lib.CC_ZETA, 0, j + 1, buf).cpu().numpy(), o, v)
        assert np.abs(zeta - m["zeta"].numpy()).max() < 1e-7 * max(1.0, float(m["zeta"].abs().max()))
        kb = torch.zeros(o * v, dtype=torch.float64, device="cuda")
        ek = ctx.export(nm._lib.CC_ETA_K, 0, j + 1, kb).cpu().numpy().reshape(o, v)
        assert np.abs(ek - m["eta_kappa"].numpy()).max() < 1e-7
        kb = ctx.export(nm._lib.CC_KAPPA, 0, j + 1, kb).cpu().numpy().reshape(o, v)
        assert np.abs(kb - m["kappa_bar"].numpy()).max() < 1e-7
        D1 = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        ctx.densities(0, j + 1, D1)
        Dref, _ = rs.effective_densities(st, m, j)
        Dg = D1.cpu().numpy()
        assert np.abs(0.5 * (Dg + Dg.T) - Dref.numpy()).max() < 1e-7
        F = ctx.nacme(0, j + 1, T(dirs["dh"]), T(dirs["dB"]))
        for q in range(2):
            dg = np.einsum("Ppq,Prs->pqrs", dirs["dB"][q], dirs["dB"][q])
            Fo = rs.coupling_direct(st, m, j, dirs["dh"][q], dg)
            assert abs(F[q] - Fo) < 1e-7 * max(1.0, abs(Fo))
    ctx.close()


@pytest.mark.parametrize("o,v,naux,seed", [(1, 5, 18, None), (2, 4, 18, None), (4, 12, 48, 2301)])
def test_energy_gradients_match_oracle(nm, o, v, naux, seed):
    """dE_j/dlambda (pairs (j, j)) of the ground and two excited states, and the
    branching-plane vectors built from them, against the oracle."""
    say(f"[energy gradients] o={o} v={v}")
    seed = synth.exact_check_seed(o, v) if seed is None else seed
    st = oracle_state(o, v, naux, seed, 2)
    sysd = st["sys"]
    n = o + v
    dirs = synth.make_directions(n, naux, seed + 17, 2)
    ctx = nm.Context(o, v, naux, T(sysd["eps"]), T(sysd["B"]))
    ctx.ground()
    # the ground-state gradient needs no EOM states
    ctx.multipliers([(0, 0)])
    w, _, _ = ctx.eom(nm.CC_BOTH, 2)
    Nf = o * v + (o * v) ** 2
    buf = torch.zeros(Nf, dtype=torch.float64, device="cuda")
    grads = {}
    for jj, jo in [(0, rs.GROUND), (1, 0), (2, 1)]:
        m = rs.gradient_multipliers(st, jo, relaxed=True)
        if jj > 0:
            ctx.multipliers([(jj, jj)])
        zeta = to_packed(ctx.export(nm._lib.CC_ZETA, jj, jj, buf).cpu().numpy(), o, v)
        assert np.abs(zeta - m["zeta"].numpy()).max() < 1e-7
        kb = torch.zeros(o * v, dtype=torch.float64, device="cuda")
        kb = ctx.export(nm._lib.CC_KAPPA, jj, jj, kb).cpu().numpy().reshape(o, v)
        assert np.abs(kb - m["kappa_bar"].numpy()).max() < 1e-7
        ctx.densities(jj, jj)
        G = ctx.nacme(jj, jj, T(dirs["dh"]), T(dirs["dB"]))
        for q in range(2):
            dg = np.einsum("Ppq,Prs->pqrs", dirs["dB"][q], dirs["dB"][q])
            Go = rs.energy_gradient(st, m, dirs["dh"][q], dg)
            assert abs(G[q] - Go) < 1e-7 * max(1.0, abs(Go))
        grads[jj] = np.asarray(G)
    # branching plane: g = grad(E2 - E1), h = (E2 - E1) F_12
    ctx.multipliers([(1, 2)])
    ctx.densities(1, 2)
    F12 = np.asarray(ctx.nacme(1, 2, T(dirs["dh"]), T(dirs["dB"])))
    for q in range(2):
        dg = np.einsum("Ppq,Prs->pqrs", dirs["dB"][q], dirs["dB"][q])
        g_ref = (rs.energy_gradient(st, rs.gradient_multipliers(st, 1), dirs["dh"][q], dg)
                 - rs.energy_gradient(st, rs.gradient_multipliers(st, 0), dirs["dh"][q], dg))
        assert abs((grads[2][q] - grads[1][q]) - g_ref) < 1e-7 * max(1.0, abs(g_ref))
        h_ref = float(st["omega"][1] - st["omega"][0]) * rs.coupling_direct(
            st, rs.multipliers(st, 0, 1), 1, dirs["dh"][q], dg)
        assert abs((w[1] - w[0]) * F12[q] - h_ref) < 1e-7 * max(1.0, abs(h_ref))
    ctx.close()


@pytest.mark.parametrize("spec,shapes,oshape", [
    ("ik,kj->ij", [(300, 70), (70, 260)], (300, 260)),
    ("ki,jk->ij", [(70, 300), (260, 70)], (300, 260)),
    ("ijcd,cdab->ijab", [(4, 33, 13, 11), (13, 11, 12, 15)], (4, 33, 12, 15)),
    ("ak,kx->ax", [(70, 4100), (4100, 3)], (70, 3)),                         # split K
    ("kicd,adkc->ia", [(5, 33, 20, 31), (127, 31, 5, 20)], (33, 127)),       # split K, packed
    ("zik,zkj->zij", [(3, 130, 41), (3, 41, 140)], (3, 130, 140)),           # batched
    ("ik,kj->ij", [(257, 1000), (1000, 300)], (257, 300)),                   # several K tiles
    ("iak,kjb->ijab", [(20, 30, 64), (64, 25, 35)], (20, 25, 30, 35)),       # rows and columns interleaved
    ("iak,kjb->ijab", [(6, 10, 4100), (4100, 7, 9)], (6, 7, 10, 9)),         # the same, split K
])
@pytest.mark.parametrize("prec", [1, 2])
def test_contract_low_precision_operands(nm, spec, shapes, oshape, prec):
    """Mixed-precision contraction, fp32 operands (prec 1) or bfloat16 pairs
    with three bf16 products (prec 2), fp32 accumulation: error at the level of
    the operand rounding (2^-24 resp. about 3 * 2^-16 of each product), and
    non-zero (the low-precision kernel really ran)."""
    say(f"[contract prec={prec}] {spec}")
    rng = np.random.default_rng(3)
    A = T(rng.normal(size=shapes[0]))
    B = T(rng.normal(size=shapes[1]))
    C = torch.zeros(oshape, dtype=torch.float64, device="cuda")
    nm.contract(spec, 1.0, A, B, 0.0, C, precision=prec)
    torch.cuda.synchronize()
    ref = torch.einsum(spec, A.cpu(), B.cpu())
    k = np.prod(shapes[0]) * np.prod(shapes[1]) / np.prod(oshape) if oshape else 1
    err = (C.cpu() - ref).abs().max().item()
    rel = 1e-5 * np.sqrt(k) if prec == 1 else 2e-4
    assert err < rel * ref.abs().max().item()
    assert err > 0.0
    if prec == 2:
        # far better than a single bf16 product (2^-8 per operand)
        A16 = A.cpu().to(torch.bfloat16).double()
        B16 = B.cpu().to(torch.bfloat16).double()
        err1 = (torch.einsum(spec, A16, B16) - ref).abs().max().item()
        assert err < 0.05 * err1


@pytest.mark.parametrize("spec,ashape", [("ik,kj->ij", (300, 64)), ("ki,kj->ij", (64, 300)),
                                         ("ik,kj->ij", (257, 100)), ("ik,kj->ij", (33, 45)),
                                         ("ki,kj->ij", (77, 129))])
def test_bf16_pair_packing_is_exact(nm, spec, ashape):
    """Through the bf16-pair path with B = identity every output is hi + lo
    of its input (B's pair is (1, 0)): the packing (fp64 -> fp32 -> hi =
    bf16 round-to-nearest-even, lo = bf16 of the remainder, in the contiguous,
    transposing and padded layouts) equals torch's conversions bit for bit."""
    say(f"[bf16 packing] {spec} {ashape}")
    rng = np.random.default_rng(17)
    A = T(rng.normal(size=ashape) * np.exp(rng.normal(size=ashape)))
    K = ashape[0] if spec.startswith("ki") else ashape[1]
    M = ashape[1] if spec.startswith("ki") else ashape[0]
    I = torch.eye(K, dtype=torch.float64, device="cuda")
    C = torch.zeros((M, K), dtype=torch.float64, device="cuda")
    nm.contract(spec, 1.0, A, I, 0.0, C, precision=2)
    torch.cuda.synchronize()
    a = (A.t() if spec.startswith("ki") else A).cpu().float()
    hi = a.to(torch.bfloat16).float()
    lo = (a - hi).to(torch.bfloat16).float()
    ref = (hi + lo).double()
    assert torch.equal(C.cpu(), ref)


@pytest.mark.parametrize("tile", [-1, 0, 1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("M,N,K", [(1, 1, 32), (130, 257, 64), (1089, 640, 320), (600, 700, 96)])
def test_gemm_bf16_pairs_kernel_surface(nm, M, N, K, tile):
    """nm_gemm_tiled with bfloat16 pairs (the split-precision kernel alone, in
    each workgroup tile shape; ragged edges in M and N, several tiles): the
    result equals the fp64 product of the pairs' values up to the dropped
    lo x lo term and fp32 accumulation, and is far closer to the fp32
    product than one bf16 product is."""
    say(f"[nm_gemm bf16x3] tile={tile} {M}x{N}x{K}")
    rng = np.random.default_rng(M + N + K)
    A = torch.as_tensor(rng.normal(size=(M, K)), dtype=torch.float32, device="cuda")
    Bt = torch.as_tensor(rng.normal(size=(N, K)), dtype=torch.float32, device="cuda")
    def pair(x):
        hi = x.to(torch.bfloat16)
        lo = (x - hi.float()).to(torch.bfloat16)
        return nm.pair_interleave(hi, lo).contiguous(), hi, lo
    Ap, ah, al = pair(A)
    Bp, bh, bl = pair(Bt)
    C0 = torch.as_tensor(rng.normal(size=(M, N)), device="cuda")
    C = C0.clone()
    nm.gemm(2, Ap, Bp, C, alpha=0.5, beta=-2.0, tile=tile)
    torch.cuda.synchronize()
    a64 = ah.double().cpu(), al.double().cpu()
    b64 = bh.double().cpu(), bl.double().cpu()
    three = a64[0] @ b64[0].T + a64[0] @ b64[1].T + a64[1] @ b64[0].T
    ref = 0.5 * three - 2.0 * C0.cpu()
    err = (C.cpu() - ref).abs().max().item()
    assert err < 1e-6 * np.sqrt(K) * max(1.0, ref.abs().max().item())
    exact = 0.5 * (A.double().cpu() @ Bt.double().cpu().T) - 2.0 * C0.cpu()
    one = 0.5 * (a64[0] @ b64[0].T) - 2.0 * C0.cpu()
    e3 = (C.cpu() - exact).abs().max().item()
    e1 = (one - exact).abs().max().item()
    assert e3 < 0.05 * e1


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (130, 257, 19), (1089, 640, 300)])
def test_gemm_kernel_surface(nm, prec, M, N, K):
    """nm_gemm, the single-launch GEMM the bench times: ragged edges in every
    dimension, fp64 operands exact to rounding, fp32 operands to fp32
    rounding of the products."""
    say(f"[nm_gemm] prec={prec} {M}x{N}x{K}")
    rng = np.random.default_rng(M + N + K)
    dt = torch.float64 if prec == 0 else torch.float32
    A = torch.as_tensor(rng.normal(size=(M, K)), device="cuda").to(dt)
    B = torch.as_tensor(rng.normal(size=(K, N)), device="cuda").to(dt)
    C0 = torch.as_tensor(rng.normal(size=(M, N)), device="cuda")
    C = C0.clone()
    nm.gemm(prec, A, B, C, alpha=0.5, beta=-2.0)
    torch.cuda.synchronize()
    ref = 0.5 * (A.double().cpu() @ B.double().cpu()) - 2.0 * C0.cpu()
    err = (C.cpu() - ref).abs().max().item()
    tol = (1e-13 if prec == 0 else 1e-6) * np.sqrt(K) * max(1.0, ref.abs().max().item())
    assert err < tol


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("o,v,naux,seed", [(2, 4, 18, None), (4, 12, 48, 2301)])
def test_mixed_precision_pipeline_matches_oracle(nm, o, v, naux, seed, prec):
    """CC_FP32_REFINE / CC_BF16X3_REFINE with every unbatched contraction
    forced onto low-precision operands: the refined energies, states and
    couplings meet the fp64 tolerances against the oracle."""
    say(f"[mixed pipeline] prec={prec} o={o} v={v}")
    seed = synth.exact_check_seed(o, v) if seed is None else seed
    nroots = 2
    st = oracle_state(o, v, naux, seed, nroots)
    sysd = st["sys"]
    dirs = synth.make_directions(o + v, naux, seed + 17, 2)
    opts = nm.default_opts(precision=prec, mixed_min_flops=0.0)
    ctx = nm.Context(o, v, naux, T(sysd["eps"]), T(sysd["B"]), opts)
    e, _, rc = ctx.ground()
    assert rc == 0
    e_hf_ref = float(ccsd.energy(torch.zeros(o, v, dtype=torch.float64),
                                 torch.zeros(o, o, v, v, dtype=torch.float64), st["h"], st["g"]))
    assert abs((e + e_hf_ref) - st["E0"]) < 1e-9
    w, _, rc = ctx.eom(nm.CC_BOTH, nroots)
    assert rc == 0
    assert np.abs(np.array(w) - st["omega"].numpy()).max() < 1e-9
    _, rc = ctx.multipliers([(1, 2), (2, 1)])
    assert rc == 0
    for (i, j) in [(0, 1), (1, 0)]:
        m = rs.multipliers(st, i, j, relaxed=True)
        ctx.densities(i + 1, j + 1)
        F = ctx.nacme(i + 1, j + 1, T(dirs["dh"]), T(dirs["dB"]))
        for q in range(2):
            dg = np.einsum("Ppq,Prs->pqrs", dirs["dB"][q], dirs["dB"][q])
            Fo = rs.coupling_direct(st, m, j, dirs["dh"][q], dg)
            assert abs(F[q] - Fo) < 1e-7 * max(1.0, abs(Fo))
    ctx.close()


@pytest.mark.parametrize("o,v", [(2, 3), (3, 5), (4, 12)])
def test_block_transforms_match_single(nm, o, v):
    """Batched right/left transforms of k vectors equal k single transforms
    (fp64), and the fp32-operand variant stays within fp32 rounding; the
    singles and doubles parts are checked against the oracle."""
    say(f"[block jacobian] o={o} v={v}")
    naux = 3 * (o + v)
    st = oracle_state(o, v, naux, synth.exact_check_seed(o, v), 2)
    sysd = st["sys"]
    # every contraction qualifies for fp32 operands in the precision=1 calls
    ctx = nm.Context(o, v, naux, T(sysd["eps"]), T(sysd["B"]), nm.default_opts(mixed_min_flops=0.0))
    ctx.ground()
    k = 3
    Nf = o * v + (o * v) ** 2
    rng = np.random.default_rng(11)
    xs = [rng.normal(size=st["x"].numel()) for _ in range(k)]
    X = torch.stack([T(to_full(x, o, v)) for x in xs])
    for side, fn in [(nm.CC_RIGHT, rs.right_transform), (nm.CC_LEFT, rs.left_transform)]:
        Y = torch.zeros_like(X)
        ctx.apply_jacobian_block(side, X, Y)
        y1 = torch.zeros(Nf, dtype=torch.float64, device="cuda")
        for z in range(k):
            ctx.apply_jacobian(side, X[z].contiguous(), y1)
            torch.cuda.synchronize()
            ref = y1.cpu().numpy()
            got = Y[z].cpu().numpy()
            assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
            orc = fn(st["x"], torch.as_tensor(xs[z]), st["h"], st["g"], o, v).numpy()
            assert np.abs(to_packed(got, o, v) - orc).max() < 1e-9
        scale = Y.abs().max().item()
        for prec, tol in [(1, 1e-5), (2, 1e-3)]:
            Ylp = torch.zeros_like(X)
            ctx.apply_jacobian_block(side, X, Ylp, precision=prec)
            torch.cuda.synchronize()
            d = (Ylp - Y).abs().max().item()
            assert d < tol * max(1.0, scale)
            assert d > 0.0   # the low-precision contractions really ran
    ctx.close()
