#!/usr/bin/env python3
"""Time-to-NACME and Jacobian-transform throughput on one MI355X.

A step is one pass of the whole path at the thymine/cc-pVDZ-shaped synthetic
workload (o = 33, v = 127, naux = 640, two excited states, 45 perturbation
directions), starting from device-resident inputs (orbital energies, DF
factor, derivative integrals):

  cc_create (integral build) -> cc_ground -> eom_solve(both sides)
  -> multipliers, densities, nacme for the ordered pairs (1,2) and (2,1).

The timed steps run the mixed-precision path (default: the eigen- and linear
solvers' contractions as bfloat16 pairs with three bf16 matrix-core products,
the ground state with fp32 operands; fp64 images of the current solutions and
fp64 residuals decide convergence; --precision mixed uses fp32 operands
throughout); one step of the plain fp64 path runs beside it for the speed-up
and the coupling agreement.  The run also measures the Jacobian transforms
per second, the ladder GEMM's roofline fraction in every precision (HIP
events on the stream the kernel runs on) and a CPU baseline (the fp64
oracle's residual at the same size on the host cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense matrix cores): FP64 78.6 TFLOP/s, FP32
# 157.3 TFLOP/s; HBM 8 TB/s.
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
# the benchmark's workload (thymine/cc-pVDZ-shaped) and the aug-cc-pVDZ-shaped
# one (o = 33, v = 250, naux = 1100, four roots in one block Davidson; its
# subspaces are capped at 48 vectors of 0.55 GB)
WORKLOADS = {
    "thymine_dz": dict(name="thymine_dz", o=33, v=127, naux=640, nroots=2, ndir=45, seed=4301),
    "thymine_adz": dict(name="thymine_adz", o=33, v=250, naux=1100, nroots=4, ndir=45, seed=6301,
                        davidson_max=48),
}
WORKLOAD = WORKLOADS["thymine_dz"]
# the ordered pairs of excited states whose couplings one step produces
PAIRS = [(1, 2), (2, 1)]
# the metric's accuracy bound on every coupling component (au)
F_TOL = 1e-6
# DF factor scale: the recipe's N(0, 0.05) gives no convergent CCSD at this
# size (ground-state iterations overflow from the MP2 start); the scale is
# reduced so that naux * sigma^2 * v keeps its value at o = 4, v = 12, naux = 48.
def sigma_b(cfg):
    return 0.05 * (48 * 12 / (cfg["naux"] * cfg["v"])) ** 0.5


SIGMA_B = sigma_b(WORKLOAD)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_step(nm, torch, inp, cfg, opts, start=None):
    """One pass of the path; every library call ends with a stream sync, so the
    host clock between calls gives the per-stage split.  start(ctx), when
    given, sets the amplitude solver's starting point (timed as "guess")."""
    st = {}
    t = time.perf_counter()

    def lap(name):
        nonlocal t
        now = time.perf_counter()
        st[name] = st.get(name, 0.0) + (now - t)
        t = now

    def need(rc, what):
        # a coupling from unconverged solutions is not a valid measurement
        if rc != nm.CC_OK:
            raise RuntimeError(f"{what} returned {rc} (not converged); the step is invalid")

    ctx = nm.Context(cfg["o"], cfg["v"], cfg["naux"], inp["eps"], inp["B"], opts)
    lap("integrals")
    if start is not None:
        start(ctx)
        lap("guess")
    e, it, rc = ctx.ground()
    need(rc, "cc_ground")
    lap("ground")
    w, itw, rc = ctx.eom(nm.CC_BOTH, cfg["nroots"])
    need(rc, "eom_solve")
    lap("eom")
    F = {}
    _, rc = ctx.multipliers(PAIRS)
    need(rc, "multipliers")
    lap("multipliers")
    for (i, j) in PAIRS:
        ctx.densities(i, j)
        lap("densities")
        F[(i, j)] = ctx.nacme(i, j, inp["dh"], inp["dB"])
        lap("nacme")
    torch.cuda.synchronize()
    return ctx, dict(e_corr=e, omega=w, ground_iters=it, eom_iters=itw, F=F, stage_s=st)


# HBM traffic of one ladder GEMM launch for a block of LADDER_VECTORS trial
# vectors (M = 2 o^2 = 2178, N = K = v^2 = 16129), from rocprofv3 --pmc
# FETCH_SIZE / WRITE_SIZE of `bench.py --roofline-only`
# (profiles/ladder_gemm_thymine_dz_traffic.md), each counter scaled by the
# ratio of a 1 GiB device copy's known bytes to what the counter reads for it.
# Set to None whenever the GEMM kernels change, until the counters are re-taken.
LADDER_TRAFFIC_BYTES = {"fp64": 3.952e+10, "fp32": 1.89e+10}
# the same for each workgroup tile of the bfloat16-pair kernel
LADDER_TRAFFIC_BYTES_BF16 = {0: 2.008e+10, 1: 4.852e+09, 2: 7.274e+09, 3: 7.389e+09, 4: 7.262e+09,
                             5: 7.351e+09, 6: 7.662e+09, 7: 7.432e+09}
# trial vectors per ladder launch: the block the EOM solver pushes through each
# Jacobian transform (the wanted roots)
LADDER_VECTORS = 2
# workgroup tiles of the bfloat16-pair kernel (nm_gemm_tiled)
BF16_TILES = {0: "128x128", 1: "256x256", 2: "256x128", 3: "128x256",
              4: "256x128 (loads 2 steps ahead)", 5: "128x256 (loads 2 steps ahead)",
              6: "256x128 (fragments 1 step ahead)", 7: "128x256 (fragments 1 step ahead)"}

# timed-step precision: library mode, dtype label, dominant ladder kernel
PRECISIONS = {
    "mixed": ("CC_FP32_REFINE", "f32+f64", "fp32"),
    "bf16x3": ("CC_BF16X3_REFINE", "bf16x3+f32+f64", "bf16x3"),
    "fp64": ("CC_FP64", "f64", "fp64"),
}


def ladder_roofline(nm, torch, cfg, dev, st, nl=10):
    """Ladder GEMM roofline: Y[z ij][ab] = sum_cd X[z ij][cd] W[cd][ab] for a
    block of LADDER_VECTORS trial vectors z, one launch of the matrix-core GEMM
    (M = LADDER_VECTORS o^2, N = K = v^2; 2 o^2 v^4 flop per vector) per operand
    precision, timed with HIP events on the stream the kernel is launched on."""
    o, v = cfg["o"], cfg["v"]
    rows = LADDER_VECTORS * o * o
    ladder_flop = 2.0 * rows * v ** 4
    roof = {}
    for pname, pcode, dt, peak in [("fp64", 0, torch.float64, PEAK_FP64_TFLOPS),
                                   ("fp32", 1, torch.float32, PEAK_FP32_TFLOPS)]:
        A = torch.randn(rows, v * v, dtype=dt, device=dev)
        Bv = torch.randn(v * v, v * v, dtype=dt, device=dev)
        C = torch.zeros(rows, v * v, dtype=torch.float64, device=dev)
        nm.gemm(pcode, A, Bv, C, stream=st)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(st)
        for _ in range(nl):
            nm.gemm(pcode, A, Bv, C, stream=st)
        ev1.record(st)
        ev1.synchronize()
        lms = ev0.elapsed_time(ev1) / nl
        tf = ladder_flop / (lms * 1e-3) / 1e12
        roof[pname] = dict(bound="mfma", achieved=tf, peak=peak, unit="TFLOP/s", frac=tf / peak,
                           traffic=(LADDER_TRAFFIC_BYTES[pname] if cfg["name"] == "thymine_dz" else None),
                           launch_ms=lms,
                           flop_per_launch=ladder_flop,
                           algorithmic_bytes=(A.numel() + Bv.numel()) * A.element_size()
                           + 8 * C.numel())
        del A, Bv, C
    # bfloat16 pairs: three bf16 products per product, K padded to a multiple
    # of 32; achieved counts the bf16 matrix-core flops (3 x the ladder's)
    Kp = (v * v + 31) // 32 * 32
    A = torch.randn(rows, 2 * Kp, device=dev).to(torch.bfloat16)
    Bt = torch.randn(v * v, 2 * Kp, device=dev).to(torch.bfloat16)
    C = torch.zeros(rows, v * v, dtype=torch.float64, device=dev)
    # every workgroup tile shape of the kernel; the fastest is the one the
    # contraction engine's autotuner keeps for this shape
    tile_ms = {}
    for tile in BF16_TILES:
        nm.gemm(2, A, Bt, C, stream=st, tile=tile)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(st)
        for _ in range(nl):
            nm.gemm(2, A, Bt, C, stream=st, tile=tile)
        ev1.record(st)
        ev1.synchronize()
        tile_ms[BF16_TILES[tile]] = ev0.elapsed_time(ev1) / nl
    best_tile = min(tile_ms, key=tile_ms.get)
    best_code = [t for t, name in BF16_TILES.items() if name == best_tile][0]
    lms = tile_ms[best_tile]
    # achieved: the method's flops (2 o^2 v^4 per vector); the three bf16
    # products each such flop issues are reported beside it
    tf = ladder_flop / (lms * 1e-3) / 1e12
    roof["bf16x3"] = dict(bound="mfma", achieved=tf, peak=PEAK_BF16_TFLOPS, unit="TFLOP/s",
                          frac=tf / PEAK_BF16_TFLOPS,
                          traffic=(LADDER_TRAFFIC_BYTES_BF16.get(best_code) if cfg["name"] == "thymine_dz"
                                   else None),
                          launch_ms=lms, flop_per_launch=ladder_flop, products_per_flop=3,
                          issued_tflops=3.0 * tf, issued_frac=3.0 * tf / PEAK_BF16_TFLOPS,
                          tile=best_tile, tile_launch_ms=tile_ms,
                          algorithmic_bytes=(A.numel() + Bt.numel()) * 2 + 8 * C.numel())
    del A, Bt, C
    roof["bf16x3"]["kernel"] = (f"{'gemm_bf16x3_kernel' if best_tile == '128x128' else 'gemm_bf16x3_big_kernel'} "
                                f"{best_tile} (ladder X[z ij][cd] x W[cd][ab], "
                                f"{LADDER_VECTORS} trial vectors, bfloat16 pairs, 3 bf16 products, "
                                "fp32 accumulation)")
    roof["fp64"]["kernel"] = (f"gemm_f64_big_kernel (ladder X[z ij][cd] x W[cd][ab], "
                              f"{LADDER_VECTORS} trial vectors, fp64 operands)")
    roof["fp32"]["kernel"] = (f"gemm_f32acc_big_kernel (ladder X[z ij][cd] x W[cd][ab], "
                              f"{LADDER_VECTORS} trial vectors, fp32 operands, fp32 accumulation)")
    return roof


def learned_guess(nm, torch, np, synth, cfg, dev, prec, n_train=48, n_eval=16, steps=3000,
                  batch=8192, lr=2e-3, tol=1e-8, n_full=2):
    """The learned-guess workload: perturbed geometries of the thymine-shaped
    system (orbital rotation exp(K), K_pq ~ N(0, 0.01^2), seeds 900 + k), a
    network trained on the converged doubles of n_train of them by the
    library's own kernels, and the amplitude solver on the n_eval others
    started from MP2 (the default) and from the network, at tolerance tol.
    Every answer is judged by the same residual tolerance.  On the first
    n_full held-out geometries the whole path to the couplings (pairs (1, 2)
    and (2, 1), 45 directions) runs from each start as well (twice each, the
    faster run reported)."""
    T = lambda x: torch.as_tensor(np.ascontiguousarray(x), device=dev)  # noqa: E731
    base = synth.make_system(cfg["o"], cfg["v"], cfg["naux"], cfg["seed"], sigma_b=sigma_b(cfg))
    eps = T(base["eps"])
    opts = nm.default_opts(precision=prec, tol_ground=tol)
    n4 = (cfg["o"] * cfg["v"]) ** 2
    F = torch.empty((n_train * n4, 8), dtype=torch.float32, device=dev)
    Z = torch.empty((n_train * n4,), dtype=torch.float32, device=dev)
    c0 = time.perf_counter()
    for k in range(n_train):
        ctx = nm.Context(cfg["o"], cfg["v"], cfg["naux"], eps, T(synth.perturbed_factor(base["B"], 900 + k)),
                         opts)
        _, _, rc = ctx.ground()
        if rc != 0:
            raise RuntimeError(f"training geometry {k}: ground state not converged")
        ctx.t2_features(F[k * n4:(k + 1) * n4])
        ctx.t2_target(Z[k * n4:(k + 1) * n4])
        ctx.close()
        log(f"[learned] training geometry {k + 1}/{n_train}")
    torch.cuda.synchronize()
    c1 = time.perf_counter()
    mu = F.mean(dim=0)
    sd = F.std(dim=0) + 1e-12
    F.sub_(mu).div_(sd)
    zs = float(Z.std())
    Z.div_(zs)
    net = nm.MLP(8, 256, 1, seed=4)
    loss = net.train(F, Z[:, None], batch=batch, steps=steps, lr=lr, seed=5)
    torch.cuda.synchronize()
    c2 = time.perf_counter()
    log(f"[learned] trained: loss {loss:.3e} in {c2 - c1:.1f} s")
    del F, Z
    mu_h, sd_h = mu.cpu().numpy(), sd.cpu().numpy()
    rows, guess_s = [], []
    for k in range(n_eval):
        Bk = T(synth.perturbed_factor(base["B"], 900 + n_train + k))
        res = {}
        for mode in ("mp2", "learned"):
            ctx = nm.Context(cfg["o"], cfg["v"], cfg["naux"], eps, Bk, opts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "learned":
                ctx.guess_t2(net, mu_h, sd_h, zs)
                torch.cuda.synchronize()
                guess_s.append(time.perf_counter() - t0)
            e, it, rc = ctx.ground()
            torch.cuda.synchronize()
            res[mode] = (e, it, rc, time.perf_counter() - t0)
            ctx.close()
        rows.append(res)
        log(f"[learned] held-out geometry {k + 1}/{n_eval}: iterations MP2 {res['mp2'][1]}, "
            f"learned {res['learned'][1]}")
    # the whole path to the couplings from each start
    full = []
    if n_full > 0:
        n = cfg["o"] + cfg["v"]
        inp = dict(eps=eps, dh=torch.empty((cfg["ndir"], n, n), dtype=torch.float64, device=dev),
                   dB=torch.empty((cfg["ndir"], cfg["naux"], n, n), dtype=torch.float64, device=dev))
        for q in range(cfg["ndir"]):
            d = synth.make_direction(n, cfg["naux"], cfg["seed"], q, sigma_b=sigma_b(cfg))
            inp["dh"][q].copy_(T(d["dh"]))
            inp["dB"][q].copy_(T(d["dB"]))
        popts = nm.default_opts(precision=prec)
        # one untimed pass first: the GEMM autotuner's first-use timings of
        # the solvers' shapes stay out of both starts' times
        inp["B"] = T(base["B"])
        ctx, _ = run_step(nm, torch, inp, cfg, popts)
        ctx.close()
        for k in range(min(n_full, n_eval)):
            inp["B"] = T(synth.perturbed_factor(base["B"], 900 + n_train + k))
            res = {}
            for mode in ("mp2", "learned"):
                start = (lambda c: c.guess_t2(net, mu_h, sd_h, zs)) if mode == "learned" else None
                # each start timed twice, the faster run kept: a GEMM shape
                # the solvers meet for the first time in this process (say a
                # block of one vector once a root has converged) puts the
                # autotuner's first-use timings into one run only
                for _ in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ctx, out = run_step(nm, torch, inp, cfg, popts, start=start)
                    rec = dict(time_to_nacme_s=time.perf_counter() - t0, stage_s=out["stage_s"],
                               ground_iters=out["ground_iters"], eom_iters=out["eom_iters"], F=out["F"])
                    ctx.close()
                    if mode not in res or rec["time_to_nacme_s"] < res[mode]["time_to_nacme_s"]:
                        res[mode] = rec
            dF = max(float(np.abs(np.asarray(res["mp2"]["F"][p]) - np.asarray(res["learned"]["F"][p])).max())
                     for p in PAIRS)
            for r in res.values():
                del r["F"]
            full.append(dict(geometry=n_train + k, max_abs_dF=dF, **res))
            log(f"[learned] full path, held-out geometry {k + 1}: MP2 {res['mp2']['time_to_nacme_s']:.3f} s, "
                f"learned {res['learned']['time_to_nacme_s']:.3f} s, max |dF| {dF:.1e}")
    net.close()
    it0 = [r["mp2"][1] for r in rows]
    it1 = [r["learned"][1] for r in rows]
    print(json.dumps(dict(
        mode="learned-guess", workload="thymine_dz perturbed geometries (orbital rotations N(0, 0.01^2))",
        n_train=n_train, n_eval=n_eval, tolerance=tol, training_s=c2 - c1, data_s=c1 - c0,
        training_loss=loss, target_variance=1.0,
        iterations_mp2=it0, iterations_learned=it1,
        mean_iterations_mp2=float(np.mean(it0)), mean_iterations_learned=float(np.mean(it1)),
        mean_time_mp2_s=float(np.mean([r["mp2"][3] for r in rows])),
        mean_time_learned_s=float(np.mean([r["learned"][3] for r in rows])),
        mean_guess_s=float(np.mean(guess_s)),
        full_path=full,
        all_converged=all(r["mp2"][2] == 0 and r["learned"][2] == 0 for r in rows),
        max_abs_d_energy=float(max(abs(r["mp2"][0] - r["learned"][0]) for r in rows)))), flush=True)


def network_only(nm, torch, cfg, dev, nl=10):
    """The learned guess's network (8 -> 256 -> 256 -> 1, bfloat16 working
    weights) on one feature row per doubles index of the workload (o^2 v^2
    rows, standard normal features): average launch time of mlp_forward's
    fused kernel with HIP events, rows per second and the bf16 products it
    issues (two per hidden product: inputs and activations as bf16 pairs;
    layer 1's K padded to 32)."""
    n = (cfg["o"] * cfg["v"]) ** 2
    g = torch.Generator(device=dev).manual_seed(5)
    X = torch.randn((n, 8), dtype=torch.float32, device=dev, generator=g)
    Y = torch.empty((n, 1), dtype=torch.float32, device=dev)
    net = nm.MLP(8, 256, 1, seed=4)
    net.forward(X, Y)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(nl):
        net.forward(X, Y)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / nl
    issued = 2.0 * 2.0 * n * (32 * 256 + 256 * 256)
    net.close()
    print(json.dumps(dict(mode="network-only", rows=n, launch_ms=ms, rows_per_s=n / ms * 1e3,
                          issued_bf16_tflops=issued / ms / 1e9,
                          issued_frac=issued / ms / 1e9 / PEAK_BF16_TFLOPS,
                          silu_per_row=512, hbm_bytes_per_row=36)), flush=True)


def roofline_only(nm, torch, cfg, dev):
    """The ladder launches alone, plus a 1 GiB device copy that calibrates the
    HBM byte counters (for rocprofv3 --pmc runs)."""
    st = torch.cuda.current_stream()
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    roof = ladder_roofline(nm, torch, cfg, dev, st, nl=3)
    print(json.dumps(dict(mode="roofline-only", copy_bytes=src.numel() * 8, ladder=roof)),
          flush=True)


def cpu_info():
    """Host CPU model, thread count and BLAS of the oracle (torch's CPU build)."""
    import torch
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cfg = torch.__config__.show()
    blas = "mkl" if "BLAS_INFO=mkl" in cfg else ("openblas" if "openblas" in cfg.lower() else "unknown")
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "MKL_NUM_THREADS",
                                          "OPENBLAS_NUM_THREADS", "GOMP_CPU_AFFINITY")}
    return dict(cpu_model=model, blas=f"torch {torch.__version__} CPU ({blas})",
                thread_env={k: v for k, v in env.items() if v is not None})


def cpu_baseline(sysd, cfg, counts):
    """The oracle timed on the host cores at the same workload: one CCSD
    residual, one right and one left Jacobian transform (at random amplitudes
    and trial vectors of the ground-state size), each scaled by how many of
    them one GPU step runs."""
    import numpy as np
    import torch

    import synth
    from oracle import ccsd as occ
    from oracle import response as ors

    o, v = cfg["o"], cfg["v"]
    threads = len(os.sched_getaffinity(0))
    torch.set_num_threads(threads)
    h, g = ors.system_hamiltonian(sysd["eps"], sysd["B"], o)
    t1o, t2o = (torch.as_tensor(x) for x in synth.random_amplitudes(o, v, seed=1, scale=0.01))
    x = occ.pack(t1o, t2o)
    r = torch.as_tensor(np.random.default_rng(2).normal(scale=1e-2, size=x.numel()))
    c0 = time.perf_counter()
    occ.residual(t1o, t2o, h, g)
    c1 = time.perf_counter()
    ors.right_transform(x, r, h, g, o, v)
    c2 = time.perf_counter()
    ors.left_transform(x, r, h, g, o, v)
    c3 = time.perf_counter()
    del h, g
    t_res, t_right, t_left = c1 - c0, c2 - c1, c3 - c2
    step_s = (counts["residuals"] * t_res + counts["right"] * t_right
              + counts["left"] * t_left)
    out = dict(value=len(PAIRS) / step_s, unit="NACME vectors/s", cores=threads, kind="oracle",
               sample=(f"oracle at o={o} v={v} naux={cfg['naux']}: one CCSD residual "
                       f"{t_res:.2f} s, one right transform {t_right:.2f} s, one left "
                       f"transform {t_left:.2f} s; scaled by the {int(counts['residuals'])} "
                       f"residuals, {int(counts['right'])} right and {int(counts['left'])} left "
                       "transforms of one GPU step (densities and contraction not counted)"),
               residual_s=t_res, right_transform_s=t_right, left_transform_s=t_left,
               step_s_estimate=step_s)
    out.update(cpu_info())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--transforms", type=int, default=3)
    ap.add_argument("--precision", choices=list(PRECISIONS), default="bf16x3",
                    help="precision of the timed steps")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the step in the other precision")
    ap.add_argument("--step-only", action="store_true",
                    help="only the warmup and timed steps (for kernel profiles of a step)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the ladder GEMM launches and a copy calibration (profiling)")
    ap.add_argument("--workload", choices=list(WORKLOADS), default="thymine_dz",
                    help="thymine_dz (default, the benchmark) or thymine_adz (v = 250, 4 roots)")
    ap.add_argument("--network-only", action="store_true",
                    help="only the learned guess's network on one row per doubles index "
                         "(fused inference kernel timing, for profiling)")
    ap.add_argument("--learned-guess", action="store_true",
                    help="only the learned-guess workload: 48 training and 16 held-out "
                         "perturbed geometries, ground-state iterations from MP2 vs the network")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for {args.gpus}); sharding a "
              "step across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2301_13264_amd as nm

    cfg = WORKLOADS[args.workload]
    sb = sigma_b(cfg)
    dev = torch.device("cuda:0")
    if args.roofline_only:
        roofline_only(nm, torch, cfg, dev)
        return
    if args.network_only:
        network_only(nm, torch, cfg, dev)
        return
    if args.learned_guess:
        learned_guess(nm, torch, np, synth, cfg, dev, getattr(nm, PRECISIONS[args.precision][0]))
        return
    sysd = synth.make_system(cfg["o"], cfg["v"], cfg["naux"], cfg["seed"], sigma_b=sb)
    T = lambda x: torch.as_tensor(np.ascontiguousarray(x), device=dev)  # noqa: E731
    inp = dict(eps=T(sysd["eps"]), B=T(sysd["B"]))
    # directions one at a time (the same values as synth.make_directions),
    # straight into device memory
    n = cfg["o"] + cfg["v"]
    inp["dh"] = torch.empty((cfg["ndir"], n, n), dtype=torch.float64, device=dev)
    inp["dB"] = torch.empty((cfg["ndir"], cfg["naux"], n, n), dtype=torch.float64, device=dev)
    for q in range(cfg["ndir"]):
        d = synth.make_direction(n, cfg["naux"], cfg["seed"], q, sigma_b=sb)
        inp["dh"][q].copy_(T(d["dh"]))
        inp["dB"][q].copy_(T(d["dB"]))
    torch.cuda.synchronize()
    prec = getattr(nm, PRECISIONS[args.precision][0])
    extra = {"davidson_max": cfg["davidson_max"]} if "davidson_max" in cfg else {}
    opts = nm.default_opts(precision=prec, **extra)

    for w in range(args.warmup):
        log(f"[bench] warmup step {w + 1}/{args.warmup} ({args.precision})")
        ctx, _ = run_step(nm, torch, inp, cfg, opts)
        ctx.close()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} step(s) ({args.precision})")
    t0 = time.perf_counter()
    ctx = None
    for s in range(args.steps):
        if ctx is not None:
            ctx.close()
        ctx, out = run_step(nm, torch, inp, cfg, opts)
        log(f"[bench] step {s + 1} done: omega={out['omega']} F12[0]={out['F'][PAIRS[0]][0]:.6e} "
            f"stages={ {k: round(x, 2) for k, x in out['stage_s'].items()} }")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = 1000.0 * (t1 - t0) / args.steps
    stats = ctx.stats()
    counts = dict(residuals=stats["residuals"], right=stats["right_transforms"],
                  left=stats["left_transforms"])
    value = len(PAIRS) * 1000.0 / ms   # NACME vectors (45 components each) per second
    if args.step_only:
        ctx.close()
        print(json.dumps(dict(mode="step-only", ms_per_step=ms, value=value, stage_s=out["stage_s"],
                              step_counts=counts, omega=out["omega"])), flush=True)
        return

    # Jacobian transforms/s at the converged amplitudes (HIP events on the
    # library's stream): k vectors per batched call, fp64 and fp32 operands;
    # the marginal cost per vector excludes the per-call linearisation.
    N = cfg["o"] * cfg["v"] + (cfg["o"] * cfg["v"]) ** 2
    st = torch.cuda.current_stream()
    tr = {}
    for pname, pcode in ([] if args.transforms <= 0 else
                         [("fp64", nm.CC_FP64), ("fp32", nm.CC_FP32_REFINE),
                          ("bf16x3", nm.CC_BF16X3_REFINE)]):
        for side, sname in [(nm.CC_RIGHT, "right"), (nm.CC_LEFT, "left")]:
            per_call = {}
            for k in (1, 4):
                X = torch.randn(k, N, dtype=torch.float64, device=dev) * 1e-2
                Y = torch.zeros_like(X)
                ctx.apply_jacobian_block(side, X, Y, precision=pcode)
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record(st)
                for _ in range(args.transforms):
                    ctx.apply_jacobian_block(side, X, Y, precision=pcode)
                ev1.record(st)
                ev1.synchronize()
                per_call[k] = ev0.elapsed_time(ev1) / args.transforms
                del X, Y
            tr[f"{sname}_{pname}"] = dict(ms_per_call_k1=per_call[1], ms_per_call_k4=per_call[4],
                                          ms_per_vector_k4=(per_call[4] - per_call[1]) / 3.0)
    ctx.close()

    other = None
    valid = True
    if not args.no_compare:
        oname = "fp64" if args.precision != "fp64" else "mixed"
        oprec = nm.CC_FP64 if args.precision != "fp64" else nm.CC_FP32_REFINE
        log(f"[bench] one step in {oname} for comparison")
        c0 = time.perf_counter()
        octx, oout = run_step(nm, torch, inp, cfg, nm.default_opts(precision=oprec, **extra))
        c1 = time.perf_counter()
        octx.close()
        dF = max(float(np.max(np.abs(np.asarray(out["F"][k]) - np.asarray(oout["F"][k]))))
                 for k in out["F"])
        dw = max(abs(a - b) for a, b in zip(out["omega"], oout["omega"]))
        # the mixed path must meet the metric's bound against the fp64 path
        valid = dF <= F_TOL
        other = dict(precision=oname, time_to_nacme_s=c1 - c0, stage_s=oout["stage_s"],
                     max_abs_dF=dF, max_abs_domega=dw, within_bound=valid, bound=F_TOL,
                     d_e_corr=abs(out["e_corr"] - oout["e_corr"]),
                     ground_iters=oout["ground_iters"], eom_iters=oout["eom_iters"])
        log(f"[bench] {oname}: {c1 - c0:.2f} s, max|dF| = {dF:.3e} "
            f"stages={ {k: round(x, 2) for k, x in oout['stage_s'].items()} }")

    roof = ladder_roofline(nm, torch, cfg, dev, st)
    main_roof = roof[PRECISIONS[args.precision][2]]

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline: oracle residual and transforms on the host")
        cpu = cpu_baseline(sysd, cfg, counts)

    res = dict(
        metric="time-to-NACME vector & Jacobian transforms/s (TFLOP/s, % MFMA peak) at <=1e-6 au",
        value=value, unit="NACME vectors/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=ms, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=PRECISIONS[args.precision][1],
        data="synthetic",
        config=dict(workload=(f"{cfg['name']}: o={cfg['o']} v={cfg['v']} naux={cfg['naux']}, "
                              f"{cfg['nroots']} roots "
                              f"(pair gap {out['omega'][1] - out['omega'][0]:.4f} Ha), "
                              f"{cfg['ndir']} directions, DF scale {sb:.5f}"),
                    global_batch=1, parallelism="none"),
        valid=valid,
        precision=args.precision,
        time_to_nacme_s=ms / 1000.0,
        compare=other,
        speedup_vs_fp64=(other["time_to_nacme_s"] / (ms / 1000.0)
                         if other and args.precision != "fp64" else None),
        stage_s=out["stage_s"],
        omega=out["omega"], e_corr=out["e_corr"],
        jacobian_transforms_per_s=({k: 1000.0 / x["ms_per_vector_k4"] for k, x in tr.items()}
                                   if tr else None),
        jacobian_transform_ms=tr,
        step_counts=counts,
        step_gemm_tflops=stats["gemm_flops"] / (ms / 1000.0) / 1e12,
        device_work_area_gb=stats["peak_bytes"] / 1e9,
        roofline=main_roof,
        ladder_roofline=roof,
        lowp_gemm_flops=stats.get("lowp_flops"),
        cpu_baseline=cpu,
    )
    print(json.dumps(res), flush=True)
    if not valid:
        log(f"[bench] INVALID: max |dF| = {other['max_abs_dF']:.3e} exceeds {F_TOL:g} au")
        sys.exit(3)


if __name__ == "__main__":
    main()
