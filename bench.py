#!/usr/bin/env python3
"""Benchmark of the GPU hot path of the matrix-pencil Prony method on one MI355X.

One step is one pass of the GPU steps of Algorithm 1 over the resident inputs
of one problem (default workload c1: d=2, n=63, N=4096, m=20, noise 1e-6):
  samples of the exponential sum on the grid -> T (materialised for the host
  SVD) -> S_1..S_d = U^* T_l V Sigma^{-1} -> Gram matrix and right-hand side
  of the coefficient least-squares problem.
The host steps (SVD, eigendecomposition, m x m solve) run once, untimed, to
produce the inputs U, Sigma, V and z of the timed GPU steps.

value = S-build flops F_S = d (8 N^2 m + 8 N m^2 + 2 m^2) (the paper's dense
work, a complex multiply-add counted as 8) divided by the time of one whole
step, in TFLOP/s; the timed step computes S in FP64 (the paper's arithmetic)
unless --prec says otherwise. The JSON line also carries the S-build alone in
FP64, FP32-MFMA and split bfloat16, the roofline of the dominant kernel of each
precision (its own MFMA work per launch over its launch time, measured with HIP
events around its launches), and the CPU oracle on a bounded sample of the same
workload.

Own work of the tile kernel (row-extended form): the product T_row V over the
(n+2)^d rows k' and N columns h, 8 (n+2)^d N m flops, plus the reductions with the
shifted U_l, 8 ells (n+2)^d m^2 flops (ells = d matrices). It is below F_S by about
the factor d: F_S counts the d products T_l V that the row-extended form shares.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "S_ℓ-build complex TFLOP/s + instances/s, FP32-MFMA vs FP64, at stated rel err"
# MI355X dense MFMA peaks; the split-bfloat16 S-build runs six bf16 products per
# FP32 product, so its FP32-equivalent ceiling is the bf16 peak (2500) / 6
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0 / 6}
DOMINANT = "pencil_tiles"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pencil_tiles_c1_traffic.json")


def s_flops(d, N, m):
    return d * (8.0 * N * N * m + 8.0 * N * m * m + 2.0 * m * m)


def tile_flops(d, n, m, ells=None):
    """Own work of one pencil_tiles launch: Z = T_row V on the (n+2)^d row-extended
    rows, and the ells reductions U_l^* Z (ells = d without S_0)."""
    ells = d if ells is None else ells
    NR, N = (n + 2) ** d, (n + 1) ** d
    return 8.0 * NR * N * m + 8.0 * ells * NR * m * m


def source_digest():
    """Digest of the code (comments and whitespace stripped) of the sources the
    dominant kernel is built from; the stored traffic counters apply while it matches."""
    h = hashlib.sha256()
    for name in ("pencil.hip", "common.h", "mfma.h", "reduce.h"):
        with open(os.path.join(ROOT, "paper_2012_11430_amd", "csrc", name)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", choices=["fp32", "fp64", "bf16x3"], default="fp64",
                    help="S-build precision of the timed step (fp64: the paper's arithmetic; fp32: FP32 MFMA; "
                         "bf16x3: split bfloat16 on the bf16 MFMA)")
    ap.add_argument("--workload", default="c1", choices=["c0", "c1", "c2"])
    ap.add_argument("--cpu-sample-steps", type=int, default=16,
                    help="oracle steps timed for the CPU baseline (0 skips it)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched (c3) and adjoint (c4) measurements")
    ap.add_argument("--no-tune", action="store_true",
                    help="do not run the autotuner; use the tuning cache if one exists")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of MIB MiB (a reference dispatch "
                         "of known traffic for hardware-counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path is a single-GPU kernel pipeline "
              "(multi-GPU sharding is described in the design notes, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2012_11430_amd import _lib, api, autotune, host
    from workload import config_instances, random_orthonormal

    _lib.load()   # fails loudly when the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    inst = config_instances(args.workload, count=1)[0]
    d, n, m, N = inst.d, inst.n, inst.m, inst.N
    level = inst.noise_levels[0]

    def to_dev(x):
        return torch.from_numpy(np.ascontiguousarray(x)).to(dev)

    # ---------------- resident inputs (untimed; host steps run once)
    t_d, c_d = to_dev(inst.t), to_dev(inst.c)
    noise_d = to_dev(inst.noise(level)) if level > 0 else None
    f = api.samples(t_d, c_d, n, noise=noise_d)
    Tbuf = torch.empty((N, N), dtype=torch.complex128, device=dev)
    api.build_T(f, d, n, 0, out=Tbuf)
    T = Tbuf.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(12345))
    blocks = (random_orthonormal(rng, N, 2 * m), random_orthonormal(rng, N, 2 * m))
    U, sig, V, _ = host.reduced_svd(T, m, start_blocks=blocks)
    del T
    Ud, sd, Vd = to_dev(U), to_dev(sig), to_dev(V)
    Sbuf = torch.empty((d, m, m), dtype=torch.complex128, device=dev)
    api.build_S(f, d, n, Ud, sd, Vd, prec="fp64", out=Sbuf)
    z, _ = host.nodes(Sbuf.cpu().numpy(), inst.mu)
    z_d = to_dev(z)

    tuned = {}
    if not args.no_tune:
        for prec in ("fp32", "fp64", "bf16x3"):
            times = autotune.tune_single(dev, d, n, m, prec, reps=20)
            # the registered winner (the finalists' re-timing can overturn the first pass)
            frag, target = autotune.registered_tile(dev, d, n, m, prec, False)
            tuned[prec] = {"fragments": frag, "target_wgs": target, "plans_timed": len(times)}
    else:
        tuned["cache_entries_loaded"] = autotune.load_cache(dev)

    def step(prec):
        api.samples(t_d, c_d, n, noise=noise_d, out=f)
        api.build_T(f, d, n, 0, out=Tbuf)
        api.build_S(f, d, n, Ud, sd, Vd, prec=prec, out=Sbuf)
        api.coeffs(z_d, f, d, n)

    # ---------------- timed region: K whole steps
    for _ in range(args.warmup):
        step(args.prec)
    torch.cuda.synchronize()
    api.profile_enable(dev, DOMINANT)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step(args.prec)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    launches, tiles_ms = api.profile_read(dev)
    api.profile_enable(dev, None)
    tiles_avg_ms = tiles_ms / max(1, launches)

    # ---------------- the S-build alone, both precisions (same inputs): per-call
    # HIP events, median (and mean) over `steps` calls after the warm-up
    def per_call_ms(fn, reps):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs]

    sbuild = {}
    S_out = {}
    for prec in ("fp32", "fp64", "bf16x3"):
        for _ in range(args.warmup):
            api.build_S(f, d, n, Ud, sd, Vd, prec=prec, out=Sbuf)
        api.profile_enable(dev, DOMINANT)
        times = per_call_ms(lambda: api.build_S(f, d, n, Ud, sd, Vd, prec=prec, out=Sbuf), max(20, args.steps))
        nl, tot = api.profile_read(dev)
        api.profile_enable(dev, None)
        med = float(np.median(times))
        sbuild[prec] = {"ms_median": round(med, 5), "ms_mean": round(float(np.mean(times)), 5),
                        "fs_equivalent_tflops": round(s_flops(d, N, m) / (med * 1e-3) / 1e12, 3),
                        "own_work_tflops": round(tile_flops(d, n, m) / (med * 1e-3) / 1e12, 3),
                        "tiles_ms": round(tot / max(1, nl), 5), "tiles_launches": nl, "calls": len(times)}
        S_out[prec] = Sbuf.cpu().numpy().copy()
        # the same build with prepared factors (U, V packed once): tile and finishing launches only
        fac = api.Factors(d, n, Ud, sd, Vd, prec=prec)
        for _ in range(args.warmup):
            fac.build_S(f, out=Sbuf)
        times = per_call_ms(lambda: fac.build_S(f, out=Sbuf), max(20, args.steps))
        torch.cuda.synchronize()
        if not np.array_equal(Sbuf.cpu().numpy(), S_out[prec]):
            raise RuntimeError(f"prepared-factor build differs from build_S ({prec})")
        fac.close()
        pmed = float(np.median(times))
        sbuild[prec]["prepared_factors_ms_median"] = round(pmed, 5)
        sbuild[prec]["prepared_factors_over_tiles"] = round(pmed / sbuild[prec]["tiles_ms"], 3)

    # ---------------- T alone (HBM-write-bound): GB/s against the 8 TB/s peak
    for _ in range(args.warmup):
        api.build_T(f, d, n, 0, out=Tbuf)
    t_times = per_call_ms(lambda: api.build_T(f, d, n, 0, out=Tbuf), max(20, args.steps))
    t_med = float(np.median(t_times))
    build_T = {"ms_median": round(t_med, 5), "bytes": 16 * N * N,
               "GB_per_s": round(16 * N * N / (t_med * 1e-3) / 1e9, 1), "peak_GB_per_s": 8000.0}

    # recovered nodes and coefficients from each precision's S (host FP64 steps:
    # eig of C_mu and the LS solve; the SVD inputs are shared)
    recovered = {}
    for prec, S_p in S_out.items():
        z_p, t_p = host.nodes(S_p, inst.mu)
        gram, rhs = api.coeffs(to_dev(z_p), f, d, n)
        recovered[prec] = (t_p, host.solve_normal_equations(gram.cpu().numpy(), rhs.cpu().numpy()))
    for prec in sbuild:
        # the whole call (pack, tiles, finish) on the kernel's own work
        sbuild[prec]["own_work_frac_of_peak"] = round(sbuild[prec]["own_work_tflops"] / PEAK_TFLOPS[prec], 4)
    sbuild["speedup_fp32_over_fp64"] = round(sbuild["fp64"]["ms_median"] / sbuild["fp32"]["ms_median"], 3)
    sbuild["speedup_bf16x3_over_fp32"] = round(sbuild["fp32"]["ms_median"] / sbuild["bf16x3"]["ms_median"], 3)

    F = s_flops(d, N, m)
    value = F / (ms_step * 1e-3) / 1e12
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    traffic_rec = {}
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            traffic_rec = json.load(fh)

    def roofline_of(prec, avg_ms, nlaunch):
        """Roofline of the tile kernel of one precision: its own MFMA work per launch
        over its average launch time (HIP events); HBM bytes per launch from the stored
        counters of the same code, workload, precision and split target (the partial
        rows written depend on the plan), else null."""
        p = autotune.plan(dev, d, n, m, prec)
        plan_key = f"{p['fragments']}x{p['workgroups']}"
        traffic = None
        if traffic_rec.get("source_digest") == source_digest() and traffic_rec.get("workload") == args.workload:
            traffic = traffic_rec.get("entries", {}).get(prec, {}).get(plan_key, {}).get("hbm_bytes_per_launch")
        achieved = tile_flops(d, n, m) / (avg_ms * 1e-3) / 1e12
        return {
            "bound": "mfma",
            "kernel": "pencil_tiles_split" if prec == "bf16x3" else DOMINANT,
            "precision": prec,
            "achieved": round(achieved, 3),
            "peak": PEAK_TFLOPS[prec],
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS[prec], 4),
            "traffic": traffic,
            "avg_launch_ms": round(avg_ms, 5),
            "launches_timed": nlaunch,
            "flops_per_launch": tile_flops(d, n, m),
            "fs_equivalent_tflops": round(F / (avg_ms * 1e-3) / 1e12, 3),
            "plan": {"fragments_per_wave": p["fragments"], "workgroups": p["workgroups"], "h_per_chunk": p["chunk"]},
        }

    result = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3"}[args.prec],
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: d={d}, n={n}, N={N}, m={m}, additive noise {level:g}*max|c|",
            "step": "samples -> T (N x N, for the host SVD) -> S_1..S_d -> Gram/rhs",
            "s_build_precision": args.prec,
            "seed": list(inst.seed),
        },
        "roofline": roofline_of(args.prec, tiles_avg_ms, launches),
        "rooflines": {p: roofline_of(p, sbuild[p]["tiles_ms"], sbuild[p]["tiles_launches"])
                      for p in ("fp64", "fp32", "bf16x3")},
        "s_build": sbuild,
        "build_T": build_T,
        "tuned_tiles": tuned,
        "wall_s_timed": round(wall, 4),
    }
    if not args.no_extra:
        result["svd_products"] = svd_products(dev, args, f, d, n, m, sig, blocks, per_call_ms)
        result["noise_sweep_c2"] = noise_sweep_c2(dev, args, per_call_ms)
        result["paper_workload"] = paper_workload(dev, args, per_call_ms)
        result["batched"] = batched_c3(dev, args)
        result["adjoint"] = adjoint_c4(dev, args)

    if args.cpu_sample_steps > 0:
        result["cpu_baseline"] = cpu_baseline(inst, U, sig, V, z, S_out, args.cpu_sample_steps, recovered,
                                              f.cpu().numpy())
    print(json.dumps(result), flush=True)


def svd_products(dev, args, f, d, n, m, sig_ref, blocks, per_call_ms):
    """Algorithm 3's block products Y = T X and T^* X on the GPU without forming T
    (r = 2m columns), and one whole block power SVD driven by them (host QRs)."""
    import numpy as np
    import torch

    from paper_2012_11430_amd import api, host

    N = (n + 1) ** d
    r = 2 * m
    X = torch.randn(N, r, dtype=torch.complex128, device=dev)
    out = {"r": r, "flops_per_product": 8.0 * N * N * r}
    for prec in ("fp64", "fp32"):
        for adj in (False, True):
            for _ in range(args.warmup):
                api.toeplitz_mm(f, d, n, X, adjoint=adj, prec=prec)
            t = float(np.median(per_call_ms(lambda: api.toeplitz_mm(f, d, n, X, adjoint=adj, prec=prec),
                                            max(20, args.steps))))
            key = f"{prec}_{'TH_X' if adj else 'T_X'}"
            out[key] = {"ms_median": round(t, 5), "tflops": round(8.0 * N * N * r / (t * 1e-3) / 1e12, 3)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U, s, V, rank, sweeps = host.power_svd(host.GpuToeplitz(f, d, n), blocks[0], blocks[1],
                                           N * np.finfo(float).eps, rank=m)
    torch.cuda.synchronize()
    out["power_svd_gpu_products"] = {"s": round(time.perf_counter() - t0, 4), "sweeps": sweeps,
                                     "sigma_rel_diff_vs_dense_T": float(f"{np.max(np.abs(s - sig_ref) / sig_ref):.3e}")}
    return out


# The paper's S-build times on its own efficiency workload (d=3, n=20, N=9261,
# deterministic inputs, noise-free; Sec. 2 timing table, complex FP64, machine of Sec. 5:
# 2x Xeon E5-2690 v3 + Tesla K40c): t_S in seconds for m = 5, 10, 15, 20.
PAPER_T_S = {5: 0.1100, 10: 0.1199, 15: 0.1290, 20: 0.1495}


def paper_workload(dev, args, per_call_ms):
    """The paper's efficiency workload on this GPU: the S-build (FP64, the paper's
    arithmetic, FP32-MFMA and split bfloat16) for m = 5..20 against the paper's t_S, the whole GPU
    path of Algorithm 1 (samples, power SVD with GPU block products, S, nodes,
    Gram/rhs, LS), and the Lanczos SVD (Algorithm 2) with GPU products."""
    import numpy as np
    import torch

    from paper_2012_11430_amd import api, host
    from workload import paper_efficiency_inputs, random_orthonormal

    d, n = 3, 20
    N = (n + 1) ** d
    out = {"workload": "d=3, n=20, N=9261, noise-free, t_j(i) = ((i-1)m+j-1) 10^-ceil(log10 dm), c_j = j + ij",
           "paper_hardware": "2x Xeon E5-2690 v3 + Tesla K40c (FP64)", "m": {}}
    mu = np.array([1.0, 1j, -0.5]) / np.linalg.norm([1.0, 1j, -0.5])
    for m in sorted(PAPER_T_S):
        t, c = paper_efficiency_inputs(d, m)
        f = api.samples(torch.from_numpy(t).to(dev), torch.from_numpy(c).to(dev), n)
        rng = np.random.Generator(np.random.PCG64(140 + m))
        blocks = (random_orthonormal(rng, N, 2 * m), random_orthonormal(rng, N, 2 * m))
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        U, s, V, rank, sweeps = host.power_svd(host.GpuToeplitz(f, d, n), blocks[0], blocks[1],
                                               N * np.finfo(float).eps, rank=m)
        Ud, sd, Vd = (torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (U, s, V))
        S = api.build_S(f, d, n, Ud, sd, Vd, prec="fp64").cpu().numpy()
        z, t_est = host.nodes(S, mu)
        gram, rhs = api.coeffs(torch.from_numpy(z).to(dev), f, d, n)
        host.solve_normal_equations(gram.cpu().numpy(), rhs.cpu().numpy())
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        lrng = np.random.Generator(np.random.PCG64(240 + m))
        p1 = lrng.standard_normal(N) + 1j * lrng.standard_normal(N)
        restarts = [lrng.standard_normal(N) + 1j * lrng.standard_normal(N) for _ in range(4)]
        torch.cuda.synchronize()
        l0 = time.perf_counter()
        _, s_l, _, rank_l = host.lanczos_svd(host.GpuToeplitz(f, d, n), p1, N * np.finfo(float).eps, restarts)
        torch.cuda.synchronize()
        lanczos = {"s": round(time.perf_counter() - l0, 4), "rank": rank_l,
                   "sigma_rel_diff_vs_power": float(f"{np.max(np.abs(s_l[:m] - s) / s):.3e}")}
        row = {"paper_t_S_s": PAPER_T_S[m], "lanczos_svd_gpu_products": lanczos,
               "paper_gflops": round(s_flops(d, N, m) / PAPER_T_S[m] / 1e9, 1),
               "algorithm1_gpu_path_s": round(wall, 4), "svd_sweeps": sweeps}
        S_p = {}
        for prec in ("fp64", "fp32", "bf16x3"):
            for _ in range(args.warmup):
                api.build_S(f, d, n, Ud, sd, Vd, prec=prec)
            ms = float(np.median(per_call_ms(lambda: api.build_S(f, d, n, Ud, sd, Vd, prec=prec), 20)))
            S_p[prec] = api.build_S(f, d, n, Ud, sd, Vd, prec=prec)
            row[prec] = {"s_build_ms": round(ms, 4),
                         "fs_equivalent_tflops": round(s_flops(d, N, m) / (ms * 1e-3) / 1e12, 2),
                         "own_work_tflops": round(tile_flops(d, n, m) / (ms * 1e-3) / 1e12, 2),
                         "speedup_vs_paper_t_S": round(PAPER_T_S[m] / (ms * 1e-3), 1)}
        # the S of each precision against the FP64 S on the same factors: the paper's
        # inputs at m >= 10 have sigma_m / sigma_1 down to ~3e-12, and Sigma^{-1}
        # amplifies the rounding of FP32 inputs by sigma_1 / sigma_m
        row["sigma_m_over_sigma_1"] = float(f"{s[-1] / s[0]:.3e}")
        for p in ("fp32", "bf16x3"):
            row[p]["s_rel_diff_vs_fp64"] = float(
                f"{float(torch.linalg.norm(S_p[p] - S_p['fp64']) / torch.linalg.norm(S_p['fp64'])):.3e}")
        out["m"][str(m)] = row
    return out


def _match_errors(t_est, c_est, t_true, c_true):
    """max torus |dt| and ||dc|| / ||c|| after an optimal assignment of the nodes."""
    import numpy as np
    from scipy.optimize import linear_sum_assignment

    diff = np.abs(t_est[None, :, :] - t_true[:, None, :]) % 1.0
    dist = np.minimum(diff, 1.0 - diff).max(axis=2)
    rows, cols = linear_sum_assignment(dist)
    dt = float(dist[rows, cols].max())
    dc = float(np.linalg.norm(c_est[cols] - c_true[rows]) / np.linalg.norm(c_true))
    return dt, dc


def noise_sweep_c2(dev, args, per_call_ms):
    """c2 (d=3, n=19, N=8000, m=30) over its noise levels: the SVD by Algorithm 3
    with GPU block products (T is never formed), S in FP64, FP32-MFMA and split
    bfloat16, the recovered t_j, c_j of each against the truth, and per level the
    operational accuracy estimates of Sec. 5 (detected rank, sigma_m / sigma_{m+1},
    relative LS residual of each precision); the S-build
    of each precision timed as the median of per-call HIP events, with the tile
    kernel's launch time and its fraction of the MFMA peak on its own work."""
    import numpy as np
    import torch

    from paper_2012_11430_amd import api, autotune, host
    from workload import config_instances, random_orthonormal

    inst = config_instances("c2", count=1)[0]
    d, n, m, N = inst.d, inst.n, inst.m, inst.N
    if not args.no_tune:
        for prec in ("fp64", "fp32", "bf16x3"):
            autotune.tune_single(dev, d, n, m, prec, reps=10)
    rng = np.random.Generator(np.random.PCG64(2020))
    blocks = (random_orthonormal(rng, N, 2 * m), random_orthonormal(rng, N, 2 * m))
    t_d = torch.from_numpy(inst.t).to(dev)
    c_d = torch.from_numpy(inst.c).to(dev)
    rows = []
    for level in inst.noise_levels:
        noise = torch.from_numpy(inst.noise(level)).to(dev) if level > 0 else None
        f = api.samples(t_d, c_d, n, noise=noise)
        tol = max(N * np.finfo(float).eps, level)
        info = {}
        U, s, V, detected, sweeps = host.power_svd(host.GpuToeplitz(f, d, n), blocks[0], blocks[1], tol, rank=m,
                                                   info=info)
        Ud, sd, Vd = (torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (U, s, V))
        # the operational accuracy estimates of Sec. 5: the rank the SVD step detects at
        # tolerance max(N eps, noise), sigma_m / sigma_{m+1} (sigma_{m+1} from the first
        # sweep's estimates) and the relative LS residual ||A^T c - f_I|| / ||f_I||
        est = info.get("first_sweep_sigma")
        row = {"noise": level, "svd_sweeps": sweeps, "detected_rank": int(detected),
               "sigma_m_over_sigma_m_plus_1": (float(f"{s[m - 1] / est[m]:.3e}")
                                               if est is not None and est.size > m and est[m] > 0 else None)}
        fI = host.samples_on_index_set(f.cpu().numpy(), d, n)
        S = {}
        for prec in ("fp64", "fp32", "bf16x3"):
            S[prec] = api.build_S(f, d, n, Ud, sd, Vd, prec=prec)
            z_p, t_p = host.nodes(S[prec].cpu().numpy(), inst.mu)
            gram, rhs, AT = api.coeffs(torch.from_numpy(z_p).to(dev), f, d, n, want_AT=True)
            c_p = host.solve_normal_equations(gram.cpu().numpy(), rhs.cpu().numpy())
            dt, dc = _match_errors(t_p, c_p, inst.t, inst.c)
            res = float(np.linalg.norm(AT.cpu().numpy() @ c_p - fI) / np.linalg.norm(fI))
            row[prec] = {"max_dt_vs_truth": float(f"{dt:.3e}"), "rel_dc_vs_truth": float(f"{dc:.3e}"),
                         "ls_rel_residual": float(f"{res:.3e}")}
        for p in ("fp32", "bf16x3"):
            row[f"s_rel_diff_{p}_vs_fp64"] = float(f"{float(torch.linalg.norm(S[p] - S['fp64']) / torch.linalg.norm(S['fp64'])):.3e}")
        rows.append(row)
    # timing (values do not matter): the last level's inputs, every precision
    timing = {}
    reps = max(20, args.steps)
    for prec in ("fp64", "fp32", "bf16x3"):
        for _ in range(args.warmup):
            api.build_S(f, d, n, Ud, sd, Vd, prec=prec)
        api.profile_enable(dev, DOMINANT)
        ms = float(np.median(per_call_ms(lambda: api.build_S(f, d, n, Ud, sd, Vd, prec=prec), reps)))
        nl, tot = api.profile_read(dev)
        api.profile_enable(dev, None)
        tiles = tot / max(1, nl)
        own = tile_flops(d, n, m)
        timing[prec] = {"s_build_ms_median": round(ms, 5), "calls": reps,
                        "fs_equivalent_tflops": round(s_flops(d, N, m) / (ms * 1e-3) / 1e12, 2),
                        "tiles_ms": round(tiles, 5), "tiles_own_work_tflops": round(own / (tiles * 1e-3) / 1e12, 2),
                        "tiles_frac_of_peak": round(own / (tiles * 1e-3) / 1e12 / PEAK_TFLOPS[prec], 4),
                        "plan": autotune.plan(dev, d, n, m, prec)}
    return {"workload": "c2: d=3, n=19, N=8000, m=30, separation 0.08, |c| log-uniform [1e-2, 1]", "levels": rows,
            "s_build": timing, "own_work_flops_per_launch": tile_flops(d, n, m)}


def _closed_form_factors(t, c, d, n):
    """Input preparation: exact reduced SVD of the noise-free T = V_z diag(c) V_z^*
    from V_z = Q R (host, O(N m^2))."""
    import itertools

    import numpy as np
    ks = np.array(list(itertools.product(range(n + 1), repeat=d)), dtype=float)
    Q, R = np.linalg.qr(np.exp(-2j * np.pi * (ks @ t.T)))
    Ub, s, Vbh = np.linalg.svd(R @ np.diag(c) @ R.conj().T)
    return Q @ Ub, s, Q @ Vbh.conj().T


def batched_c3(dev, args):
    """c3: 512 uneven instances; FP32 batched S-build replayed from a HIP graph vs
    the plain FP64 per-instance loop. Returns instances/s and TFLOP/s."""
    import numpy as np
    import torch

    from paper_2012_11430_amd import api, autotune
    from workload import config_instances

    insts = config_instances("c3")
    dev_inst = []
    flops = own = 0.0
    for inst in insts:
        U, s, V = _closed_form_factors(inst.t, inst.c, inst.d, inst.n)
        f = api.samples(torch.from_numpy(inst.t).to(dev), torch.from_numpy(inst.c).to(dev), inst.n,
                        noise=torch.from_numpy(inst.noise()).to(dev))
        dev_inst.append((inst.d, inst.n, f, torch.from_numpy(U).to(dev), torch.from_numpy(s).to(dev),
                         torch.from_numpy(V).to(dev)))
        flops += s_flops(inst.d, inst.N, inst.m)
        own += tile_flops(inst.d, inst.n, inst.m)
    tuned = None
    if not args.no_tune:
        tuned = autotune.tune_batch(dev_inst, "fp32", reps=2)
    else:
        autotune.load_cache(dev)
    batch = api.Batch(dev_inst, prec="fp32")
    reps = max(3, args.steps // 4)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_graph():
        batch.capture()
        for _ in range(2):
            batch.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            batch.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    batch.set_schedule("queue")        # one persistent launch over all tiles
    ms_queue = time_graph()
    batch.set_schedule("classes")      # the default: one launch per tile class, four streams
    ms_graph = time_graph()

    # the batched form in FP64 (class launches, graph replays): batching alone, same precision
    batch64 = api.Batch(dev_inst, prec="fp64")
    batch64.capture()
    for _ in range(2):
        batch64.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        batch64.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_graph64 = e0.elapsed_time(e1) / reps
    batch64.close()

    outs = [torch.empty_like(S) for S in batch.S]

    def loop64():
        for (d, n, f, U, s, V), o in zip(dev_inst, outs):
            api.build_S(f, d, n, U, s, V, prec="fp64", out=o)
    loop64()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        loop64()
    e1.record()
    torch.cuda.synchronize()
    ms_loop = e0.elapsed_time(e1) / reps
    rel = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(batch.S, outs))
    batch.close()
    n_inst = len(insts)
    return {
        "workload": "c3: 512 instances, d~U{1,2,3}, N log-uniform in [64,4096], m~U{2..32}, noise 1e-7",
        "instances_per_s_fp32_batched_graph": round(n_inst / (ms_graph * 1e-3), 1),
        "instances_per_s_fp64_per_instance_loop": round(n_inst / (ms_loop * 1e-3), 1),
        "speedup": round(ms_loop / ms_graph, 2),
        "ms_fp32_graph": round(ms_graph, 4),
        "schedule": "classes (one launch per tile class over four streams; the default)",
        "ms_fp32_graph_queue": round(ms_queue, 4),
        "ms_fp64_graph_batched": round(ms_graph64, 4),
        "speedup_fp64_batched_over_fp64_loop": round(ms_loop / ms_graph64, 2),
        "ms_fp64_loop": round(ms_loop, 4),
        "fs_equivalent_tflops_fp32_graph": round(flops / (ms_graph * 1e-3) / 1e12, 3),
        "own_work_tflops_fp32_graph": round(own / (ms_graph * 1e-3) / 1e12, 3),
        "rel_err_fp32_vs_fp64": float(f"{rel:.3e}"),
        "tuning": tuned,
    }


def adjoint_c4(dev, args):
    """c4: 64 instances (d=2, n=47, m=16); forward FP32 S-build + hand-written
    adjoint (FP32 accumulate) through torch.autograd: all instances in one batched
    forward and one batched adjoint, and, for comparison, one instance at a time."""
    import numpy as np
    import torch

    from paper_2012_11430_amd import api
    from paper_2012_11430_amd.autograd import BatchedPencil, pencil
    from workload import config_instances

    insts = config_instances("c4")
    data = []
    for inst in insts:
        U, s, V = _closed_form_factors(inst.t, inst.c, inst.d, inst.n)
        t_d, c_d = torch.from_numpy(inst.t).to(dev), torch.from_numpy(inst.c).to(dev)
        clean = api.samples(t_d, c_d, inst.n)
        noisy = api.samples(t_d, c_d, inst.n, noise=torch.from_numpy(inst.noise()).to(dev))
        Ud, sd, Vd = torch.from_numpy(U).to(dev), torch.from_numpy(s).to(dev), torch.from_numpy(V).to(dev)
        # S_l(f) - S_l^ref = S_l(f - f0): the loss is formed from the sample difference
        data.append((inst, noisy - clean, Ud, sd, Vd))

    bp = BatchedPencil([(inst.d, inst.n, Ud, sd, Vd) for inst, delta, Ud, sd, Vd in data], prec="fp32")
    delta_all = torch.cat([delta for inst, delta, *_r in data])

    def fwd_bwd_batched():
        f = delta_all.detach().requires_grad_(True)
        torch.sum(torch.abs(bp(f)) ** 2).backward()
        return f.grad

    def fwd_bwd_loop():
        for inst, delta, Ud, sd, Vd in data:
            f = delta.detach().requires_grad_(True)
            S = pencil(f, inst.d, inst.n, Ud, sd, Vd, "fp32", "fp32")
            torch.sum(torch.abs(S) ** 2).backward()

    def timed(fn, reps):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_batched = timed(fwd_bwd_batched, max(5, args.steps // 2))
    ms_loop = timed(fwd_bwd_loop, 3)
    # adjoint kernels alone (batched): device time of the backward's library launches
    gS_all = torch.randn(sum(bp.gs_sizes), dtype=torch.complex128, device=dev)
    ms_adj = timed(lambda: bp.batch.adjoint(gS_all), max(5, args.steps // 2))
    ms_fwd = timed(bp.batch.run, max(5, args.steps // 2))
    bp.close()
    inst = insts[0]
    f1 = s_flops(inst.d, inst.N, inst.m)
    # own work of the adjoint tiles (row-extended form): the (n+2)^d x N product of
    # inner dimension m, 8 (n+2)^d N m flops
    adj_own = 8.0 * (inst.n + 2) ** inst.d * inst.N * inst.m
    flops = len(insts) * 2 * f1
    return {
        "workload": "c4: 64 instances of d=2, n=47, m=16, noise 1e-6; L = sum_l ||S_l - S_l^ref||_F^2 "
                    "= sum_l ||S_l(f - f0)||_F^2",
        "ms_forward_backward_64_batched": round(ms_batched, 4),
        "fs_equivalent_tflops_forward_plus_adjoint_batched": round(flops / (ms_batched * 1e-3) / 1e12, 3),
        "ms_batched_forward_kernels": round(ms_fwd, 4),
        "ms_batched_adjoint_kernels": round(ms_adj, 4),
        "fs_equivalent_tflops_batched_adjoint_kernels": round(len(insts) * f1 / (ms_adj * 1e-3) / 1e12, 3),
        "own_work_tflops_batched_adjoint_kernels": round(len(insts) * adj_own / (ms_adj * 1e-3) / 1e12, 3),
        "own_work_tflops_batched_forward_kernels": round(len(insts) * tile_flops(inst.d, inst.n, inst.m)
                                                         / (ms_fwd * 1e-3) / 1e12, 3),
        "ms_forward_backward_64_one_instance_at_a_time": round(ms_loop, 4),
    }


def cpu_baseline(inst, U, sig, V, z, S_gpu, steps, recovered, grid_gpu):
    """The CPU oracle timed on `steps` whole steps of the same workload, and its
    S-build alone (median of 3, all host threads and one thread); also the relative
    error of the GPU S-build against the oracle on the same inputs."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import prony_oracle as O

    d, n = inst.d, inst.n
    level = inst.noise_levels[0]
    noise = inst.noise(level) if level > 0 else None
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    t0 = time.perf_counter()
    for _ in range(steps):
        grid = O.samples(inst.t, inst.c, n, abs_noise=noise)
        O.toeplitz(grid, d, n, 0)
        S = O.pencil_matrices(grid, d, n, U, sig, V)
        O.coefficient_products(z, grid, d, n)
    el = (time.perf_counter() - t0) / steps

    def s_only():
        t = time.perf_counter()
        O.pencil_matrices(grid, d, n, U, sig, V)
        return time.perf_counter() - t
    s_all = float(np.median([s_only() for _ in range(3)]))
    with threadpool_limits(limits=1):
        s_one = s_only()
    F = s_flops(d, inst.N, inst.m)
    rel = {p: max(float(np.linalg.norm(S_gpu[p][l] - S[l]) / np.linalg.norm(S[l])) for l in range(d))
           for p in S_gpu}
    # t_j, c_j of each precision against the FP64 oracle pipeline (same SVD inputs)
    # and against the truth; host FP64 steps: SVD, eig, LS
    z_or, t_or, _ = O.nodes_from_pencil(S, inst.mu)
    c_or, _ = O.least_squares_coefficients(z_or, grid, d, n)
    recovery = {"fp64_host_steps": "SVD (Algorithm 3 on T), eig of C_mu, LS (normal equations)"}
    dt, dc = O.recovery_errors(dict(t=t_or, c=c_or), inst.t, inst.c)
    recovery["oracle_vs_truth"] = {"max_dt": float(f"{dt:.3e}"), "rel_dc": float(f"{dc:.3e}")}
    for p, (t_p, c_p) in recovered.items():
        dt_o, dc_o = O.recovery_errors(dict(t=t_p, c=c_p), t_or, c_or)
        dt_t, dc_t = O.recovery_errors(dict(t=t_p, c=c_p), inst.t, inst.c)
        recovery[p] = {"max_dt_vs_oracle": float(f"{dt_o:.3e}"), "rel_dc_vs_oracle": float(f"{dc_o:.3e}"),
                       "max_dt_vs_truth": float(f"{dt_t:.3e}"), "rel_dc_vs_truth": float(f"{dc_t:.3e}")}
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": round(F / el / 1e12, 6),
        "unit": "TFLOP/s",
        "cores": int(threads),
        "cores_note": "BLAS threads the oracle's matrix products ran on (the rest of the oracle is one thread)",
        "host_cpus_available": len(os.sched_getaffinity(0)),
        "kind": "oracle",
        "sample": f"{steps} whole oracle steps (samples, T, S_1..S_d, Gram/rhs) of the same workload, "
                  f"{el:.3f} s per step",
        "cpu_model": model,
        "s_build_only": {"s_median_all_threads": round(s_all, 4), "tflops_all_threads": round(F / s_all / 1e12, 6),
                         "s_one_thread": round(s_one, 4), "tflops_one_thread": round(F / s_one / 1e12, 6)},
        "s_rel_err_vs_oracle": {p: float(f"{v:.3e}") for p, v in rel.items()},
        "recovery_vs_oracle": recovery,
        "samples_max_abs_err": float(f"{np.max(np.abs(grid_gpu - grid)):.3e}"),
    }


if __name__ == "__main__":
    main()
