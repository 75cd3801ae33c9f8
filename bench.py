#!/usr/bin/env python3
"""MGM-GMRES solve benchmark on one MI355X.

Workload (the paper's headline use of MGM: a right preconditioner for GMRES,
Sec. 4.6/5): torus R=1, r=1/3 with N=160,000 Poisson-disk points, RBF-FD
PHS r^5 + degree-3 polynomials on 50-point stencils, the surface Poisson
problem solved as the bordered system (Sec. 4.4), zero-mean trigonometric
right-hand side, FGMRES(40) to relative residual 1e-10 with one MGM V(1,1)
cycle per iteration. Inputs are seeded and synthetic (no dataset).

A step is one complete solve from x0 = 0 (right-hand side resident in HBM,
setup excluded as in the paper). The FP64 V-cycle and the reduced-precision
V-cycles (FP32; FP16 values with FP32 row scales) are timed in turn; `value`
is the solve time with the FP32 V-cycle (FP64 Krylov), the FP64 solve time
and the ratio are reported beside it.

learned_smoothers: the same FP32 solve with learned per-node Chebyshev
smoothers (an extension; the paper smooths with Gauss-Seidel): each smoothed
level trains its own network on the GPU, keeps it when its measured
convergence factor beats Gauss-Seidel's, and the solve is timed again (not
`value`, which stays the paper's method).

roofline: the dominant kernel is the patch-blocked Gauss-Seidel launch
(k_gs_patch, FP32 here: about 70% of the V-cycle's device time). Every
smoother launch of one V-cycle (all smoothed levels, pre- and post-sweeps) is
queued back to back on the launch stream between two HIP events through
mgm_time_kernel; achieved = algorithmic bytes per launch (operator values and
column indices of the rows a launch updates, plus their f, u read, u write,
inverse diagonal and local colour, each once) / mean launch time. `traffic`
is the HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE and
WRITE_SIZE, scaled by what they read for a plain copy of known size) over the
same launches; it is reported only while the kernel source is the one that
was measured (null otherwise).

cpu_baseline: the CPU oracle's FGMRES solve (same algorithm, FP64, NumPy/SciPy,
single thread) on the same workload (N=160,000; one solve of about 3 s after a
setup of about a minute that is not timed). `--cpu-sample N` runs it on a
smaller torus instead and scales the time linearly in N (iteration counts are
N-independent for MGM, Tables 2-3), which underestimates: at N=40,000 the
scaled figure is 0.78 s against 2.6 s measured at N=160,000.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of the dominant kernel from two rocprofv3 --pmc passes over
# `bench.py --workload traffic` (summary and commands in
# profiles/gs_patch_torus160k_traffic.md): bytes per launch, valid only for
# the kernel source it was measured on (SHA-256 over lane_ops.h + gs_patch.h,
# which also fixes which levels stage their halo).
GS_TRAFFIC = {"source_sha256": "0681a9d6c2c43480c901c3f88aa869920316267d93121901513d4dae4a6e7307", "bytes_per_launch": 23478655,
              "summary": "profiles/gs_patch_torus160k_traffic.md"}


def gs_traffic():
    import hashlib
    h = hashlib.sha256()
    for name in ("lane_ops.h", "gs_patch.h"):
        with open(os.path.join(ROOT, "paper_2204_06154_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != GS_TRAFFIC["source_sha256"]:
        return None
    return GS_TRAFFIC["bytes_per_launch"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(n_sample: int, n_full: int, reps: int = 3):
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import hierarchy, krylov, vcycle

    wl = synth.torus_workload(n_sample)
    t0 = time.perf_counter()
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    setup_s = time.perf_counter() - t0
    A = vcycle.make_operator(H)
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)
    f = np.concatenate([wl.f, [0.0]])
    ts = []
    with threadpool_limits(limits=1):
        for _ in range(reps):
            t0 = time.perf_counter()
            _, info = krylov.fgmres(A, M, f, tol=1e-10, restart=40, maxit=400)
            ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    scale = n_full / n_sample
    where = (f"the torus workload itself (N={n_full})" if n_sample == n_full else
             f"the torus workload at N={n_sample}, scaled x{scale:g} to N={n_full}")
    return {"value": round(t * 1e3 * scale, 1), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": f"oracle FP64 FGMRES(40) + V(1,1) solve to 1e-10 on {where}: {info.iters} iterations, "
                      f"median of {reps} solve(s) {t:.3f} s, setup ({setup_s:.0f} s, multi-threaded) excluded; "
                      f"SciPy sparse kernels, BLAS limited to 1 thread"}


def timed_solves(m, f, u, krylov, steps, warmup, **kw):
    import numpy as np
    import torch
    for _ in range(warmup):
        u.zero_()
        m.solve(f, u, krylov=krylov, **kw)
    torch.cuda.synchronize()
    times, info = [], None
    for _ in range(steps):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = m.solve(f, u, krylov=krylov, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return 1e3 * float(np.mean(times)), info


def bench_learned(args):
    """Star surface with 16:1 density bumps (N=500,000), RBF-FD r^3 + degree 2, k=30,
    screened Poisson (mu=1): FGMRES(40) to 1e-10 with the Gauss-Seidel V-cycle
    vs. the learned per-node Chebyshev smoother on the fine level."""
    import numpy as np
    import torch

    import synth
    from paper_2204_06154_amd import mgm

    t0 = time.perf_counter()
    wl = synth.star_density_workload(args.n)
    log(f"inputs N={args.n} generated in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    m = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, precision=args.vcycle_precision), device=0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    f = torch.tensor(wl.f, device="cuda")
    u = torch.zeros_like(f)
    out = {"workload": f"star surface, 16:1 density bumps, N={args.n}, RBF-FD r^3+deg2 k=30, screened mu=1, "
                       f"FGMRES(40) to 1e-10, V-cycle {args.vcycle_precision}",
           "levels": [int(x) for x in m.export("level_sizes")], "setup_s": round(setup_s, 2)}
    ms, info = timed_solves(m, f, u, "fgmres", args.steps, args.warmup, restart=40, maxit=400, rtol=1e-10)
    vc_ms, _ = m.time_kernel("vcycle", 0, reps=10)
    out["gs"] = {"ms": round(ms, 3), "iters": info["iters"], "rel_res": info["rel_res_true"], "vcycle_us": round(vc_ms * 1e3, 1)}
    log(f"GS: {ms:.2f} ms, {info['iters']} iters, V-cycle {vc_ms * 1e3:.0f} us")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2204)
    starts = torch.randn((4, args.n), generator=gen, device="cuda", dtype=torch.float64)
    t0 = time.perf_counter()
    tr = m.train_smoother(starts, steps=args.train_steps, lr=1e-3, s=3, iters_per_start=2, seed=5, init=True,
                          activate=1)
    train_s = time.perf_counter() - t0
    out["training"] = {"steps": args.train_steps, "snapshots": 8, "seconds": round(train_s, 2), "lam": tr["lam"],
                       "loss_first": tr["loss_first"], "loss_last": tr["loss_last"], "rate_gs": tr["rate_gs"],
                       "rate_learned": tr["rate_learned"], "active": tr["active"]}
    log(f"training {train_s:.1f} s, loss {tr['loss_first']:.4f} -> {tr['loss_last']:.4f}, "
        f"rates GS {tr['rate_gs']:.3f} learned {tr['rate_learned']:.3f}, active {tr['active']}")
    m.set_smoother(True)
    ms, info = timed_solves(m, f, u, "fgmres", args.steps, args.warmup, restart=40, maxit=400, rtol=1e-10)
    vc_ms, _ = m.time_kernel("vcycle", 0, reps=10)
    out["learned"] = {"ms": round(ms, 3), "iters": info["iters"], "rel_res": info["rel_res_true"],
                      "vcycle_us": round(vc_ms * 1e3, 1)}
    log(f"learned: {ms:.2f} ms, {info['iters']} iters, V-cycle {vc_ms * 1e3:.0f} us")
    out["speedup_learned_vs_gs"] = round(out["gs"]["ms"] / out["learned"]["ms"], 3)
    # per-level learned smoothing: train every coarse smoothed level on its own
    # sub-hierarchy (same recipe), keep those whose factor beats Gauss-Seidel
    sizes = out["levels"]
    mask = 1 if tr["active"] else 0
    levels = []
    t0 = time.perf_counter()
    for j in range(1, len(sizes) - 1):
        sj = torch.randn((4, sizes[j]), generator=gen, device="cuda", dtype=torch.float64)
        tj = m.train_smoother(sj, steps=args.train_steps, lr=1e-3, s=3, iters_per_start=2, seed=5 + j, init=True,
                              activate=1, level=j)
        levels.append({"level": j, "rate_gs": tj["rate_gs"], "rate_learned": tj["rate_learned"],
                       "active": tj["active"]})
        if tj["active"]:
            mask |= 1 << j
    train_levels_s = time.perf_counter() - t0
    m.set_smoother(mask)
    ms, info = timed_solves(m, f, u, "fgmres", args.steps, args.warmup, restart=40, maxit=400, rtol=1e-10)
    vc_ms, _ = m.time_kernel("vcycle", 0, reps=10)
    out["learned_all_levels"] = {"ms": round(ms, 3), "iters": info["iters"], "rel_res": info["rel_res_true"],
                                 "vcycle_us": round(vc_ms * 1e3, 1), "level_mask": mask, "levels": levels,
                                 "training_s": round(train_levels_s, 2)}
    log(f"learned on levels (mask {mask:#x}): {ms:.2f} ms, {info['iters']} iters, V-cycle {vc_ms * 1e3:.0f} us; "
        f"coarse rates {[(l['rate_gs'], l['rate_learned']) for l in levels]}")
    print(json.dumps(out), flush=True)
    m.close()


def bench_torus_learned(args, m, f, u, sizes, prec, gs):
    """The torus solve with learned per-node Chebyshev smoothers: every
    smoothed level trains its own network on the GPU (4 random starts x 2
    MGM iterations of snapshots on its bordered sub-hierarchy, Adam) with its
    own number of Richardson steps per sweep (default 2 on every level),
    each step holding the multiplier fixed; a level keeps it when its
    measured convergence factor beats Gauss-Seidel's (one step per sweep
    loses that comparison on the coarse levels here, although forcing it on
    would shorten the solve)."""
    import torch
    m.set_precision(prec)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2204)
    s_by_level = [int(x) for x in str(args.learned_s).split(",")]
    levels, mask = [], 0
    t0 = time.perf_counter()
    for j in range(len(sizes) - 1):
        sj = torch.randn((4, sizes[j]), generator=gen, device="cuda", dtype=torch.float64)
        s_j = s_by_level[min(j, len(s_by_level) - 1)]
        tj = m.train_smoother(sj, steps=args.learned_steps, lr=args.learned_lr, s=s_j, iters_per_start=2,
                              seed=5 + j, init=True, activate=1, level=j)
        levels.append({"level": j, "s": s_j, "rate_gs": round(tj["rate_gs"], 4), "rate_learned": round(tj["rate_learned"], 4),
                       "loss_first": round(tj["loss_first"], 5), "loss_last": round(tj["loss_last"], 5),
                       "active": tj["active"]})
        if tj["active"]:
            mask |= 1 << j
    train_s = time.perf_counter() - t0
    m.set_smoother(mask)
    ms, info = timed_solves(m, f, u, "fgmres", args.steps, args.warmup, restart=40, maxit=400, rtol=1e-10)
    vc_ms, _ = m.time_kernel("vcycle", 0, reps=20)
    out = {"precision": prec, "s_by_level": [l["s"] for l in levels], "adam_steps": args.learned_steps,
           "lr": args.learned_lr, "training_s": round(train_s, 2),
           "level_mask": mask, "levels": levels, "ms": round(ms, 3), "iters": info["iters"],
           "rel_res_true": float(f"{info['rel_res_true']:.4g}"), "vcycle_us": round(vc_ms * 1e3, 1),
           "speedup_vs_gs": round(gs["ms"] / ms, 3)}
    log(f"learned smoothers (mask {mask:#x}, s={[l['s'] for l in levels]}, trained in {train_s:.1f} s): {ms:.2f} ms/solve, "
        f"{info['iters']} iters, V-cycle {vc_ms * 1e3:.0f} us; factors "
        f"{[(l['rate_gs'], l['rate_learned']) for l in levels]}")
    if mask:
        # the Richardson launches of one V-cycle (k_rowop_patch in Richardson
        # mode on patch-blocked levels), timed back to back like the GS roofline
        lr_ms, lr_bytes = m.time_kernel("learned", -1, reps=20)
        lr_gbs = lr_bytes / (lr_ms * 1e-3) / 1e9
        out["smoother_roofline"] = {"bound": "hbm", "kernel": f"learned Richardson steps {prec}, mean over one V-cycle",
                                    "achieved": round(lr_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(lr_gbs / HBM_PEAK_GBS, 4), "us_per_launch": round(lr_ms * 1e3, 3),
                                    "algorithmic_bytes_per_launch": round(lr_bytes)}
        log(f"learned smoother launches: {lr_ms * 1e3:.2f} us, {lr_bytes / 1e6:.2f} MB -> {lr_gbs:.0f} GB/s")
        # the same smoothers in the other V-cycle precisions
        out["solves"] = {prec: {"ms": out["ms"], "iters": out["iters"], "vcycle_us": out["vcycle_us"]}}
        for p2 in args.precisions.split(","):
            if p2 == prec:
                continue
            m.set_precision(p2)
            ms2, info2 = timed_solves(m, f, u, "fgmres", args.steps, args.warmup, restart=40, maxit=400, rtol=1e-10)
            vc2, _ = m.time_kernel("vcycle", 0, reps=20)
            out["solves"][p2] = {"ms": round(ms2, 3), "iters": info2["iters"],
                                 "rel_res_true": float(f"{info2['rel_res_true']:.4g}"), "vcycle_us": round(vc2 * 1e3, 1)}
            log(f"learned smoothers {p2}: {ms2:.2f} ms/solve, {info2['iters']} iters, V-cycle {vc2 * 1e3:.0f} us")
        if "fp64" in out["solves"] and prec != "fp64":
            out["speedup_mixed_vs_fp64"] = round(out["solves"]["fp64"]["ms"] / out["ms"], 3)
        m.set_precision(prec)
    m.set_smoother(False)
    return out


def bench_sphere1m(args):
    """Unit sphere N=1,048,576, GFD degree 2, k=25, screened Poisson (mu=1),
    BiCGSTAB to 1e-10 with the FP64 and the FP16-row-scale V-cycles."""
    import numpy as np
    import torch

    import synth
    from paper_2204_06154_amd import mgm

    t0 = time.perf_counter()
    wl = synth.big_sphere_workload(args.n)
    log(f"inputs N={args.n} generated in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    m = mgm.Mgm(wl.xyz, wl.normals, wl.params, device=0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    f = torch.tensor(wl.f, device="cuda")
    u = torch.zeros_like(f)
    out = {"workload": f"unit sphere N={args.n} Fibonacci, GFD deg2 k=25 alpha=16, screened mu=1, BiCGSTAB to 1e-10",
           "levels": [int(x) for x in m.export("level_sizes")], "setup_s": round(setup_s, 2)}
    ref = None
    for prec in ("fp64", "fp32", "fp16"):
        m.set_precision(prec)
        ms, info = timed_solves(m, f, u, "bicgstab", args.steps, args.warmup, maxit=400, rtol=1e-10)
        vc_ms, vc_b = m.time_kernel("vcycle", 0, reps=10)
        sol = u.cpu().numpy()
        if ref is None:
            ref = sol
        err = float(np.linalg.norm(sol - ref) / np.linalg.norm(ref))
        out[prec] = {"ms": round(ms, 3), "iters": info["iters"], "rel_res": info["rel_res_true"],
                     "vcycle_us": round(vc_ms * 1e3, 1), "vcycle_GBps": round(vc_b / (vc_ms * 1e-3) / 1e9, 1),
                     "err_vs_fp64_solution": err}
        log(f"{prec}: {ms:.2f} ms, {info['iters']} applications, V-cycle {vc_ms * 1e3:.0f} us, err {err:.1e}")
    out["speedup_fp16_vs_fp64"] = round(out["fp64"]["ms"] / out["fp16"]["ms"], 3)
    # bandwidth of the operator and smoother kernels on an operator larger than
    # the 256 MB Infinity Cache, next to what a plain device copy reaches
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * src.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    out["copy_GBps"] = round(copy_gbps, 1)

    def rl(ms, nbytes, kernel):
        gbps = nbytes / (ms * 1e-3) / 1e9
        return {"kernel": kernel, "bound": "hbm", "us_per_launch": round(ms * 1e3, 2), "bytes_per_launch": nbytes,
                "achieved": round(gbps, 1), "peak": 8000.0, "unit": "GB/s", "frac": round(gbps / 8000.0, 4),
                "frac_of_copy": round(gbps / copy_gbps, 4)}

    m.set_precision("fp64")
    sp_ms, sp_b = m.time_kernel("spmv", 0, reps=20)
    out["spmv_roofline"] = rl(sp_ms, sp_b, "outer FP64 operator, fine level")
    out["gs_roofline"] = {}
    for prec in ("fp64", "fp32", "fp16"):
        m.set_precision(prec)
        g_ms, g_b = m.time_kernel("gs", 0, reps=10)
        out["gs_roofline"][prec] = rl(g_ms, g_b, f"k_gs_patch {prec}: one fine-level sweep")
    log(f"copy {copy_gbps:.0f} GB/s; SpMV {out['spmv_roofline']['achieved']:.0f} GB/s; fine GS sweep "
        + ", ".join(f"{k} {v['achieved']:.0f} GB/s" for k, v in out["gs_roofline"].items()))
    print(json.dumps(out), flush=True)
    m.close()


def bench_sbdf2(args):
    """Repeated screened solves: SBDF2 steps of u_t = Delta u on a sphere of N
    points (RBF-FD r^3 + deg 2, k=30, dt = 0.05, so L = I - (2 dt / 3) D),
    FGMRES + MGM to 1e-8 from the extrapolated guess 2u^n - u^{n-1} (warm)
    and from zero (cold); the right-hand sides are formed on the device."""
    import numpy as np
    import torch

    import synth
    from paper_2204_06154_amd import mgm

    t0 = time.perf_counter()
    wl = synth.sbdf2_workload(args.n)
    log(f"inputs N={args.n} generated in {time.perf_counter() - t0:.1f} s")
    prec = args.vcycle_precision
    m = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, precision=prec), device=0)
    u0 = torch.tensor(wl.f, device="cuda")
    out = {"workload": f"SBDF2 time stepping of u_t = Delta u, unit sphere N={args.n}, RBF-FD r^3+deg2 k=30, "
                       f"dt=0.05, FGMRES(40)+MGM to 1e-8, V-cycle {prec}",
           "levels": [int(x) for x in m.export("level_sizes")]}
    nsteps = max(args.steps, 1) * 4
    for mode in ("warm", "cold"):
        u_prev, u_cur = u0.clone(), u0.clone()
        iters, times = [], []
        for k in range(nsteps + 1):      # step 0 warms the graphs up and is not timed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rhs = (4.0 * u_cur - u_prev) / 3.0
            u = 2.0 * u_cur - u_prev if mode == "warm" else torch.zeros_like(u_cur)
            u, info = m.solve(rhs, u, krylov="fgmres", restart=40, maxit=200, rtol=1e-8, x0=(mode == "warm"))
            torch.cuda.synchronize()
            if k > 0:
                times.append(time.perf_counter() - t0)
                iters.append(info["iters"])
            u_prev, u_cur = u_cur, u
        out[mode] = {"steps": nsteps, "ms_per_step": round(1e3 * float(np.mean(times)), 3), "iters": iters}
        log(f"{mode}: {out[mode]['ms_per_step']:.2f} ms per step, iterations {iters}")
    out["speedup_warm_vs_cold"] = round(out["cold"]["ms_per_step"] / out["warm"]["ms_per_step"], 3)
    print(json.dumps(out), flush=True)
    m.close()


def bench_harmonics(args):
    """Repeated solves with an indefinite shift: shift-invert Arnoldi (ARPACK
    through scipy) for the 9 eigenvalues of D_h nearest sigma = -1 on a unit
    sphere of N points (RBF-FD l = 5, k = 5, n = 42), every Arnoldi step one
    FGMRES + MGM solve of (D_h + I) v = x to 1e-10 on the device."""
    import numpy as np
    import torch

    import synth
    from paper_2204_06154_amd import mgm
    from paper_2204_06154_amd.shift_invert import shift_invert_eigs

    t0 = time.perf_counter()
    wl = synth.harmonics_workload(args.n)
    log(f"inputs N={args.n} generated in {time.perf_counter() - t0:.1f} s")
    prec = args.vcycle_precision
    t0 = time.perf_counter()
    m = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, precision=prec), device=0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    f = torch.tensor(wl.f, device="cuda")
    m.solve(f, krylov="fgmres", restart=40, maxit=400, rtol=1e-10)   # graphs warmed up, not timed
    ev, iters, solve_s, total_s = shift_invert_eigs(m, wl.params["mu"], 9, wl.f, ncv=36)
    # Sphere eigenvalues -l(l+1) have multiplicity 2l+1; the discretisation
    # splits each multiplet only slightly, so single-vector Arnoldi may return
    # a member of the next multiplet instead of the last of one: each value is
    # compared with its nearest -l(l+1).
    ll = np.arange(0, 8)
    exact = -(ll * (ll + 1.0))
    near = exact[np.argmin(np.abs(ev.real[:, None] - exact[None, :]), axis=1)]
    out = {"workload": f"shift-invert Arnoldi, 9 eigenvalues nearest sigma=-1, unit sphere N={args.n}, "
                       f"RBF-FD r^11+deg5 k=42, FGMRES(40)+MGM to 1e-10, V-cycle {prec}",
           "levels": [int(x) for x in m.export("level_sizes")], "setup_s": round(setup_s, 2),
           "solves": len(iters), "iters_median": float(np.median(iters)), "iters_max": int(max(iters)),
           "solve_s": round(solve_s, 4), "ms_per_solve": round(1e3 * solve_s / len(iters), 3),
           "eigs_total_s": round(total_s, 4),
           "eigenvalues": [round(float(v), 9) for v in ev.real],
           "max_err_vs_minus_l_lp1": float(np.max(np.abs(ev.real - near)))}
    log(f"{len(iters)} solves, median {out['iters_median']} / max {out['iters_max']} iterations, "
        f"{out['ms_per_solve']:.2f} ms per solve, eigenvalue error {out['max_err_vs_minus_l_lp1']:.2e}")
    print(json.dumps(out), flush=True)
    m.close()


def bench_setup(args):
    """Preprocessing time (Alg. 2) of the torus workload: everything on the
    host, with the batched device weight solve, and with the kNN searches and
    Galerkin products on the device as well (median of 3 set-ups each)."""
    import numpy as np
    import torch

    import synth
    from paper_2204_06154_amd import mgm

    wl = synth.torus_workload(args.n)
    out = {"workload": f"setup of the torus N={args.n}, RBF-FD r^5+deg3 k=50, bordered Poisson"}
    for name, flags in (("host", dict(device_weights=0, device_setup=0)),
                        ("device_weights", dict(device_weights=1, device_setup=0)),
                        ("device_weights_knn_rap", dict(device_weights=1, device_setup=1))):
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, **flags), device=0)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            m.close()
        out[name + "_s"] = round(float(np.median(ts)), 3)
        log(f"setup {name}: {out[name + '_s']:.3f} s")
    out["host_threads"] = len(os.sched_getaffinity(0))
    print(json.dumps(out), flush=True)


def bench_geodesic(args):
    """Heat-method geodesic distance on the unit sphere (N points; LBO RBF-FD
    l = 3, n = 20; surface gradient RBF-FD l = 2, n = 12): three backward-Euler
    heat solves, the normalised gradient and its divergence, and the bordered
    Poisson solve, all to 1e-8 with FGMRES + MGM, timed end to end; the
    surface-operator kernels are also timed on their own (algorithmic bytes:
    weights, columns, the input once and the output once per node)."""
    import numpy as np
    import torch

    import synth
    from paper_2204_06154_amd import mgm
    from paper_2204_06154_amd.geodesic import heat_distance

    t0 = time.perf_counter()
    wl = synth.geodesic_workload(args.n)
    hp = wl.heat
    log(f"inputs N={args.n} generated in {time.perf_counter() - t0:.1f} s")
    prec = args.vcycle_precision
    t0 = time.perf_counter()
    m = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, precision=prec), device=0)
    m.surface_ops_setup(hp["grad_phs_order"], hp["grad_degree"], hp["grad_stencil"])
    mh = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, problem="screened", mu=hp["dt"], precision=prec), device=0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    heat_distance(mh, m, hp["source"], steps=hp["steps"])          # graphs warmed up, not timed
    times = []
    for _ in range(max(args.steps, 1)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, iters = heat_distance(mh, m, hp["source"], steps=hp["steps"])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    x = wl.xyz
    exact = np.arccos(np.clip(x @ x[hp["source"]], -1.0, 1.0))
    err = np.abs(d.cpu().numpy() - exact)
    n, ns = args.n, hp["grad_stencil"]
    u = torch.rand(n, dtype=torch.float64, device="cuda")
    g = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    dv = torch.empty(n, dtype=torch.float64, device="cuda")
    kern = {}
    for name, fn, nbytes in (("grad_normalise", lambda: m.surface_gradient(u, g, normalise=True),
                              n * ns * 28 + n * 8 + n * 24),
                             ("divergence", lambda: m.surface_divergence(g, dv), n * ns * 28 + n * 24 + n * 8)):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 50
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        kern[name] = {"us": round(us, 2), "bytes": nbytes, "GB_s": round(nbytes / us / 1e3, 1)}
        log(f"{name}: {us:.1f} us, {nbytes / 1e6:.1f} MB -> {nbytes / us / 1e3:.0f} GB/s")
    out = {"workload": f"heat-method geodesics, unit sphere N={args.n}, LBO RBF-FD r^7+deg3 k=20, gradient "
                       f"RBF-FD r^5+deg2 k=12, dt={hp['dt']} x{hp['steps']}, FGMRES(40)+MGM to 1e-8, V-cycle {prec}",
           "levels": [int(v) for v in m.export("level_sizes")], "setup_s": round(setup_s, 2),
           "ms_total": round(1e3 * float(np.median(times)), 3), "iters": iters,
           "mean_err_vs_great_circle": float(err.mean()), "max_err_vs_great_circle": float(err.max()),
           "kernels": kern}
    log(f"distance in {out['ms_total']:.2f} ms, iterations {iters}, mean error {err.mean():.4f}")
    print(json.dumps(out), flush=True)
    m.close()
    mh.close()


def bench_table2(args):
    """The paper's scaling study on the sphere (Table 2): icosahedral nodes
    N = 10,242 ... 655,362, shifted Poisson (mu = 1) with a random
    right-hand side, RBF-FD l = 3, 5, 7 (k = l, n = (l+1)(l+2)), MGM-GMRES(40),
    MGM-BiCGSTAB and standalone MGM (the stationary iteration) to 1e-12:
    iteration counts with the FP64 cycle beside the paper's, and solve times
    with the FP64 and FP32 cycles."""
    import numpy as np
    import torch

    import synth
    from paper_2204_06154_amd import mgm

    paper = {r[0]: r for r in json.load(open(os.path.join(ROOT, "tests", "golden", "table2_sphere_rbffd_mgm.json")))["rows"]}
    rows = []
    for k in (5, 6, 7, 8):
        for ell in (3, 5, 7):
            wl = synth.icosahedral_workload(k, ell)
            n = len(wl.xyz)
            t0 = time.perf_counter()
            m = mgm.Mgm(wl.xyz, wl.normals, wl.params, device=0)
            torch.cuda.synchronize()
            setup_s = time.perf_counter() - t0
            f = torch.tensor(wl.f, device="cuda")
            u = torch.zeros_like(f)
            row = {"N": n, "l": ell, "levels": [int(v) for v in m.export("level_sizes")], "setup_s": round(setup_s, 2)}
            for prec in ("fp64", "fp32"):
                m.set_precision(prec)
                for kry in ("fgmres", "bicgstab") + (("stationary",) if prec == "fp64" else ()):
                    ms, info = timed_solves(m, f, u, kry, 2, 1, restart=40, maxit=300, rtol=1e-12)
                    row[f"{kry}_{prec}"] = {"iters": info["iters"], "ms": round(ms, 3), "rel_res": info["rel_res_true"]}
            col = {3: 1, 5: 3, 7: 5}[ell]
            row["paper"] = {"gmres": paper[n][col], "bicgstab": paper[n][col + 1]}
            rows.append(row)
            log(f"N={n} l={ell}: GMRES {row['fgmres_fp64']['iters']} (paper {paper[n][col]}), BiCGSTAB "
                f"{row['bicgstab_fp64']['iters']} (paper {paper[n][col + 1]}), standalone MGM "
                f"{row['stationary_fp64']['iters']}; FP32-cycle GMRES "
                f"{row['fgmres_fp32']['ms']:.2f} ms, setup {setup_s:.1f} s")
            m.close()
    print(json.dumps({"workload": "icosahedral sphere, shifted Poisson mu=1, random RHS, RBF-FD l=3/5/7, tol 1e-12",
                      "rows": rows}), flush=True)


def bench_weights(n_sys: int):
    """Batched per-node weight solves: n_sys star-surface stencils (n = 50, r^3 + degree 3: 60x60 systems), the
    FP64 matrix-core kernel and the mixed-precision one, each the median of 5 timed calls."""
    import numpy as np
    import torch

    import synth
    from paper_2204_06154_amd import mgm

    t0 = time.perf_counter()
    wl4 = synth.star_workload(n_sys)
    sten = mgm.stencils(wl4.xyz, 50)
    log(f"star surface N={n_sys} + stencils in {time.perf_counter() - t0:.1f} s")
    d_x = torch.tensor(wl4.xyz, device="cuda")
    d_n = torch.tensor(wl4.normals, device="cuda")
    d_s = torch.tensor(sten, device="cuda")
    d_w = torch.empty((n_sys, 50), dtype=torch.float64, device="cuda")
    mgm.batched_weights(d_x, d_n, d_s, 1, 3, d_w)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    ts = []
    for _ in range(reps):
        ev0.record()
        mgm.batched_weights(d_x, d_n, d_s, 1, 3, d_w)
        ev1.record()
        ev1.synchronize()
        ts.append(ev0.elapsed_time(ev1))
    wms = float(np.median(ts))
    S = 60
    flops = (2.0 / 3.0 * S ** 3 + 2.0 * S * S) * n_sys
    # the FP32 matrix-core elimination with FP64 refinement, same systems
    d_wm = torch.empty_like(d_w)
    mgm.batched_weights(d_x, d_n, d_s, 1, 3, d_wm, mixed=True)
    tsm = []
    for _ in range(reps):
        ev0.record()
        mgm.batched_weights(d_x, d_n, d_s, 1, 3, d_wm, mixed=True)
        ev1.record()
        ev1.synchronize()
        tsm.append(ev0.elapsed_time(ev1))
    wms_mixed = float(np.median(tsm))
    mixed_diff = float((torch.abs(d_wm - d_w).amax(dim=1) / torch.abs(d_w).amax(dim=1)).max())
    bw = {"systems": n_sys, "system_size": S, "ms": round(wms, 3),
          "systems_per_s": round(n_sys / (wms * 1e-3)),
          "TFLOPs_lu_model": round(flops / (wms * 1e-3) / 1e12, 2),
          "frac_fp64_peak": round(flops / (wms * 1e-3) / 1e12 / 78.6, 4),
          "note": "FP64 Gauss-Jordan with partial pivoting, one wavefront per system, in panels of 4 columns "
                  "whose updates run on the FP64 matrix cores (MFMA); flops = (2/3)S^3 + 2S^2",
          "mixed": {"ms": round(wms_mixed, 3), "max_rel_diff_vs_fp64": float(f"{mixed_diff:.3g}"),
                    "note": "FP32 Gauss-Jordan on [A | I] on the FP32 matrix cores, then FP64 iterative "
                            "refinement (mgm_batched_weights_mixed)"}}
    log(f"batched weights: {wms:.2f} ms for {n_sys} systems ({bw['TFLOPs_lu_model']} TFLOP/s LU model); "
        f"mixed precision {wms_mixed:.2f} ms, max rel diff {mixed_diff:.1e}")
    return bw


def bench_traffic(args):
    """Launch set for the HBM-traffic counters: FP32 patch-GS launches of the
    torus workload as the roofline times them (every smoother launch of a
    V-cycle, `--steps` times), then three 256 MiB device copies whose
    FETCH_SIZE / WRITE_SIZE readings calibrate the counters (each copy moves
    exactly 256 MiB in and 256 MiB out)."""
    import torch

    import synth
    from paper_2204_06154_amd import mgm

    wl = synth.torus_workload(args.n)
    m = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, gs_block=args.gs_block, gs_flow=args.gs_flow,
                                         precision=mgm.FP32), device=0)
    f = torch.tensor(__import__("numpy").concatenate([wl.f, [0.0]]), device="cuda")
    m.vcycle(f)
    ms, nbytes = m.time_kernel("gs", -1, reps=args.steps)
    torch.cuda.synchronize()
    x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "traffic", "n": args.n, "gs_us_per_launch": round(ms * 1e3, 3),
                      "gs_bytes_per_launch": round(nbytes), "copy_bytes_each_way": 256 * 1024 * 1024}), flush=True)
    m.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=160_000)
    ap.add_argument("--precisions", default="fp64,fp32,fp16")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle points (0 = the workload's N)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--weights-n", type=int, default=500_000)
    ap.add_argument("--gs-block", type=int, default=256)
    ap.add_argument("--gs-flow", type=int, choices=[0, 1], default=1,
                    help="1: one launch per patch-blocked sweep (dataflow order between patches); "
                         "0: one launch per patch colour")
    ap.add_argument("--cycle", choices=["V", "W", "F"], default="V", help="multigrid cycle of the torus workload")
    ap.add_argument("--workload", choices=["torus", "learned", "sphere1m", "traffic", "sbdf2", "harmonics",
                                                 "setup", "geodesic", "table2", "weights"],
                    default="torus")
    ap.add_argument("--train-steps", type=int, default=200)
    ap.add_argument("--learned-steps", type=int, default=400,
                    help="Adam steps per level of the torus run's learned smoothers (0: skip that part)")
    ap.add_argument("--learned-lr", type=float, default=3e-3, help="Adam learning rate of the torus run's learned smoothers")
    ap.add_argument("--learned-s", default="2",
                    help="Richardson steps per sweep of the torus run's learned smoothers, by level (the last value "
                         "holds for the remaining levels)")
    ap.add_argument("--vcycle-precision", default="fp32", help="V-cycle precision of the learned and sbdf2 workloads")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the MGM solve is not sharded across GPUs (a single-GPU "
              "implementation; multi-GPU runs are not supported).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2204_06154_amd import mgm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "learned":
        if args.n == 160_000:
            args.n = 500_000
        return bench_learned(args)
    if args.workload == "traffic":
        return bench_traffic(args)
    if args.workload == "weights":
        n_sys = args.weights_n if args.weights_n > 0 else 500_000
        bw = bench_weights(n_sys)
        print(json.dumps(dict(workload=f"batched PHS weight solves, star surface, {n_sys} stencils n=50, "
                                       "r^3 + degree 3 (60x60 systems)", **bw)), flush=True)
        return
    if args.workload == "sbdf2":
        if args.n == 160_000:
            args.n = 300_000
        return bench_sbdf2(args)
    if args.workload == "table2":
        return bench_table2(args)
    if args.workload == "geodesic":
        if args.n == 160_000:
            args.n = 872_773
        return bench_geodesic(args)
    if args.workload == "setup":
        return bench_setup(args)
    if args.workload == "harmonics":
        if args.n == 160_000:
            args.n = 436_605
        return bench_harmonics(args)
    if args.workload == "sphere1m":
        if args.n == 160_000:
            args.n = 1 << 20
        return bench_sphere1m(args)
    t0 = time.perf_counter()
    wl = synth.torus_workload(args.n)
    log(f"inputs N={args.n} generated in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    m = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, gs_block=args.gs_block, gs_flow=args.gs_flow, cycle=args.cycle),
                device=0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    sizes = [int(s) for s in m.export("level_sizes")]
    ncol = [int(c) for c in m.export("ncolours")]
    log(f"setup {setup_s:.1f} s, levels {sizes}, colours {ncol}")
    f = torch.tensor(np.concatenate([wl.f, [0.0]]), device="cuda")
    u = torch.zeros_like(f)

    results = {}
    for prec in args.precisions.split(","):
        m.set_precision(prec)
        for _ in range(args.warmup):
            u.zero_()
            m.solve(f, u, krylov="fgmres", restart=40, maxit=400, rtol=1e-10)
        torch.cuda.synchronize()
        times = []
        info = None
        for _ in range(args.steps):
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = m.solve(f, u, krylov="fgmres", restart=40, maxit=400, rtol=1e-10)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        vc_ms, vc_bytes = m.time_kernel("vcycle", 0, reps=20)
        results[prec] = dict(ms=1e3 * float(np.mean(times)), ms_min=1e3 * float(np.min(times)), iters=info["iters"],
                             rel_res_true=info["rel_res_true"], vcycle_ms=vc_ms, vcycle_bytes=vc_bytes)
        log(f"{prec}: {results[prec]['ms']:.2f} ms/solve, {info['iters']} iters, "
            f"res {info['rel_res_true']:.2e}, V-cycle {vc_ms * 1e3:.0f} us")

    main_prec = "fp32" if "fp32" in results else list(results)[0]
    m.set_precision(main_prec)
    gs_ms, gs_bytes = m.time_kernel("gs", -1, reps=20)      # every smoother launch of a V-cycle
    gs0_ms, gs0_bytes = m.time_kernel("gs", 0, reps=10)     # fine-level launches alone
    m.set_precision("fp64")
    sp_ms, sp_bytes = m.time_kernel("spmv", 0, reps=50)
    gs_gbs = gs_bytes / (gs_ms * 1e-3) / 1e9
    sp_gbs = sp_bytes / (sp_ms * 1e-3) / 1e9
    gs0_gbs = gs0_bytes / (gs0_ms * 1e-3) / 1e9
    log(f"GS launches ({main_prec}, all levels of a V-cycle): {gs_ms * 1e3:.2f} us, {gs_bytes / 1e6:.2f} MB "
        f"-> {gs_gbs:.0f} GB/s; fine level alone {gs0_ms * 1e3:.2f} us, {gs0_bytes / 1e6:.2f} MB -> {gs0_gbs:.0f} GB/s")
    log(f"SpMV (fp64, fine level): {sp_ms * 1e3:.2f} us, {sp_bytes / 1e6:.1f} MB -> {sp_gbs:.0f} GB/s")

    learned = bench_torus_learned(args, m, f, u, sizes, main_prec, results[main_prec]) if args.learned_steps > 0 else None

    # batched per-node weight solves (500,000 star-surface stencils, n=50, r^3 + degree 3: 60x60 systems)
    bw = bench_weights(args.weights_n) if args.weights_n > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        cpu = cpu_baseline(args.cpu_sample or args.n, args.n)
        log(f"cpu baseline {cpu['value']} ms (took {time.perf_counter() - t0:.0f} s)")

    r = results[main_prec]
    out = {
        "metric": "MGM-GMRES solve time to 1e-10 rel. residual (FP64 vs mixed); SpMV HBM GB/s",
        "value": round(r["ms"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": f"{main_prec} V-cycle, f64 Krylov",
        "data": "synthetic (seeded Poisson-disk torus points, random trigonometric rhs)",
        "config": {"workload": f"torus R=1 r=1/3, N={args.n} Poisson-disk points, RBF-FD r^5+deg3 k=50, "
                               f"bordered surface Poisson, FGMRES(40)+MGM {args.cycle}(1,1) to 1e-10",
                   "levels": sizes, "colours": ncol, "setup_s": round(setup_s, 2)},
        "solves": {p: {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in d.items()}
                   for p, d in results.items()},
        "speedup_mixed_vs_fp64": round(results["fp64"]["ms"] / r["ms"], 3) if "fp64" in results else None,
        "spmv": {"kernel": "outer FP64 operator, fine level (k_rowop_patch on the patch ELL; k_spmv on plain levels)",
                 "us": round(sp_ms * 1e3, 2), "bytes": sp_bytes,
                 "GBps": round(sp_gbs, 1), "frac": round(sp_gbs / HBM_PEAK_GBS, 4)},
        "roofline": {"bound": "hbm",
                     "kernel": f"k_gs_patch {main_prec}: mean over the smoother launches of one V-cycle",
                     "achieved": round(gs_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gs_gbs / HBM_PEAK_GBS, 4),
                     "traffic": gs_traffic() if main_prec == "fp32" else None,
                     "algorithmic_bytes_per_launch": round(gs_bytes), "us_per_launch": round(gs_ms * 1e3, 3),
                     "fine_level": {"us_per_launch": round(gs0_ms * 1e3, 3), "bytes_per_launch": round(gs0_bytes),
                                    "GBps": round(gs0_gbs, 1)}},
        "learned_smoothers": learned,
        "batched_weights": bw,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    m.close()


if __name__ == "__main__":
    main()
