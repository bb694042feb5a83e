#!/usr/bin/env python3
"""Throughput benchmark of the scatter-limited hybrid step on one MI355X.

Headline workload (default): the large resident solve, 1024x1024 cells on
[0,10]^2 with sigma_s and sigma_a uniform on [0.01, 20] per 32x32-cell block,
unit source on the central 2x2 blocks, N_s = 3, 1e8 source particles per MC
pass, dt = 0.05, 50 time steps from t = 0, S_16, FP64, vacuum boundaries.  A
step is one whole hybrid time step: the scatter-limited MC pass, the DG S_N
collided solve, the remap source, the remap MC pass and the census cap.
Inputs are resident on the device before the timed region; the timed steps
are one solve on a fresh solver (warm-up steps run on another solver).

The timed steps run in the library's timing mode (the MC-pass kernels
launched between HIP events on the solver's stream, the rest of each step as
graphs), so the roofline of the dominant kernel is measured over the timed
region itself; the one-graph-per-step production mode is timed as well.

Prints one JSON line: segments/s (value), per-step time, the roofline of both
MC-pass kernels, the FP32-tracking run with its relative L2 deviation from
FP64 and the QMC error at the same particle count, the precision form (256^2
thick medium with voids), the benchmark checkerboard, a bounded serving run
against one-solve-at-a-time, and the CPU oracle on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "track segments/s FP32 vs FP64 at fixed L2 error; p50/p99 batched solve latency"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes: per segment the (sigma_s, sigma_a) gather and one FP64
# tally read-modify-write; per census particle its state (x, y, Ox, Oy, w and
# the cell index; the 8-byte history id is not counted) read once by each
# pass, and each census candidate written once by the remap pass
SEG_BYTES = {0: 16 + 16, 1: 8 + 16}
CENSUS_BYTES = {0: 5 * 8 + 4, 1: 5 * 4 + 4}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PROFILES = {"c5": "k_mc_pass_random_blocks_1024_counters.txt",
            "c2": "k_mc_pass_checkerboard_140_counters.txt"}
WORKLOAD_NAMES = {
    "c5": "large resident solve (1024x1024 random blocks)",
    "c5_sub": "128x128 subproblem of the large resident solve",
    "c2": "checkerboard 7x7 unit blocks (absorber sigma_a=10 / scatterer sigma_s=1), unit "
          "source in the centre block",
    "c3": "thick medium with voids",
    "c1": "homogeneous box"}


# Collided-solve acceleration per workload when --si-accel is not given: the
# 1024x1024 solve (22 plain source iterations per step) takes the diffusion
# synthetic acceleration (12); its fixed point is the same to si_tol.
SI_ACCEL_DEFAULT = {"c5": 1}


def make_problem(args, precision):
    from paper_2511_16821_amd import workloads as W
    kw = dict(precision=precision)
    acc = args.si_accel if args.si_accel is not None else SI_ACCEL_DEFAULT.get(args.workload)
    if acc is not None:
        kw["si_accel"] = acc
    if args.ns is not None:
        kw["n_s"] = args.ns
    if args.particles:
        kw["n_particles"] = args.particles
    if args.workload == "c2":
        return W.c2(**kw)
    if args.workload == "c1":
        return W.c1(**kw)
    if args.workload == "c3":
        return W.c3(**kw)
    if args.workload == "c5":
        return W.c5(**kw)
    if args.workload == "c5_sub":
        return W.c5_subproblem(**kw)
    raise SystemExit("unknown workload " + args.workload)


def describe(p):
    return ("%dx%d cells on [%g,%g]x[%g,%g], N_s=%d, %d particles/pass, dt=%g, S_%d"
            % (p["nx"], p["ny"], p["x_lo"], p["x_hi"], p["y_lo"], p["y_hi"], p["n_s"],
               p["n_particles"], p["dt"], p["sn_order"]))


DIRECT = False  # --direct: kernels launched one by one, no graphs (counter runs)


def timed_run(S, torch, p, steps, warmup, timing=True, keep=False):
    """Times `steps` steps of a fresh solver (after `warmup` steps on another
    one).  timing: steps in timing mode (kernel times from HIP events).
    Returns (wall seconds, stats[, solver if keep])."""
    if warmup > 0:
        w = S.Solver(p)
        w.set_graphs(not DIRECT)
        w.advance(warmup, allow_not_converged=True)
        w.synchronize(allow_not_converged=True)
        w.destroy()
    s = S.Solver(p)
    s.set_graphs(not DIRECT)
    s.set_timing(timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance(steps, allow_not_converged=True)
    s.synchronize(allow_not_converged=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = s.get_stats()
    if keep:
        return t1 - t0, st, s
    s.destroy()
    return t1 - t0, st


def kernel_source_digest():
    """Digest of the MC-pass kernel sources; counter figures taken for another
    digest describe a different kernel and are not reported."""
    import hashlib
    h = hashlib.sha256()
    for f in ("mc.hip", "slh_common.hpp"):
        with open(os.path.join(ROOT, "paper_2511_16821_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_entries(profile):
    """The key: value lines of the committed rocprofv3 summary `profile`, or
    None when it is missing or was taken on other kernel code."""
    path = os.path.join(ROOT, "profiles", profile) if profile else ""
    if not profile or not os.path.isfile(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_digest") != kernel_source_digest():
        return None
    return kv


def measured_traffic(profile, kernel, prec):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary `profile` (FETCH_SIZE + WRITE_SIZE, scaled by the plain-copy
    calibration), or None when the summary is missing or was taken on other
    kernel code."""
    kv = _profile_entries(profile)
    if kv is None:
        return None
    key = "hbm_bytes_per_launch[%s,%s]" % (kernel, "fp64" if prec == 0 else "fp32")
    return float(kv[key]) if key in kv else None


def measured_issue(profile, kernel, prec):
    """What bounds `kernel` besides HBM, from the SQ/TCC counters of the same
    summary: the share of SIMD cycles issuing a VALU instruction, the active
    lanes per VALU instruction and the L2 hit rate (FP64 tracking only), or
    None."""
    kv = _profile_entries(profile)
    key = "counters[%s,%s]" % (kernel, "fp64" if prec == 0 else "fp32")
    if kv is None or key not in kv:
        return None
    f = dict(t.split("=", 1) for t in kv[key].split() if "=" in t)
    try:
        return {"valu_issue": float(f["valu_issue"]), "active_lanes": float(f["active_lanes"]),
                "l2_hit": float(f["l2_hit"])}
    except (KeyError, ValueError):
        return None


def rooflines(st, steps, prec, profile):
    """Roofline of each MC-pass kernel over the timed steps: algorithmic bytes
    per launch (per segment SEG_BYTES; per census-in particle CENSUS_BYTES
    read by each pass; per census candidate CENSUS_BYTES written by the
    remap pass) over the kernel's mean duration from HIP events.  Returns
    (dominant, both)."""
    rows = []
    for name, ms, seg, extra in (
            ("k_mc_pass<step 1>", st["ms_kernel_mc_total"], st["seg_mc_total"],
             CENSUS_BYTES[prec] * st["census_in_total"]),
            ("k_mc_pass<step 3>", st["ms_kernel_remap_total"], st["seg_remap_total"],
             CENSUS_BYTES[prec] * (st["census_in_total"] + st["census_out_total"]))):
        byts = SEG_BYTES[prec] * seg + extra
        per_launch_bytes = byts / steps
        per_launch_s = ms * 1e-3 / steps
        achieved = per_launch_bytes / per_launch_s / 1e9 if per_launch_s > 0 else 0.0
        rows.append({"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(profile, name, prec),
                     "issue": measured_issue(profile, name, prec),
                     "kernel": name, "avg_launch_ms": round(ms / steps, 4),
                     "bytes_per_launch": int(per_launch_bytes),
                     "segments_per_launch": int(seg / steps)})
    return max(rows, key=lambda r: r["avg_launch_ms"]), rows


def _oracle_pass_worker(job):
    """One scatter-limited MC pass of the oracle (step 1 of the first time
    step, no census) on problem `p` with `n_src` particles and seed `seed`;
    returns (segments, seconds)."""
    p, n_src, seed = job
    import numpy as np
    from oracle import oracle as O
    O.build()
    mesh = O.Mesh(p)
    pts = O.Points(int(p.get("points", 0)))
    q4 = np.repeat(np.asarray(p["q"], dtype=np.float64).ravel(), 4)
    t0 = time.perf_counter()
    _, _, _, seg, _ = O.mc_pass(mesh, pts, 1, int(p["n_s"]), q4, n_src, O.Bank(0), seed, 0,
                                float(p.get("w_cut_rel", 1e-8)), False)
    return seg, time.perf_counter() - t0


def cpu_baseline(p, n_src, workers):
    """The CPU oracle on a bounded sample of the headline workload: the
    scatter-limited MC pass of its first step (the oracle's DG solve of a
    1024^2 mesh with 256 directions would take minutes per sweep, and the
    metric counts track segments), with n_src particles, first on one core,
    then as `workers` independent processes with different seeds on as many
    cores; segments/s of the all-core run is the value."""
    import multiprocessing as mp
    from oracle import oracle as O
    O.build()
    seg1, t1 = _oracle_pass_worker((p, n_src, int(p["seed"])))
    ctx = mp.get_context("spawn")
    jobs = [(p, n_src, int(p["seed"]) + 7919 * (k + 1)) for k in range(workers)]
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_pass_worker, jobs)
    seg = sum(r[0] for r in res)
    wall = max(r[1] for r in res)  # the slowest process's pass (start-up excluded)
    return {"value": seg / wall, "unit": "segments/s", "cores": workers, "kind": "oracle",
            "single_core_value": seg1 / t1,
            "sample": "the scatter-limited MC pass of the first step of the same workload "
                      "(%d source particles, %d segments in %.1f s on one core), then %d "
                      "concurrent processes with different seeds, one per core (%d segments; "
                      "the slowest pass took %.1f s)" % (n_src, seg1, t1, workers, seg, wall)}


def fp32_error(S, p64, p32, steps):
    """Max over steps of rel-L2(phi_R FP32-tracking, phi_R FP64), same seed."""
    import numpy as np
    a, b = S.Solver(p64), S.Solver(p32)
    worst = 0.0
    for _ in range(steps):
        a.advance(1, allow_not_converged=True)
        b.advance(1, allow_not_converged=True)
        x, y = a.get_flux(0), b.get_flux(0)
        worst = max(worst, float(np.linalg.norm(y - x) / max(np.linalg.norm(x), 1e-300)))
    a.destroy()
    b.destroy()
    return worst


def downsample4(phi):
    """4x4 block average (256x256 -> 64x64)."""
    ny, nx = phi.shape
    return phi.reshape(ny // 4, 4, nx // 4, 4).mean(axis=(1, 3))


def precision_form(S, torch, args):
    """Thick diffusive medium with voids, 256x256 cells: FP32-tracking vs FP64
    throughput at the same particle count and seed, the FP32 result's
    relative L2 deviation from the FP64 path on the 64x64 downsample (every
    step, max reported), and the QMC error of one run at that particle count,
    e_QMC = ||s|| / ||mean|| over independent Owen seeds (FP64, last step,
    same downsample).  The FP64 device path equals the CPU oracle to 1e-10
    (parity tests), so the deviation from it stands for the deviation from
    the oracle at this size."""
    import numpy as np
    from paper_2511_16821_amd import workloads as W
    out = []
    for ns in [int(v) for v in args.c3_ns.split(",") if v != ""]:
        kw = dict(n_s=ns, n_steps=args.c3_steps)
        if args.c3_particles:
            kw["n_particles"] = int(args.c3_particles)
        p64 = W.c3(precision=0, **kw)
        p32 = W.c3(precision=1, **kw)
        steps = args.c3_steps
        w64, st64 = timed_run(S, torch, p64, steps, 1)
        w32, st32 = timed_run(S, torch, p32, steps, 1)
        seg64 = st64["seg_mc_total"] + st64["seg_remap_total"]
        seg32 = st32["seg_mc_total"] + st32["seg_remap_total"]
        a, b = S.Solver(p64), S.Solver(p32)
        worst = 0.0
        for _ in range(steps):
            a.advance(1, allow_not_converged=True)
            b.advance(1, allow_not_converged=True)
            x = downsample4(a.get_flux(0).reshape(p64["ny"], p64["nx"]))
            y = downsample4(b.get_flux(0).reshape(p64["ny"], p64["nx"]))
            worst = max(worst, float(np.linalg.norm(y - x) / max(np.linalg.norm(x), 1e-300)))
        a.destroy()
        b.destroy()
        runs = []
        for r in range(args.c3_seeds):
            pr = dict(p64)
            pr["seed"] = int(p64["seed"]) + 1000003 * (r + 1)
            sr = S.Solver(pr)
            sr.advance(steps, allow_not_converged=True)
            runs.append(downsample4(sr.get_flux(0).reshape(p64["ny"], p64["nx"])))
            sr.destroy()
        runs = np.stack(runs)
        e_qmc = float(np.linalg.norm(runs.std(axis=0, ddof=1)) /
                      max(np.linalg.norm(runs.mean(axis=0)), 1e-300))
        row = {"n_s": ns, "n_particles": int(p64["n_particles"]), "steps": steps,
               "fp64_segments_per_s": seg64 / w64, "fp32_segments_per_s": seg32 / w32,
               "fp32_speedup": (seg32 / w32) / (seg64 / w64),
               "fp64_ms_per_step": 1e3 * w64 / steps, "fp32_ms_per_step": 1e3 * w32 / steps,
               "fp64_mc_kernel_ms_per_step": (st64["ms_kernel_mc_total"] +
                                              st64["ms_kernel_remap_total"]) / steps,
               "fp32_mc_kernel_ms_per_step": (st32["ms_kernel_mc_total"] +
                                              st32["ms_kernel_remap_total"]) / steps,
               "rel_l2_fp32_vs_fp64_max_over_steps": worst,
               "e_qmc": e_qmc, "e_qmc_seeds": args.c3_seeds,
               "fp32_within_bound": bool(worst < min(1e-4, e_qmc))}
        log("precision form:", json.dumps(row))
        out.append(row)
    return {"workload": "256x256 cells on [0,10]^2, sigma_s=100, sigma_a=0.01, 20% area of "
                        "seeded rectangular voids (sigma_t=0.1), unit source on the central "
                        "32x32 cells, dt=0.01, S_8, Owen-scrambled Sobol points",
            "downsample": "64x64 (4x4 block average) of phi_R at each step", "rows": out}


def cellwise_ns(S, torch, args):
    """Space-dependent scatter limit N_s(x) (the paper's stated next step) on
    the C3 thick medium with voids: limit k in the thick scatterer and 0 in the
    voids, against uniform limits k and 0.  Per map: time per step,
    segments/s, source iterations of the last step, and the relative L2
    difference of phi_R after the run from the uniform-0 run (same seed; all
    maps estimate the same flux)."""
    import numpy as np
    from paper_2511_16821_amd import workloads as W
    steps = args.nsx_steps
    rows = []
    base_flux = None
    for k in [int(v) for v in args.nsx_ns.split(",") if v != ""]:
        for name in ("uniform", "thick_k_voids_0"):
            if name == "thick_k_voids_0" and k == 0:
                continue
            p = W.c3(n_s=k, n_particles=int(args.nsx_particles), n_steps=steps)
            if name == "thick_k_voids_0":
                ss = np.asarray(p["sigma_s"], dtype=np.float64).ravel()
                p["n_s_cell"] = np.where(ss > 1.0, k, 0).astype(np.int32)
            s = S.Solver(p)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.advance(steps)
            s.synchronize(allow_not_converged=True)
            t = time.perf_counter() - t0
            st = s.get_stats()
            seg = st["seg_mc_total"] + st["seg_remap_total"]
            f = s.get_flux(0)
            s.destroy()
            if base_flux is None:
                base_flux = f
            row = {"map": name, "k": k, "ms_per_step": 1e3 * t / steps, "segments_per_s": seg / t,
                   "segments_per_step": seg / steps, "si_iterations_last": st["si_iterations"],
                   "rel_l2_phi_R_vs_uniform_0": float(np.linalg.norm(f - base_flux) /
                                                      np.linalg.norm(base_flux))}
            log("cellwise N_s:", json.dumps(row))
            rows.append(row)
    return {"workload": "C3 thick medium with voids (256x256, sigma_s=100 / voids sigma_t=0.1, "
                        "%g particles/pass, dt=0.01, S_8), %d steps; N_s(x) = k in the thick "
                        "medium and 0 in the voids, against uniform limits"
                        % (args.nsx_particles, steps), "rows": rows}


def reflective(S, torch, args):
    """Reflective sides on the C1 box (20x20 on [0,2]^2, sigma_s = 1,
    sigma_a = 0.1, central source, dt = 0.1, S_8; 1e6 particles per pass so
    that histories reach the sides within the run) against the vacuum case:
    all four sides, and x_lo + y_lo (the quarter of a symmetric problem).
    Time per step, segments/s, source iterations of the last step, leakage."""
    from paper_2511_16821_amd import workloads as W
    steps = args.reflect_steps
    rows = []
    for name, bc in (("vacuum", 0), ("x_lo+y_lo", 5), ("all four", 15)):
        p = W.c1(n_s=args.ns if args.ns is not None else 2, n_steps=steps, boundary=bc,
                 n_particles=10 ** 6)
        s = S.Solver(p)
        s.advance(2)
        s.synchronize(allow_not_converged=True)
        st0 = s.get_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(steps)
        s.synchronize(allow_not_converged=True)
        t = time.perf_counter() - t0
        st = s.get_stats()
        seg = (st["seg_mc_total"] + st["seg_remap_total"]
               - st0["seg_mc_total"] - st0["seg_remap_total"])
        bal = s.get_balance(2)
        row = {"sides": name, "ms_per_step": 1e3 * t / steps, "segments_per_s": seg / t,
               "si_iterations_last": st["si_iterations"], "leaked_last_remap": bal["leaked"]}
        s.destroy()
        log("reflective:", json.dumps(row))
        rows.append(row)
    return {"workload": "C1 box (20x20 on [0,2]^2, N_s=%d, 1e6 particles/pass, dt=0.1, S_8), "
                        "%d timed steps after 2" % (args.ns if args.ns is not None else 2, steps),
            "rows": rows}


def protocol(S, torch, args):
    """The paper's measurements on a stand-in (Sec. 3, Table 1 protocol): for
    each scatter limit N_s (-1 = unlimited, the plain MC reference case), the
    relative L2 error of phi_R after the last step against a same-method
    reference at 2^22 particles, for scrambled-Sobol' points (RMS over Owen
    seeds), pseudo-random points (RMS over seeds) and the paper's Halton points
    (RMS over random shifts), at particle counts 2^10
    .. 2^18; the same for scrambled Sobol' with the census histories drawing
    from their cells' cohort streams (census_qmc = 1, against its own
    reference); the fitted slopes alpha (error ~ N^-alpha), the
    source-iteration count of the collided solve, and the time per step."""
    import numpy as np
    from paper_2511_16821_amd import workloads as W
    ns_list = [int(v) for v in args.protocol_ns.split(",") if v != ""]
    ladder = [2 ** k for k in range(10, 19, 2)]
    rows = []
    for ns in ns_list:
        base = W.c1(n_s=ns, n_steps=args.protocol_steps, dt=args.protocol_dt)

        def run(n, points, seed, census=0):
            p = dict(base)
            p.update(n_particles=int(n), points=points, seed=int(seed), census_qmc=census)
            s = S.Solver(p, torch_allocator=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.advance(args.protocol_steps, allow_not_converged=True)
            f = s.get_flux(0)
            t = time.perf_counter() - t0
            it = s.get_stats()["si_iterations"]
            s.destroy()
            return f, t / args.protocol_steps, it

        refs = {c: run(2 ** 22, 0, 7777, c)[0] for c in (0, 1)}
        row = {"n_s": ns, "particles": ladder, "steps": args.protocol_steps}
        for name, mode, census in (("qmc", 0, 0), ("qmc_census_cohorts", 0, 1), ("mc", 1, 0),
                                   ("halton", 2, 0)):
            ref = refs[census]
            nref = max(np.linalg.norm(ref), 1e-300)
            errs, times, iters = [], [], []
            for n in ladder:
                e2 = 0.0
                for r in range(args.protocol_seeds):
                    f, t, it = run(n, mode, 1000 + 17 * r, census)
                    e2 += float(np.linalg.norm(f - ref) / nref) ** 2
                    times.append(t)
                    iters.append(it)
                errs.append((e2 / args.protocol_seeds) ** 0.5)
            slope = -float(np.polyfit(np.log(ladder), np.log(errs), 1)[0])
            row[name] = {"rel_l2": errs, "alpha": slope,
                         "ms_per_step_mean": 1e3 * float(np.mean(times))}
            row["si_iterations_last_step"] = int(np.median(iters))
        log("protocol:", json.dumps(row))
        rows.append(row)
    return {"workload": "20x20 cells on [0,2]^2, sigma_s=1, sigma_a=0.1, Q=1 on the central 2x2 "
                        "cells, dt=%g, S_8 (the C1 family); error of phi_R after %d steps against "
                        "a 2^22-particle run of the same method" % (args.protocol_dt,
                                                                    args.protocol_steps),
            "rows": rows}


def steady_protocol(S, torch, args):
    """The paper's own setting (Sec. 3, Table 1): steady state (one infinite
    time step), N_s in {0, 5, 10, 20, unlimited}, S_4, on the two stand-ins:
    the multi-region slab (80 cells) and the bent duct (30 x 50 cells).  For
    each N_s: the relative L2 error of phi_R against a 2^22-particle run of the
    same method, RMS over seeds, for Owen-scrambled Sobol', shifted Halton and
    pseudo-random points at 2^10 .. 2^18 particles, the fitted slopes, the
    time per solve, and the source-iteration count with the whole-flux
    stopping test (tolerance 1e-6) and, for comparison, the collided-only
    test at the same tolerance; where every cell has sigma_t > 0 (the duct),
    also the distance of the diffusion closing stage's solution from the S_N
    reference at the same particle count."""
    import numpy as np
    from paper_2511_16821_amd import workloads as W
    ns_list = [int(v) for v in args.steady_ns.split(",") if v != ""]
    ladder = [2 ** k for k in range(10, 19, 2)]
    out = {}
    for name, make in (("slab", W.slab_regions), ("duct", W.duct)):
        rows = []
        for ns in ns_list:
            base = make(n_s=ns, si_norm=1, si_tol=1e-6)

            def run(n, points, seed, **kw):
                p = dict(base)
                p.update(n_particles=int(n), points=points, seed=int(seed), **kw)
                s = S.Solver(p, torch_allocator=False)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.advance(1, allow_not_converged=True)
                f = s.get_flux(0)
                t = time.perf_counter() - t0
                it = s.get_stats()["si_iterations"]
                s.destroy()
                return f, t, it

            ref, _, it_ref = run(2 ** 22, 0, 7777)
            _, _, it_coll = run(2 ** 16, 0, 7777, si_norm=0)
            nref = max(np.linalg.norm(ref), 1e-300)
            row = {"n_s": ns, "particles": ladder, "si_iterations": it_ref,
                   "si_iterations_collided_test": it_coll}
            if ns >= 0 and min(np.min(base["sigma_a"] + base["sigma_s"]), 1.0) > 0.0:
                # the diffusion closing stage at 2^22 particles against the S_N
                # reference: the modelling error of the cheaper closure
                fd, td, itd = run(2 ** 22, 0, 7777, closure=1, si_tol=1e-12, si_max_iter=5000)
                row["diffusion"] = {"rel_l2_vs_sn_reference": float(np.linalg.norm(fd - ref) / nref),
                                    "cg_iterations": itd, "ms_per_solve": 1e3 * td}
            for pname, mode in (("qmc", 0), ("halton", 2), ("mc", 1)):
                errs, times = [], []
                for n in ladder:
                    e2, tt = 0.0, []
                    for r in range(args.protocol_seeds):
                        f, t, _ = run(n, mode, 1000 + 17 * r)
                        e2 += float(np.linalg.norm(f - ref) / nref) ** 2
                        tt.append(t)
                    errs.append((e2 / args.protocol_seeds) ** 0.5)
                    times.append(1e3 * float(np.median(tt)))
                slope = -float(np.polyfit(np.log(ladder), np.log(errs), 1)[0])
                row[pname] = {"rel_l2": errs, "alpha": slope, "ms_per_solve": times}
            log("steady protocol:", name, json.dumps(row))
            rows.append(row)
        out[name] = rows
    out["workloads"] = {
        "slab": "steady slab, 80 cells on [0,8] (regions: absorber with source sigma_a=20 Q=20; "
                "absorber sigma_a=3; void; scatterer sigma_s=0.8 sigma_a=0.2 Q=1; scatterer "
                "sigma_s=0.95 sigma_a=0.05), reflective at x=0 and in y, S_4, horizon 200",
        "duct": "steady bent duct, 30x50 cells on [0,3]x[0,5], duct sigma_s=sigma_a=1e-4, "
                "medium sigma_s=0.9 sigma_a=0.1, unit source in the duct's first 0.5x0.5, "
                "vacuum sides, S_4, horizon 200",
        "error": "relative L2 of phi_R against a 2^22-particle Sobol'-Owen run of the same "
                 "method, RMS over %d seeds" % args.protocol_seeds}
    return out


def closure_cmp(S, torch, args):
    """The closing stages on the benchmark workload (checkerboard 140x140, 1e6
    particles per pass): DG S_N source iteration, the same with diffusion
    synthetic acceleration, and the cell-centred diffusion solve (conjugate
    gradients), for several N_s: time per step, iterations of the last step,
    the collided stage's share of the step, and the relative L2 distance of
    the final phi_R from the plain S_N run (for the diffusion stage the
    modelling difference of the closures, not a parity figure); then plain
    and accelerated S_N on two scattering-dominated steady problems."""
    import numpy as np
    from paper_2511_16821_amd import workloads as W
    rows = []
    for ns in [int(v) for v in args.closure_ns.split(",") if v != ""]:
        row = {"n_s": ns}
        flux = {}
        for name, cl, acc in (("sn", 0, 0), ("sn_dsa", 0, 1), ("diffusion", 1, 0)):
            p = W.c2(n_s=ns, closure=cl, si_accel=acc)
            wall, st = timed_run(S, torch, p, args.closure_steps, 1)
            s = S.Solver(p)
            s.advance(args.closure_steps, allow_not_converged=True)
            flux[name] = s.get_flux(0)
            s.destroy()
            row[name] = {"ms_per_step": 1e3 * wall / args.closure_steps,
                         "iterations_last_step": int(st["si_iterations"]),
                         "ms_collided_last_step": float(st["ms_dg"])}
        row["rel_l2_diffusion_vs_sn"] = float(np.linalg.norm(flux["diffusion"] - flux["sn"]) /
                                              np.linalg.norm(flux["sn"]))
        row["rel_l2_sn_dsa_vs_sn"] = float(np.linalg.norm(flux["sn_dsa"] - flux["sn"]) /
                                           np.linalg.norm(flux["sn"]))
        log("closures:", json.dumps(row))
        rows.append(row)
    # scattering-dominated steady problems, where the acceleration matters
    steady = []
    for tag, p in (("duct N_s=0", W.duct(n_s=0, n_particles=65536)),
                   ("closed box N_s=0 (C1 box, all sides reflective)",
                    W.c1(n_s=0, steady=True, n_particles=65536, boundary=15, si_max_iter=2000))):
        row = {"problem": tag}
        for name, acc in (("sn", 0), ("sn_dsa", 1)):
            q = dict(p, si_accel=acc)
            wall, st = timed_run(S, torch, q, 1, 1)
            row[name] = {"ms_per_solve": 1e3 * wall, "sweeps": int(st["si_iterations"])}
        log("closures:", json.dumps(row))
        steady.append(row)
    large = None
    if args.closures_c5:
        # the large random-block solve, where the sweeps are expensive
        large = {"workload": "random blocks 1024x1024, 1e8 particles/pass, S_16, 5 steps"}
        for name, acc in (("sn", 0), ("sn_dsa", 1)):
            wall, st = timed_run(S, torch, W.c5(si_accel=acc), 5, 1)
            large[name] = {"ms_per_step": 1e3 * wall / 5, "sweeps_last_step": int(st["si_iterations"])}
        log("closures:", json.dumps(large))
    return {"workload": "checkerboard 140x140, 1e6 particles/pass, dt=0.05, S_12, %d steps"
                        % args.closure_steps, "rows": rows, "steady": steady, "large": large}


def serve_bench(S, torch, args):
    """Poisson arrivals of mixed solve requests; continuous batching on the
    server vs the same stream served one solve at a time on the same GPU
    (FIFO, no overlap: completion times from each request's measured service
    time alone).  The stream is drawn once (unit-rate arrival times scaled by
    mean service time / rho), so every rho serves the same requests."""
    import numpy as np
    from paper_2511_16821_amd import workloads as W
    sides = tuple(x for x in (32, 64, 128, 256, 512) if x <= args.serve_max_side)
    stream = W.request_stream(n_req=args.serve_requests, rho=1.0, seed=args.serve_seed,
                              sides=sides, np_range=(1e4, args.serve_max_particles))
    unit_arrivals = np.array([a for a, _ in stream])
    reqs = [p for _, p in stream]
    service, seg_alone, flux_alone = [], [], []
    for p in reqs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = S.Solver(p, torch_allocator=False)
        s.advance(int(p["n_steps"]), allow_not_converged=True)
        f = s.get_flux(0)
        st = s.get_stats()
        s.destroy()
        service.append(time.perf_counter() - t0)
        seg_alone.append(st["seg_mc_total"] + st["seg_remap_total"])
        flux_alone.append(f)
    service = np.array(service)
    t_mean = float(service.mean())
    log("serving: %d requests, serial service sum %.1f s" % (len(reqs), service.sum()))
    rows = []
    for rho in [float(v) for v in str(args.rho).split(",") if v != ""]:
        arrivals = unit_arrivals * t_mean / rho
        done, lat_serial = 0.0, []
        for a, t in zip(arrivals, service):
            done = max(a, done) + t
            lat_serial.append(done - a)
        serial_span = done - arrivals[0]
        budget = int(args.serve_budget_gib * (1 << 30))
        srv = S.Server(hbm_budget_bytes=budget, max_slots=args.serve_slots)
        t_start = time.perf_counter()
        tickets = []
        for a, p in zip(arrivals, reqs):
            wait = t_start + a - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            tickets.append(srv.submit(p, int(p["n_steps"])))
        res = [srv.result(t) for t in tickets]
        t_end = time.perf_counter()
        srv.destroy()
        lat = np.array([r[2]["latency_ms"] for r in res]) / 1e3
        seg = sum(r[2]["segments"] for r in res)
        same = all(np.array_equal(r[0], f) for r, f in zip(res, flux_alone))
        row = {"rho": rho,
               "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
               "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
               "segments_per_s": seg / (t_end - t_start),
               "one_at_a_time": {
                   "p50_latency_ms": float(np.percentile(lat_serial, 50) * 1e3),
                   "p99_latency_ms": float(np.percentile(lat_serial, 99) * 1e3),
                   "segments_per_s": float(sum(seg_alone) / serial_span)},
               "results_identical_to_alone": bool(same)}
        log("serving rho=%g:" % rho, json.dumps(row))
        rows.append(row)
    return {
        "requests": len(reqs), "slots": args.serve_slots, "budget_gib": args.serve_budget_gib,
        "mean_service_ms": 1e3 * t_mean, "rows": rows,
        "stream": "Poisson arrivals at rate rho/mean service time; sides %s, N_s in {0,1,2,4}, "
                  "particles log-uniform 1e4-%g, 5-50 steps, FP32/FP64 mixed, lognormal "
                  "8x8-block materials" % (list(sides), args.serve_max_particles),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the "
                    "workload's step count)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5",
                    help="c5 (default: the large resident solve), c2, c3, c1, c5_sub")
    ap.add_argument("--ns", type=int, default=None, help="N_s (default: the workload's)")
    ap.add_argument("--particles", type=int, default=None)
    ap.add_argument("--si-accel", type=int, default=None, choices=(0, 1),
                    help="collided solve: 0 plain source iteration, 1 with the diffusion "
                         "synthetic acceleration (default: 1 for c5, else the workload's)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-particles", type=int, default=2_000_000,
                    help="source particles of the oracle's bounded sample (per process)")
    ap.add_argument("--no-graph-run", action="store_true",
                    help="skip the timing of the one-graph-per-step production mode")
    ap.add_argument("--qmc-seeds", type=int, default=4,
                    help="Owen seeds (runs) for the QMC error of the headline workload")
    ap.add_argument("--no-c2", action="store_true", help="skip the checkerboard row")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving row")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the FP32-vs-FP64 precision form (256x256 thick medium)")
    ap.add_argument("--c3-ns", default="2")
    ap.add_argument("--c3-steps", type=int, default=20)
    ap.add_argument("--c3-seeds", type=int, default=4)
    ap.add_argument("--c3-particles", type=float, default=None)
    ap.add_argument("--protocol", action="store_true",
                    help="also run the paper's protocol: QMC vs MC convergence slopes and "
                         "source-iteration counts for several N_s")
    ap.add_argument("--protocol-ns", default="0,1,2,4,-1")
    ap.add_argument("--protocol-steps", type=int, default=10)
    ap.add_argument("--protocol-dt", type=float, default=0.1)
    ap.add_argument("--protocol-seeds", type=int, default=4)
    ap.add_argument("--steady", action="store_true",
                    help="the paper's steady-state protocol on the slab and duct stand-ins")
    ap.add_argument("--steady-ns", default="0,5,10,20,-1")
    ap.add_argument("--closures", action="store_true",
                    help="DG S_N against the diffusion closing stage on the benchmark workload")
    ap.add_argument("--closure-ns", default="0,1,2,4")
    ap.add_argument("--closure-steps", type=int, default=20)
    ap.add_argument("--closures-c5", action="store_true",
                    help="with --closures: also S_N with and without DSA on the 1024x1024 solve")
    ap.add_argument("--reflect", action="store_true",
                    help="reflective sides on the C1 box against vacuum")
    ap.add_argument("--reflect-steps", type=int, default=10)
    ap.add_argument("--nsx", action="store_true",
                    help="space-dependent N_s(x) on the C3 medium against uniform limits")
    ap.add_argument("--nsx-ns", default="0,1,2,4")
    ap.add_argument("--nsx-steps", type=int, default=10)
    ap.add_argument("--nsx-particles", type=float, default=2e6)
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the serving row (the full stream: 256)")
    ap.add_argument("--serve-max-side", type=int, default=256,
                    help="largest mesh side of the serving row (the full stream: 512)")
    ap.add_argument("--serve-max-particles", type=float, default=1e6,
                    help="largest particle count of the serving row (the full stream: 1e7)")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-seed", type=int, default=4)
    ap.add_argument("--rho", default="1.0", help="comma-separated loads, e.g. 0.5,1,2")
    ap.add_argument("--direct", action="store_true",
                    help="launch every kernel directly instead of as graphs (for counter "
                         "collection, which instruments each dispatch)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    global DIRECT
    DIRECT = args.direct
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no inter-GPU sharding); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20)
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "launches": 5}))
        return
    from paper_2511_16821_amd import slh as S
    S.lib()

    import numpy as np
    p64 = make_problem(args, 0)
    steps = args.steps or int(p64["n_steps"])
    profile = PROFILES.get(args.workload, "")
    log("workload:", describe(p64), "steps", steps)
    wall, st, s64 = timed_run(S, torch, p64, steps, args.warmup, timing=True, keep=True)
    seg = st["seg_mc_total"] + st["seg_remap_total"]
    value = seg / wall
    dom, both = rooflines(st, steps, 0, profile)
    log("fp64: %.3f s, %.3e segments/s, kernel ms mc %.1f remap %.1f" %
        (wall, value, st["ms_kernel_mc_total"], st["ms_kernel_remap_total"]))
    out = {
        "metric": METRIC, "value": value, "unit": "segments/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES.get(args.workload, args.workload) + ": " +
                   describe(p64), "n_steps": steps, "precision": "fp64",
                   "points": "sobol-owen", "timing": "MC-pass kernels between HIP events, "
                   "the rest of each step as graphs; no host wait inside a step",
                   "collided_solve": "DG S_N, source iteration" + (
                       " with diffusion synthetic acceleration" if p64.get("si_accel") else "")},
        "roofline": dom, "roofline_kernels": both, "segments": int(seg),
        "si_iterations_last_step": st["si_iterations"],
    }
    if not args.no_graph_run:
        wall_g, st_g = timed_run(S, torch, p64, steps, 0, timing=False)
        seg_g = st_g["seg_mc_total"] + st_g["seg_remap_total"]
        out["one_graph_per_step"] = {"value": seg_g / wall_g, "unit": "segments/s",
                                     "ms_per_step": 1e3 * wall_g / steps,
                                     "graph_launches": st_g["graph_launches_total"]}
        log("one graph per step: %.3e segments/s, %.2f ms/step" % (seg_g / wall_g,
                                                                  1e3 * wall_g / steps))
        if p64.get("si_accel"):  # the same steps with the plain source iteration
            p0 = dict(p64, si_accel=0)
            n0 = min(steps, 10)
            wall_0, st_0 = timed_run(S, torch, p0, n0, 0, timing=False)
            out["plain_source_iteration"] = {
                "value": (st_0["seg_mc_total"] + st_0["seg_remap_total"]) / wall_0,
                "unit": "segments/s", "ms_per_step": 1e3 * wall_0 / n0, "steps": n0,
                "si_iterations_last_step": st_0["si_iterations"]}
            log("plain source iteration: %.2f ms/step, %d iterations" %
                (1e3 * wall_0 / n0, st_0["si_iterations"]))
    x64 = s64.get_flux(0)
    s64.destroy()
    if not args.no_fp32:
        p32 = make_problem(args, 1)
        wall32, st32, s32 = timed_run(S, torch, p32, steps, args.warmup, timing=True, keep=True)
        seg32 = st32["seg_mc_total"] + st32["seg_remap_total"]
        x32 = s32.get_flux(0)
        s32.destroy()
        err = float(np.linalg.norm(x32 - x64) / max(np.linalg.norm(x64), 1e-300))
        runs = [x64]
        for r in range(args.qmc_seeds - 1):
            sr = S.Solver(dict(p64, seed=int(p64["seed"]) + 1000003 * (r + 1)))
            sr.advance(steps)
            sr.synchronize(allow_not_converged=True)
            runs.append(sr.get_flux(0))
            sr.destroy()
            log("qmc error: seed run %d done" % (r + 1))
        runs = np.stack(runs)
        e_qmc = float(np.linalg.norm(runs.std(axis=0, ddof=1)) /
                      max(np.linalg.norm(runs.mean(axis=0)), 1e-300))
        dom32, both32 = rooflines(st32, steps, 1, profile)
        out["fp32_track"] = {"value": seg32 / wall32, "unit": "segments/s",
                             "ms_per_step": 1e3 * wall32 / steps,
                             "speedup_vs_fp64": (seg32 / wall32) / value,
                             "rel_l2_vs_fp64_last_step": err,
                             "e_qmc_last_step": e_qmc, "e_qmc_seeds": args.qmc_seeds,
                             "fp32_within_bound": bool(err < min(1e-4, e_qmc)),
                             "roofline": dom32, "roofline_kernels": both32}
        log("fp32-track: %.3f s, %.3e segments/s, rel-L2 vs fp64 %.2e, e_qmc %.2e" %
            (wall32, seg32 / wall32, err, e_qmc))
    if not args.no_c3:
        out["precision_form"] = precision_form(S, torch, args)
    if not args.no_c2:
        pc2 = W_c2()
        w2, st2 = timed_run(S, torch, pc2, int(pc2["n_steps"]), 2, timing=True)
        seg2 = st2["seg_mc_total"] + st2["seg_remap_total"]
        dom2, both2 = rooflines(st2, int(pc2["n_steps"]), 0, PROFILES["c2"])
        out["checkerboard"] = {"workload": WORKLOAD_NAMES["c2"] + ": " + describe(pc2),
                               "value": seg2 / w2, "unit": "segments/s",
                               "ms_per_step": 1e3 * w2 / int(pc2["n_steps"]),
                               "roofline": dom2, "roofline_kernels": both2}
        log("checkerboard: %.3e segments/s, %.2f ms/step" % (seg2 / w2,
                                                            1e3 * w2 / int(pc2["n_steps"])))
    if args.protocol:
        out["protocol"] = protocol(S, torch, args)
    if args.steady:
        out["steady_protocol"] = steady_protocol(S, torch, args)
    if args.closures:
        out["closures"] = closure_cmp(S, torch, args)
    if args.nsx:
        out["cellwise_ns"] = cellwise_ns(S, torch, args)
    if args.reflect:
        out["reflective"] = reflective(S, torch, args)
    if not args.no_serve:
        out["serving"] = serve_bench(S, torch, args)
        log("serving:", json.dumps(out["serving"]))
    if not args.no_cpu:
        workers = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(p64, args.cpu_particles, workers)
        log("cpu oracle: %.3e segments/s on %d cores" % (out["cpu_baseline"]["value"], workers))
    print(json.dumps(out), flush=True)


def W_c2():
    from paper_2511_16821_amd import workloads as W
    return W.c2(n_s=2)


if __name__ == "__main__":
    main()
