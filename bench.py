#!/usr/bin/env python3
"""Benchmark of the superblock projection + Davidson hot path on one MI355X.

Workload: the two-site Hubbard superblock with m = 2048 states per block
(t = 1, U = 4, U(1)xU(1) sectors, 241 sectors, target-sector dimension
n = 37 668, 12 terms), seeded synthetic operators.

One step = one pass of the whole hot path on that input, inputs resident in
HBM: a ground-state solve by the device Davidson iteration with the
projection in reduced precision (FP32 by default) and FP64 refinement to a
residual of 1e-10 (energy within 1e-8 of the FP64 result), replayed from
captured hipGraphs, followed by the energy gradient dE/dc_k through the
adjoint kernel.  `value` = Davidson iterations per second over the timed
steps.  The projection alone is also timed (HIP events, FP64/FP32/BF16) and
reported in TFLOP/s, and the FP64-only solve is timed for comparison.

Beside the headline line (unless --no-extras): time to solution in mixed
precision and in FP64 from the same start vector at two residual tolerances,
with the energy error against an FP64 solve at 1e-12; plan creation plus the
first solve on a fresh plan; compact projection and solve figures of the
Heisenberg m=1024 superblock and the 64-member batch; block Davidson-Liu for
the four lowest states; and the l-1-1-r strategy on a Hubbard superblock of two
512-state blocks and two sites.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "f64_TFs": 78.6, "f32_TFs": 157.3, "bf16_TFs": 2500.0}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="f32", choices=["f32", "bf16"], help="reduced precision of phase 1")
    ap.add_argument("--proj-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-renorm", action="store_true",
                    help="skip the eigen-decomposition / selection timing and the infinite-lattice run "
                         "reported beside the solve")
    ap.add_argument("--quick", action="store_true", help="skip the projection and FP64 comparison timings")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the time-to-solution table, the fresh-plan solve and the other workloads "
                         "(block Davidson-Liu, l-1-1-r, Heisenberg m=1024, the 64-member batch)")
    ap.add_argument("--workload", default="hubbard_m2048",
                    choices=["hubbard_m2048", "heisenberg_m1024", "j1j2_m1024", "batched_64", "gemv", "pmc",
                             "pmc_heisenberg", "infinite_heisenberg", "block_projection"],
                    help="hubbard_m2048 is the headline line; the others time the projection and the "
                         "mixed-precision solve of the other synthetic workloads")
    return ap.parse_args()


def timed_projection(plan, psi, y, prec, reps, torch):
    """Average duration of one projection call, HIP events on the launch stream."""
    s = torch.cuda.current_stream()
    for _ in range(5):
        plan.project_raw(psi, prec=prec, out=y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        plan.project_raw(psi, prec=prec, out=y)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def projection_stats(plan, psi, y, prec, torch, reps=200, flush=None):
    """Per-call durations of the projection (a HIP event pair around each call on the
    launch stream): median, p10, p90 in microseconds.  With `flush` (a device buffer),
    each call is preceded by a write of that buffer, which evicts L2 and the
    Infinity Cache (cold-cache variant)."""
    import numpy as np

    s = torch.cuda.current_stream()
    for _ in range(20):
        plan.project_raw(psi, prec=prec, out=y)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        if flush is not None:
            flush.fill_(1.0)
        a.record(s)
        plan.project_raw(psi, prec=prec, out=y)
        b.record(s)
    torch.cuda.synchronize()
    d = np.array([a.elapsed_time(b) * 1e3 for a, b in ev])
    return {"median_us": float(np.median(d)), "p10_us": float(np.percentile(d, 10)),
            "p90_us": float(np.percentile(d, 90))}


def density_stats(plan, psi, reps, torch):
    """Both blocks' reduced density matrices (Alg. 1, step 5) from psi: average
    duration of one call (HIP events on the launch stream) and its algorithmic
    work, a symmetric rank-K update per pair and side (d (d + 1) K FLOP, psi
    read once and both outputs written once)."""
    import numpy as np

    lo, ro = plan.density_layout()
    out = (torch.empty(int(lo[-1]), dtype=torch.float64, device=psi.device),
           torch.empty(int(ro[-1]), dtype=torch.float64, device=psi.device))
    lay = plan.layout()
    dl = np.sqrt(np.diff(lo)).round().astype(np.int64)
    dr = np.sqrt(np.diff(ro)).round().astype(np.int64)
    assert np.array_equal(dl * dr, np.diff(lay["pair_off"]))
    flop = int(np.sum(dl * (dl + 1) * dr + dr * (dr + 1) * dl))
    nbytes = 8 * int(plan.n + lo[-1] + ro[-1])
    s = torch.cuda.current_stream()
    for _ in range(5):
        plan.density(psi, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        plan.density(psi, out=out)
    e1.record(s)
    e1.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    return {"us": t * 1e6, "flop": flop, "bytes": nbytes, "tflops": flop / t * 1e-12, "GBs": nbytes / t * 1e-9}


def renorm_stats(plan, psi, torch, reps=10):
    """The rest of the renormalization step on the device (Alg. 1, steps 6-7)
    for the left block of the state psi (the ground state in the bench line):
    eigen-decomposition of every density-matrix block
    (dmrg_eigh_blocks) and the state selection (dmrg_truncate).  Per-call
    durations from HIP event pairs on the launch stream (the work copy of rho
    that each eigen-decomposition overwrites is refreshed outside the pair)."""
    import ctypes

    import numpy as np

    from paper_1309_5571_amd import _native as N

    lo, _ = plan.density_layout()
    rl, _ = plan.density(psi, right=False)
    dims = np.sqrt(np.diff(lo)).round().astype(np.int64)
    dev = psi.device
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    off, woff = t(lo[:-1].astype(np.int64)), t(np.concatenate([[0], np.cumsum(dims)[:-1]]).astype(np.int64))
    tdim = t(dims.astype(np.int32))
    work, u = torch.empty_like(rl), torch.empty_like(rl)
    w = torch.empty(int(dims.sum()), dtype=torch.float64, device=dev)
    # one group per member, each keeping a quarter of its states
    groups = np.bincount(plan.layout()["member"], minlength=len(plan.problems))
    gb = np.concatenate([[0], np.cumsum(groups)]).astype(np.int32)
    ms = np.array([max(1, int(dims[gb[g]:gb[g + 1]].sum()) // 4) for g in range(groups.size)], dtype=np.int32)
    gblk, tm = t(gb), t(ms)
    keep = torch.empty(dims.size, dtype=torch.int32, device=dev)
    disc = torch.empty(groups.size, dtype=torch.float64, device=dev)
    P = lambda x: ctypes.c_void_p(x.data_ptr())
    lib, s = N.lib(), torch.cuda.current_stream()
    te, tt = [], []
    for i in range(reps + 1):
        work.copy_(rl)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(s)
        N.check(lib.dmrg_eigh_blocks(int(dims.size), P(off), P(tdim), P(woff), P(work), P(w), P(u), None,
                                     ctypes.c_void_p(s.cuda_stream)))
        e[1].record(s)
        N.check(lib.dmrg_truncate(int(groups.size), P(gblk), P(tdim), P(woff), P(w), P(tm), P(keep), P(disc),
                                  ctypes.c_void_p(s.cuda_stream)))
        e[2].record(s)
        e[2].synchronize()
        if i:  # the first call is a warm-up
            te.append(e[0].elapsed_time(e[1]) * 1e3)
            tt.append(e[1].elapsed_time(e[2]) * 1e3)
    return {"blocks": int(dims.size), "max_block": int(dims.max()), "states": int(dims.sum()),
            "groups": int(groups.size), "m_keep": int(ms.sum()),
            "eigh_us": float(np.median(te)), "truncate_us": float(np.median(tt)),
            "discarded": float(disc.sum().cpu())}


def block_projection(p, reps, sizes=(1, 2, 4, 8, 16, 32)):
    """b vectors projected in one launch (a plan of b copies of the superblock,
    whose output tiles share one persistent grid): the throughput a block
    Davidson would see on a latency-bound workload.  FP64, HIP events on the
    launch stream, average over `reps` back-to-back calls."""
    import numpy as np
    import torch

    import paper_1309_5571_amd as dm

    rows = []
    for b in sizes:
        plan = dm.Plan([p] * b)
        x = torch.from_numpy(np.random.default_rng(b).standard_normal(plan.n)).cuda()
        y = torch.empty_like(x)
        t = timed_projection(plan, x, y, "f64", reps, torch)
        rows.append({"vectors": b, "us_per_call": t * 1e6, "us_per_vector": t * 1e6 / b,
                     "tflops": plan.flop / t * 1e-12, "GBs_algorithmic": plan.bytes / t * 1e-9})
        plan.close()
    return {"workload": "block_projection_hubbard_m2048", "rows": rows}


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def _solve_ms(plan, x0, prec, tol, reps, torch):
    """Warm solves of one plan from the same start vector: median wall time of
    dmrg_davidson (host clock around the call, stream drained on both sides),
    with the last call's energies and infos."""
    out = None
    for _ in range(2):
        plan.davidson(x0, tol=tol, prec=prec)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = plan.davidson(x0, tol=tol, prec=prec)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    _, E, info, st = out
    if st != 0:
        raise RuntimeError(f"Davidson status {st}: {info}")
    return _median(ts) * 1e3, E, info


def solve_comparison(plan, x0, prec, torch, tols=(1e-5, 1e-10), reps=5):
    """Time to solution, mixed precision against FP64, from the same start
    vector: for each residual tolerance, the warm solve time, the iterations, the
    host waits and the largest energy error against an FP64 solve at 1e-12.
    `time_to_1e-8` is, per precision, the fastest solve whose energies are all
    within 1e-8 of that reference."""
    import numpy as np

    _, Eref, _ = _solve_ms(plan, x0, "f64", 1e-12, 1, torch)
    rows = []
    best = {}
    for pr in (prec, "f64"):
        for tol in tols:
            ms, E, info = _solve_ms(plan, x0, pr, tol, reps, torch)
            dE = float(np.max(np.abs(np.asarray(E) - Eref)))
            rows.append({"prec": pr, "tol": tol, "ms": ms, "dE": dE,
                         "iterations": max(i["iterations"] for i in info),
                         "iterations_lowprec": max(i["iterations_low"] for i in info),
                         "host_waits": info[0]["host_waits"]})
            if dE <= 1e-8:
                best[pr] = min(best.get(pr, float("inf")), ms)
    return {"rows": rows, "time_to_1e-8_ms": best,
            "mixed_over_fp64": best[prec] / best["f64"] if prec in best and "f64" in best else None}


def fresh_plan_solve(p, x0_np, prec, torch, reps=3):
    """What every DMRG step pays: plan creation (operator upload, records, task
    lists, low-precision copies) and the first solve on that plan (workspace
    allocation and graph capture included), FP64 and mixed, to 1e-10.  Median of
    `reps` fresh plans, host clock with the stream drained."""
    import paper_1309_5571_amd as dm

    res = {}
    for pr in ("f64", prec):
        tp, ts = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = dm.Plan(p, prec=pr)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x0 = torch.from_numpy(x0_np).cuda()
            _, _, info, st = plan.davidson(x0, tol=1e-10, prec=pr)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if st != 0:
                raise RuntimeError(f"Davidson status {st}: {info}")
            plan.close()
            tp.append(t1 - t0)
            ts.append(t2 - t1)
        res[pr] = {"plan_ms": _median(tp) * 1e3, "first_solve_ms": _median(ts) * 1e3,
                   "total_ms": (_median(tp) + _median(ts)) * 1e3}
    return res


def config_summary(cfg, prec, torch, proj_reps=100, reps=3):
    """Compact figures of another workload: the projection per precision (µs,
    TFLOP/s and the fraction of that precision's dense MFMA peak) and the solve to
    1e-10 in mixed precision against FP64 (ms, iterations, host waits)."""
    import gen
    import paper_1309_5571_amd as dm

    p = gen.config(cfg)
    plan = dm.Plan(p, prec=prec)
    planb = dm.Plan(p, prec="bf16") if prec != "bf16" else plan
    x0 = torch.from_numpy(gen.start_vector(plan.n, 7)).cuda()
    psi = x0 / x0.norm()
    y = torch.empty_like(psi)
    peak = {"f64": PEAK["f64_TFs"], "f32": PEAK["f32_TFs"], "bf16": PEAK["bf16_TFs"]}
    proj = {}
    for pr, pl in (("f64", plan), (prec, plan), ("bf16", planb)):
        t = timed_projection(pl, psi, y, pr, proj_reps, torch)
        tf = plan.flop / t * 1e-12
        proj[pr] = {"us": t * 1e6, "tflops": tf, "frac_mfma_peak": tf / peak[pr]}
    solve = {}
    for pr in (prec, "f64"):
        ms, E, info = _solve_ms(plan, x0, pr, 1e-10, reps, torch)
        solve[pr] = {"ms": ms, "iterations": max(i["iterations"] for i in info),
                     "host_waits": info[0]["host_waits"], "energy0": float(E[0])}
    res = {"workload": gen.CONFIG_NAMES[cfg], "members": len(plan.problems), "n": plan.n, "flop": plan.flop,
           "projection": proj, "solve": solve,
           "mixed_over_fp64_solve": solve[prec]["ms"] / solve["f64"]["ms"]}
    if planb is not plan:
        planb.close()
    plan.close()
    return res


def block_summary(p, torch, b=4, reps=3, proj_reps=100):
    """Block Davidson-Liu on one superblock: the b lowest eigenpairs to 1e-10
    (median wall time, iterations, restarts) and the b-vector projection per
    vector against b single projections (HIP events on the launch stream)."""
    import numpy as np

    import gen
    import paper_1309_5571_amd as dm

    plan = dm.Plan(p)
    X0 = torch.from_numpy(np.stack([gen.start_vector(plan.n, 7 + j) for j in range(b)])).cuda()
    Y = torch.empty_like(X0)
    s = torch.cuda.current_stream()
    for _ in range(5):
        plan.project_block(X0, out=Y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(proj_reps):
        plan.project_block(X0, out=Y)
    e1.record(s)
    e1.synchronize()
    t_blk = e0.elapsed_time(e1) * 1e-3 / proj_reps
    t_one = timed_projection(plan, X0[0].contiguous(), Y[0], "f64", proj_reps, torch)
    out = None
    plan.block_davidson(X0, tol=1e-10)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = plan.block_davidson(X0, tol=1e-10)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    _, E, R, info, st = out
    _, E1, _, _ = plan.davidson(X0[0], tol=1e-10)
    plan.close()
    return {"nroots": b, "solve_ms": _median(ts) * 1e3, "status": st, "energies": [float(e) for e in E],
            "max_residual": float(np.max(R)), "iterations": info["iterations"], "restarts": info["restarts"],
            "projections": info["projections"], "E0_minus_single_vector": float(E[0] - E1[0]),
            "projection_us_per_vector": t_blk * 1e6 / b, "projection_us_single": t_one * 1e6}


def l11r_summary(torch, m=512, reps=3, proj_reps=100):
    """The l-1-1-r strategy (Eq. 12-13, Alg. 2) on the Hubbard superblock of
    two m-state blocks and two sites (the enlarged blocks have 4 m states, as
    the LR workload at m = 4 m): FP64 projection time and FLOP rate, and the
    FP64 ground-state solve to 1e-10."""
    import gen
    import paper_1309_5571_amd as dm

    p = gen.hubbard_l11r_synthetic(m)
    plan = dm.Plan(p)
    x0 = torch.from_numpy(gen.start_vector(plan.n, 7)).cuda()
    psi = x0 / x0.norm()
    y = torch.empty_like(psi)
    t = timed_projection(plan, psi, y, "f64", proj_reps, torch)
    ms, E, info = _solve_ms(plan, x0, "f64", 1e-10, reps, torch)
    res = {"workload": f"hubbard_l11r_m{m}", "n": plan.n, "records": plan.nrec, "flop": plan.flop,
           "algorithmic_bytes": plan.bytes, "projection_us": t * 1e6, "tflops": plan.flop / t * 1e-12,
           "solve_ms": ms, "iterations": info[0]["iterations"], "energy": float(E[0])}
    plan.close()
    return res


def infinite_workload(nsites=100, m=32, reps=3):
    """The whole infinite-lattice iteration (Alg. 1) grown from 4 to `nsites`
    sites of the Heisenberg chain keeping m states: wall time per growth step
    (median of `reps` runs after one warm-up) and the energy per site from the
    last two steps against Hulthen's 1/4 - ln 2."""
    import math

    import torch

    from paper_1309_5571_amd import infinite

    infinite.run(12, m=m)  # warm-up (library load, first kernels)
    times, res = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = infinite.run(nsites, m=m)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = sorted(times)[len(times) // 2]
    e = [r.energy for r in res]
    per_site = (e[-1] - e[-2]) / 2
    return {"workload": f"infinite_heisenberg_N{nsites}_m{m}", "steps": len(res), "seconds": t,
            "ms_per_step": t / len(res) * 1e3, "energy": e[-1], "energy_per_site": per_site,
            "hulthen": 0.25 - math.log(2.0), "max_discarded": max(r.discarded for r in res),
            "davidson_iterations": sum(r.iterations for r in res),
            "davidson_retries": sum(r.retries for r in res)}


def cpu_baseline(p, x0):
    """The FP64 oracle (NumPy + OpenBLAS) on the host: one full Davidson solve
    of the same workload from the same start vector, plus projection timing."""
    import numpy as np

    from oracle import davidson as odav
    from oracle import projection

    threads = int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    t0 = time.perf_counter()
    r = odav.ground_state_davidson(p, x0, tol=1e-10)
    t_dav = time.perf_counter() - t0
    flop = projection.flop_count(p)
    reps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 3.0:
        projection.project_sectors(p, x0)
        reps += 1
    t_proj = (time.perf_counter() - t0) / reps
    # the same on one host thread (BLAS limited to one thread for the oracle's products)
    one = None
    try:
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            r1 = odav.ground_state_davidson(p, x0, tol=1e-10)
            t_dav1 = time.perf_counter() - t0
            reps1 = 0
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < 2.0:
                projection.project_sectors(p, x0)
                reps1 += 1
            t_proj1 = (time.perf_counter() - t0) / reps1
        one = {"value": r1.iterations / t_dav1, "unit": "iter/s", "cores": 1, "solve_s": t_dav1,
               "projection_ms": t_proj1 * 1e3}
    except ImportError:
        pass
    return {
        "value": r.iterations / t_dav,
        "unit": "iter/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one FP64 oracle Davidson solve of the m=2048 Hubbard superblock to ||r|| <= 1e-10 "
                  f"({r.iterations} iterations, {t_dav:.2f} s) and {reps} oracle projections; the same "
                  f"solve and 2 s of projections again on one thread (one_thread)",
        "projection_ms": t_proj * 1e3,
        "projection_gflops": flop / t_proj * 1e-9,
        "energy": r.energy,
        "one_thread": one,
    }, r.energy


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


COPY_BYTES = 256 << 20  # calibration copy: reads and writes this many bytes


def pmc_workload(cfg=3):
    """Dispatches for the hardware counters (run under rocprofv3 --pmc): a plain
    device copy of COPY_BYTES (calibrates FETCH_SIZE / WRITE_SIZE), then 20
    projections of the workload in each precision, FP64 first, then FP32 and BF16
    (distinct kernel instantiations, so the counters separate by kernel name)."""
    import torch

    import gen
    import paper_1309_5571_amd as dm

    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    p = gen.config(cfg)
    plans = {"f32": dm.Plan(p, prec="f32"), "bf16": dm.Plan(p, prec="bf16")}
    plan = plans["f32"]
    psi = torch.from_numpy(gen.start_vector(plan.n, 7)).cuda()
    psi /= psi.norm()
    out = torch.empty_like(psi)
    for prec, pl in (("f64", plan), ("f32", plan), ("bf16", plans["bf16"])):
        for _ in range(20):
            pl.project_raw(psi, prec=prec, out=out)
        torch.cuda.synchronize()
    return {"workload": "pmc", "config": gen.CONFIG_NAMES[cfg], "copy_bytes": COPY_BYTES,
            "projections_per_precision": 20, "projection_algorithmic_bytes": plan.bytes,
            "projection_algorithmic_flop": plan.flop}


def traffic_from_profile(plan_bytes):
    """HBM bytes per projection from the committed counter summary, if it was
    taken on the current kernel sources (else None)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_projection_hubbard_m2048.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return rec.get("bytes_per_projection")


def gemv_sweep(reps=100):
    """The tall-skinny products of the orthogonalization (dmrg_gemv_t / _n) at the
    heights the paper sweeps (1e5, 5e5, 1e6) plus 4e6, widths 1..32, FP64.
    GB/s counts the algorithmic bytes: V (k columns) + x + s for V^T x, V + y for V s."""
    import torch

    import paper_1309_5571_amd as dm

    rows = []
    s = torch.cuda.current_stream()
    for n in (100_000, 500_000, 1_000_000, 4_000_000):
        V = torch.randn(32, n, dtype=torch.float64, device="cuda")
        x = torch.randn(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for k in (1, 2, 4, 8, 16, 20, 32):
            sv = dm.gemv_t(V, x, k)
            for name, fn, nbytes in (("gemv_t", lambda: dm.gemv_t(V, x, k), 8 * n * (k + 1)),
                                     ("gemv_n", lambda: dm.gemv_n(V, sv, y, 0.0, k), 8 * n * (k + 1))):
                for _ in range(5):
                    fn()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                for _ in range(reps):
                    fn()
                e1.record(s)
                e1.synchronize()
                t = e0.elapsed_time(e1) * 1e-3 / reps
                rows.append({"op": name, "n": n, "k": k, "us": t * 1e6, "GBs": nbytes / t * 1e-9,
                             "frac_hbm": nbytes / t * 1e-9 / PEAK["hbm_GBs"]})
        log(f"gemv n={n} done")
        del V, x, y
    return rows


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(the path is not sharded across GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import gen
    import paper_1309_5571_amd as dm

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.workload == "gemv":
        print(json.dumps({"workload": "gemv_sweep", "unit": "GB/s", "rows": gemv_sweep()}))
        return
    if args.workload in ("pmc", "pmc_heisenberg"):
        print(json.dumps(pmc_workload(3 if args.workload == "pmc" else 2)))
        return
    if args.workload == "infinite_heisenberg":
        print(json.dumps(infinite_workload()))
        return
    if args.workload == "block_projection":
        print(json.dumps(block_projection(gen.config(3), args.proj_reps)))
        return
    cfg = {"hubbard_m2048": 3, "heisenberg_m1024": 2, "j1j2_m1024": 5, "batched_64": 4}[args.workload]
    p = gen.config(cfg)
    plan = dm.Plan(p, prec=args.prec)
    x0_np = gen.start_vector(plan.n, 7)
    x0 = torch.from_numpy(x0_np).to(dev)
    coef = plan.coef.clone()
    nmem = len(plan.problems)

    def step(prec):
        psi, E, info, st = plan.davidson(x0, coef, tol=1e-10, prec=prec)
        if st != 0:
            raise RuntimeError(f"Davidson status {st}: {info}")
        _, gcoef = plan.backward_raw(psi, psi, coef, want_psi=False, want_coef=True)
        return E, info, gcoef

    log(f"plan ready: n={plan.n}, records={plan.nrec}, flop/projection={plan.flop}")
    for _ in range(args.warmup):
        step(args.prec)
    torch.cuda.synchronize()
    log("warmup done")
    iters = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        E, info, gcoef = step(args.prec)
        iters += sum(i["iterations"] for i in info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} steps: {dt / args.steps * 1e3:.3f} ms/step, {iters / dt:.1f} iter/s")
    E_mixed = float(E[0])

    extra = {}
    if not args.quick:
        # FP64-only solve of the same problem
        for _ in range(2):
            step("f64")
        torch.cuda.synchronize()
        it64 = 0
        t1 = time.perf_counter()
        n64 = max(3, args.steps // 2)
        for _ in range(n64):
            E64, info64, _ = step("f64")
            it64 += sum(i["iterations"] for i in info64)
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t1
        extra["fp64_solve"] = {"iters_per_s": it64 / dt64, "ms_per_solve": dt64 / n64 * 1e3,
                               "iterations": sum(i["iterations"] for i in info64) / nmem,
                               "energy": float(E64[0])}
        # projection alone, per precision (events on the launch stream)
        psi = torch.from_numpy(x0_np / np.linalg.norm(x0_np)).to(dev)
        y = torch.empty_like(psi)
        planb = dm.Plan(p, prec="bf16") if args.prec != "bf16" else plan
        proj = {}
        for prec, pl in (("f64", plan), (args.prec, plan), ("bf16", planb)):
            t = timed_projection(pl, psi, y, prec, args.proj_reps, torch)
            proj[prec] = {"us": t * 1e6, "tflops": plan.flop / t * 1e-12}
        extra["projection"] = proj
        log(f"projection: {proj}")
        flush = torch.empty(64 << 20, dtype=torch.float64, device=dev)  # 512 MiB
        stats = {}
        for prec, pl in (("f64", plan), (args.prec, plan), ("bf16", planb)):
            stats[prec] = {"warm": projection_stats(pl, psi, y, prec, torch),
                           "cold": projection_stats(pl, psi, y, prec, torch, reps=50, flush=flush)}
        del flush
        extra["projection_percall"] = stats
        log(f"projection per call: {stats}")
        extra["density"] = density_stats(plan, psi, args.proj_reps, torch)
        log(f"density matrices: {extra['density']}")
        if not args.no_renorm:
            # the density matrix of the ground state, as the renormalization step takes it
            psi_gs, _, _, st_gs = plan.davidson(x0, coef, tol=1e-10)
            if st_gs != 0:
                raise RuntimeError(f"Davidson status {st_gs}")
            extra["renormalization"] = renorm_stats(plan, psi_gs, torch)
            log(f"eigen-decomposition and selection: {extra['renormalization']}")
        if cfg == 3 and not args.no_renorm:  # the whole infinite-lattice iteration, Heisenberg chain to 100 sites
            extra["infinite_heisenberg"] = infinite_workload(reps=1)
            log(f"infinite-lattice DMRG: {extra['infinite_heisenberg']}")
        extra["mixed_vs_fp64_time_ratio"] = (dt / args.steps * 1e3) / extra["fp64_solve"]["ms_per_solve"]
    if not args.quick and not args.no_extras:
        extra["solve"] = solve_comparison(plan, x0, args.prec, torch)
        log(f"time to solution, mixed vs FP64: {extra['solve']}")
        extra["fresh_plan"] = fresh_plan_solve(p, x0_np, args.prec, torch)
        log(f"fresh plan + first solve: {extra['fresh_plan']}")
        if cfg == 3:
            extra["other_configs"] = [config_summary(c, args.prec, torch) for c in (2, 4)]
            log(f"other workloads: {extra['other_configs']}")
            extra["block_davidson"] = block_summary(p, torch)
            log(f"block Davidson-Liu: {extra['block_davidson']}")
            extra["l11r"] = l11r_summary(torch)
            log(f"l-1-1-r: {extra['l11r']}")

    # roofline of the dominant kernel: the FP64 projection, bound by HBM bytes at
    # this workload's arithmetic intensity (algorithmic FLOP / algorithmic bytes = 5)
    t_proj = extra["projection"]["f64"]["us"] * 1e-6 if "projection" in extra else None
    roof = None
    if t_proj:
        achieved = plan.bytes / t_proj * 1e-9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                "frac": achieved / PEAK["hbm_GBs"],
                "traffic": traffic_from_profile(plan.bytes) if cfg == 3 else None,
                "kernel": "projection (f64)", "algorithmic_bytes": plan.bytes, "algorithmic_flop": plan.flop}

    cpu = None
    E_ref = None
    if not args.no_cpu_baseline and nmem == 1:
        log("cpu baseline (oracle)")
        cpu, E_ref = cpu_baseline(p, x0_np)

    out = {
        "metric": ("H·ψ projection TFLOP/s + Davidson iters/s at m=2048 Hubbard; mixed vs FP64 @1e-8 dE"
                   if cfg == 3 else f"projection TFLOP/s + Davidson iters/s ({args.workload})"),
        "value": iters / dt,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.prec}+f64",
        "data": "synthetic",
        "config": ({"workload": "hubbard_m2048_two_site", "m": 2048, "n": plan.n, "sectors": int(p.left.nsec),
                    "terms": int(len(p.coef)), "t": 1.0, "U": 4.0, "tol": 1e-10,
                    "phase1": args.prec, "refine": "f64", "graph": True} if cfg == 3 else
                   {"workload": args.workload, "members": nmem, "n": plan.n, "tol": 1e-10,
                    "phase1": args.prec, "refine": "f64", "graph": True}),
        "iterations_per_step": sum(i["iterations"] for i in info) / nmem,
        "iterations_lowprec": sum(i["iterations_low"] for i in info) / nmem,
        "energy": E_mixed,
        "dE_vs_fp64_oracle": (E_mixed - E_ref) if E_ref is not None else None,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
