"""Benchmark of the EFE residual-Chebyshev hot path on one MI355X.

One step = one pass of the hot path over the 64-atom cluster workload
(16^3 cells, p = 6, 160 vectors, Chebyshev degree 40):
  rebuild of the potential-dependent operators (cell Hamiltonians, B, H^phiphi),
  Lanczos spectrum bound, residual Chebyshev filter, Rayleigh-Ritz.
The headline value is the filter throughput in DoF * vector * degree / s with
DoF = interior CFE nodes + enrichment rows, averaged over the timed steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c64] [--no-cpu]

Prints one JSON line (rank 0, N = 1 only: this build runs on one GPU).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "hbm": 8.0e12}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(w, seconds_cap=60.0):
    """The oracle's H^E apply on the same workload with a bounded number of
    vectors (one Chebyshev degree step is one H apply), timed after setup."""
    from oracle import enrich, fe, psp
    from paper_2607_06848_amd import workloads as wl
    t0 = time.perf_counter()
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    s = enrich.EFESystem(mesh, w)
    X = mesh.quad_coords()
    vq = np.zeros(X.shape[:2])
    for R in np.asarray(w["xyz"]):
        vq += psp.v_local(np.linalg.norm(X - R, axis=-1), w["Z"], w["loc_rc"], w["loc_amp"],
                          w["loc_rg"])
    s.set_potential(vq)
    t_setup = time.perf_counter() - t0
    nvec = 8
    V = wl.random_block(s.rows, nvec, 5)
    t0 = time.perf_counter()
    s.apply_H(V)
    t = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    n_dof = len(s.active())
    return {"value": n_dof * nvec / t, "unit": "DoF*vec*deg/s", "cores": cores, "kind": "oracle",
            "sample": f"one H^E apply (= one Chebyshev degree step) of {nvec} of the "
                      f"{w['nvec']} vectors on the full {w['name']} mesh, FP64 NumPy/SciPy, "
                      f"setup {t_setup:.1f} s excluded, apply {t:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c64")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path shards by "
              "vector columns, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_06848_amd import efe
    from paper_2607_06848_amd import workloads as wl

    w = wl.make(args.workload)
    N, deg = w["nvec"], w["degree"]
    log("workload", args.workload, "N", N, "degree", deg)
    t0 = time.perf_counter()
    ctx = efe.Context(w)
    vq = ctx.local_potential()
    ctx.set_potential(vq)
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t0:.2f} s rows {ctx.rows} dof {ctx.n_dof} "
        f"enr {ctx.n_enr} cells {ctx.n_cells}")
    V = torch.from_numpy(wl.random_block(ctx.rows, N, w["v0_seed"])).cuda()
    v0 = torch.from_numpy(wl.random_vector(ctx.rows, 7)).cuda()
    lam, res = ctx.rayleigh_ritz(V)
    stream = torch.cuda.current_stream()

    def step(timed):
        ctx.set_potential(vq)                       # per-SCF operator rebuild
        b = ctx.spectrum_upper_bound(v0, 20)        # spectrum bound
        l = lam_box[0].cpu().numpy()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.cheb_filter(V, lam_box[0], deg, float(l[-1]), b, float(l[0]))
        e1.record(stream)
        lam_box[0], res_box[0] = ctx.rayleigh_ritz(V)
        return e0, e1

    lam_box, res_box = [lam], [res]
    for i in range(args.warmup):
        step(False)
        log("warmup step", i, "done")
    torch.cuda.synchronize()
    ctx.timing(True)
    ev = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev.append(step(True))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    filt_ms = [a.elapsed_time(b) for a, b in ev]
    ncell_l, cell_ms = ctx.timing_get("cell")
    napp, app_ms = ctx.timing_get("apply")
    nrr, rr_ms = ctx.timing_get("rr")
    nrec, rec_ms = ctx.timing_get("recur")
    ctx.timing(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    filt_s = np.mean(filt_ms) * 1e-3
    value = ctx.n_dof * N * deg / filt_s
    log(f"step {ms_step:.1f} ms, filter {np.mean(filt_ms):.1f} ms, applies {napp} "
        f"({app_ms / max(napp, 1):.3f} ms avg), cell launches {ncell_l} "
        f"({cell_ms / max(ncell_l, 1):.3f} ms avg), RR {rr_ms / max(nrr, 1):.1f} ms, "
        f"recurrence {rec_ms / max(nrec, 1):.3f} ms avg")
    # roofline of the dominant kernel: one colour pass of the FP64 cell GEMM
    cells_per_launch = ctx.n_cells / 8.0
    flops_per_launch = 2.0 * ctx.nloc ** 2 * N * cells_per_launch
    avg_cell_s = cell_ms * 1e-3 / max(ncell_l, 1)
    achieved = flops_per_launch / avg_cell_s
    out = {
        "metric": "Cheb-filter DoF*vec*deg/s",
        "value": value,
        "unit": "DoF*vec*deg/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w['name']}: {len(w['xyz'])}-atom jittered cubic Gaussian-"
                               f"pseudopotential cluster, {w['ncell'][0]}^3 cells p={w['p']}, "
                               f"N={N} vectors, Chebyshev degree {deg}, residual filter FP64",
                   "n_dof": ctx.n_dof, "rows": ctx.rows, "filter_ms": float(np.mean(filt_ms)),
                   "rr_ms": rr_ms / max(nrr, 1), "h_apply_ms": app_ms / max(napp, 1),
                   "recurrence_ms": rec_ms / max(nrec, 1)},
        "roofline": {"bound": "mfma", "kernel": "k_cell_f64 (one colour pass of the cell GEMM)",
                     "achieved": achieved / 1e12, "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK["fp64"], "traffic": None,
                     "launch_ms": avg_cell_s * 1e3, "flops_per_launch": flops_per_launch},
    }
    ctx.close()
    if not args.no_cpu:
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
