"""Benchmark of the EFE residual-Chebyshev hot path on one MI355X.

One step = one SCF step over the 64-atom cluster workload (16^3 cells, p = 6,
160 vectors, Chebyshev degree 40): Poisson solve for the electrostatic
remainder, effective potential, rebuild of the cell Hamiltonians and
enrichment blocks, Lanczos spectrum bound, residual Chebyshev filter,
Rayleigh-Ritz, Fermi level, density, energies, Anderson mixing.

Headline value: filter throughput in DoF * vector * degree / s over the timed
steps (DoF = interior CFE nodes + enrichment rows; filter time measured
around efe_cheb_filter inside the step).  Also reported: ms per SCF step,
time to SCF convergence at 1e-5 Ha/atom in FP64 from the superposition guess
and with FP32 cell GEMMs from the learned initial density, the
roofline of the dominant kernel (one colour pass of the cell GEMM, timed with
HIP events on the library stream) and the CPU oracle on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp64|fp32|bf16]
                    [--workload c64] [--no-cpu] [--no-scf]
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
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
COL_CHUNK = 160   # column chunk of the filter and of one cell GEMM launch
CELL_KERNEL = {"fp64": "k_cell2<double, 1, 10>", "fp32": "k_cell2<float, 1, 10>",
               "bf16": "k_cell_bf16<32>"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (rocprofv3 FETCH_SIZE and WRITE_SIZE runs, each scaled by the same
    counter's reading for a 1 GiB device copy), or None when the summary is
    missing or was taken from a different source of the cell GEMM."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "cell_gemm_c64_traffic.json")
    src = os.path.join(ROOT, "paper_2607_06848_amd", "csrc", "apply.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    k = rec.get("kernels", {}).get(kernel)
    if k is None or rec.get("apply_hip_sha256") != sha:
        return None
    return k["read_bytes"] + k["write_bytes"]


def cpu_baseline(w):
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


def profile_applies(w, prec, k):
    """A short program for hardware-counter runs: K H^E applies of the
    workload's block under the local pseudopotential, then one plain device
    copy of 1 GiB."""
    import torch
    from paper_2607_06848_amd import efe
    from paper_2607_06848_amd import workloads as wl
    ctx = efe.Context(w)
    vq = ctx.local_potential()
    ctx.set_potential(vq, precisions=(1 << efe.EFE_FP32) | (1 << efe.EFE_BF16))
    N = w["nvec"]
    X = torch.from_numpy(wl.random_block(ctx.rows, N, w["v0_seed"])).cuda()
    Y = torch.empty_like(X)
    torch.cuda.synchronize()
    ctx.timing(True)
    for _ in range(k):
        ctx.apply_H_prec(X, prec, Y)
    n, ms = ctx.timing_get("cell")
    na, msa = ctx.timing_get("apply")
    ctx.timing(False)
    log(f"{k} applies: cell launches {n} ({ms / max(n, 1):.3f} ms avg), "
        f"apply {msa / max(na, 1):.3f} ms avg")
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log("copied 1 GiB (read 1 GiB, write 1 GiB)")
    ctx.close()


def precision_error(w):
    """Differences between one FP64 and one FP32 SCF step from the same
    start (superposition density, seeded block): occupied eigenvalues, the
    output density (relative L2 over the Gauss points) and the energy."""
    import torch
    from paper_2607_06848_amd import efe
    from paper_2607_06848_amd import workloads as wl
    N, deg = w["nvec"], w["degree"]
    out = {}
    for name, p in (("fp64", PREC["fp64"]), ("fp32", PREC["fp32"])):
        ctx = efe.Context(w)
        V = torch.empty(ctx.rows, N, dtype=torch.float64, device="cuda")
        for r0, blk in wl.random_block_rows(ctx.rows, N, w["v0_seed"], 1 << 18):
            V[r0:r0 + len(blk)].copy_(torch.from_numpy(blk))
        lam = torch.zeros(N, dtype=torch.float64, device="cuda")
        v0 = torch.from_numpy(wl.random_vector(ctx.rows, 7)).cuda()
        t0 = time.perf_counter()
        rep = ctx.scf_step(V, lam, v0, deg, prec=p, passes_first=4, passes=1,
                           progress=lambda i, tf, tr: log(f"  {name} pass {i}: filter {tf:.0f} ms"))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _, wq = ctx.quadrature()
        out[name] = dict(E=rep["E"], lam=lam.cpu().numpy(), rho=ctx.get_density(1).cpu().numpy(),
                         wq=wq.cpu().numpy(), seconds=dt)
        log(f"{name}: step {dt:.1f} s, E {rep['E']:.8f}")
        ctx.close()
        del V
        torch.cuda.empty_cache()
    a, b = out["fp64"], out["fp32"]
    ne = int(round(float(np.sum(w["Zs"])))) // 2
    wq = a["wq"]
    drho = np.sqrt(np.sum(wq * (b["rho"] - a["rho"]) ** 2) / np.sum(wq * a["rho"] ** 2))
    print(json.dumps({"workload": w["name"], "natoms": len(w["xyz"]), "vectors": N,
                      "step": "first SCF step: Rayleigh-Ritz of the seeded block + 4 passes",
                      "seconds": {"fp64": a["seconds"], "fp32": b["seconds"]},
                      "occupied_eigenvalue_max_abs_diff_Ha": float(
                          np.abs(b["lam"][:ne] - a["lam"][:ne]).max()),
                      "density_rel_L2_diff": float(drho),
                      "energy_diff_Ha_per_atom": abs(b["E"] - a["E"]) / len(w["xyz"])}),
          flush=True)


def time_to_scf(args, w, new_run, on_pass):
    """The time-to-SCF runs named by --scf-runs, each from its own fresh
    context and seeded start block; returns the time_to_scf record."""
    import torch
    from paper_2607_06848_amd import efe
    deg = w["degree"]
    from paper_2607_06848_amd import learned
    model = learned.Model.load(args.model) if os.path.exists(args.model) else None
    runs = []
    for name in args.scf_runs.split(","):
        p, g = name.split("_")
        if g == "learned" and model is None:
            log(f"no density model at {args.model}: skipping {name}")
            continue
        runs.append((name, PREC[p], model if g == "learned" else None))
    res = {}
    for name, prec_k, mdl in runs:
        log(f"time to SCF: {name}")
        ctx, V, lam, v0 = new_run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fb, fac = mdl.apply(ctx) if mdl is not None else ctx.density_guess(None)
        hist = efe.scf_run(ctx, V, lam, v0, deg, tol=1e-5, max_iter=args.max_scf_steps,
                           prec=prec_k,
                           passes_first=4, passes=1, progress=on_pass,
                           log=lambda i, r: log(f" {name} step {i}: E {r['E']:.8f} "
                                                f"dE {r['dE']:.2e} drho {r['drho']:.2e} "
                                                f"at {time.perf_counter() - t0:.1f} s"))
        torch.cuda.synchronize()
        t_scf = time.perf_counter() - t0
        ctx.close()
        res[name] = {"seconds": t_scf, "steps": len(hist),
                     "filter_passes": sum(h["passes"] for h in hist), "E_Ha": hist[-1]["E"],
                     "converged": len(hist) > 1 and abs(hist[-1]["dE"]) / len(w["xyz"]) < 1e-5
                     and hist[-1]["drho"] / hist[-1]["n_el"] < 1e-5,
                     "last_dE_per_atom": abs(hist[-1]["dE"]) / len(w["xyz"]),
                     "last_drho_per_electron": hist[-1]["drho"] / hist[-1]["n_el"],
                     "guess": "learned" if mdl is not None and not fb else "superposition",
                     "filter_precision": "fp64" if prec_k == 0 else "fp32"}
        log(f"SCF {name}: {len(hist)} steps, {t_scf:.1f} s, E {hist[-1]['E']:.8f}")
    if "fp32_learned" in res and "fp64_sad" in res:
        a, b = res["fp64_sad"], res["fp32_learned"]
        res["speedup"] = a["seconds"] / b["seconds"]
        res["dE_per_atom"] = abs(a["E_Ha"] - b["E_Ha"]) / len(w["xyz"])
    res["tol_Ha_per_atom"] = 1e-5
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp64", choices=sorted(PREC))
    ap.add_argument("--workload", default="c64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-scf", action="store_true", help="skip the time-to-SCF runs")
    ap.add_argument("--scf-runs", default="fp64_sad,fp32_learned",
                    help="time-to-SCF runs, comma separated <fp64|fp32>_<sad|learned>")
    ap.add_argument("--profile-applies", type=int, default=0, metavar="K",
                    help="profiling mode: set up the workload with its local pseudopotential, "
                         "run K H^E applies of the N-vector block in --prec, copy a 1 GiB buffer "
                         "once (a plain copy of known size for counter calibration), print "
                         "timings and exit without the JSON line")
    ap.add_argument("--prec-error", action="store_true",
                    help="one SCF step (Rayleigh-Ritz + first-step passes) in FP64 and in FP32 "
                         "from the same start; print the eigenvalue, density and energy "
                         "differences as one JSON line and exit")
    ap.add_argument("--max-scf-steps", type=int, default=60,
                    help="step cap of each time-to-SCF run (a capped run reports converged: false)")
    ap.add_argument("--scf-only", action="store_true",
                    help="only the time-to-SCF runs: one JSON line with time_to_scf and no "
                         "timed steps")
    ap.add_argument("--model", default=os.path.join(ROOT, "paper_2607_06848_amd", "weights",
                                                    "density_c64.npz"),
                    help="trained initial-density network for the mixed + learned SCF run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the path is measured on "
              "one GPU; it would shard over GPUs by vector columns", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_06848_amd import efe
    from paper_2607_06848_amd import workloads as wl

    w = wl.make(args.workload)
    N, deg = w["nvec"], w["degree"]
    prec = PREC[args.prec]
    log("workload", args.workload, "N", N, "degree", deg, "filter precision", args.prec)
    if args.profile_applies:
        profile_applies(w, prec, args.profile_applies)
        return
    if args.prec_error:
        precision_error(w)
        return

    def new_run():
        ctx = efe.Context(w)
        V = torch.empty(ctx.rows, N, dtype=torch.float64, device="cuda")
        for r0, blk in wl.random_block_rows(ctx.rows, N, w["v0_seed"], 1 << 18):
            V[r0:r0 + len(blk)].copy_(torch.from_numpy(blk))
        lam = torch.zeros(N, dtype=torch.float64, device="cuda")
        v0 = torch.from_numpy(wl.random_vector(ctx.rows, 7)).cuda()
        return ctx, V, lam, v0

    t0 = time.perf_counter()
    ctx, V, lam, v0 = new_run()
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t0:.2f} s rows {ctx.rows} dof {ctx.n_dof} "
        f"enr {ctx.n_enr} cells {ctx.n_cells}")
    def on_pass(i, tf, tr):
        log(f"  pass {i}: filter {tf:.0f} ms, Rayleigh-Ritz {tr:.0f} ms")

    if args.scf_only:
        ctx.close()
        del V
        torch.cuda.empty_cache()
        print(json.dumps({"workload": w["name"], "natoms": len(w["xyz"]), "vectors": N,
                          "degree": deg, "time_to_scf": time_to_scf(args, w, new_run, on_pass)}),
              flush=True)
        return

    kw = dict(prec=prec, passes_first=4, passes=1, progress=on_pass)
    for i in range(args.warmup):
        r = ctx.scf_step(V, lam, v0, deg, **kw)
        log(f"warmup step {i}: E {r['E']:.8f} dE {r['dE']:.2e} filter {r['t_filter_ms']:.0f} ms")
    torch.cuda.synchronize()
    ctx.timing(True)
    reps = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        reps.append(ctx.scf_step(V, lam, v0, deg, **kw))
        log(f"step {i}: E {reps[-1]['E']:.8f} dE {reps[-1]['dE']:.2e} CG iterations "
            f"{reps[-1]['cg_iters']}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ncell_l, cell_ms = ctx.timing_get("cell")
    napp, app_ms = ctx.timing_get("apply")
    nrr, rr_ms = ctx.timing_get("rr")
    nrec, rec_ms = ctx.timing_get("recur")
    ctx.timing(False)
    ctx.close()
    ms_step = (t1 - t0) * 1e3 / args.steps
    filt_ms = sum(r["t_filter_ms"] for r in reps)
    npass = sum(r["passes"] for r in reps)
    value = ctx.n_dof * N * deg * npass / (filt_ms * 1e-3)
    log(f"step {ms_step:.1f} ms, filter {filt_ms / npass:.1f} ms/pass, applies {napp} "
        f"({app_ms / max(napp, 1):.3f} ms avg), cell launches {ncell_l} "
        f"({cell_ms / max(ncell_l, 1):.3f} ms avg), RR {rr_ms / max(nrr, 1):.1f} ms, "
        f"recurrence {rec_ms / max(nrec, 1):.3f} ms avg")
    breakdown = {k: float(np.mean([r[k] for r in reps])) for k in
                 ("t_poisson_ms", "t_operators_ms", "t_bound_ms", "t_filter_ms", "t_rr_ms",
                  "t_density_ms", "t_energy_ms", "t_other_ms")}
    # roofline of the dominant kernel: one colour pass of the cell GEMM
    # one launch multiplies one colour's cells into one column chunk of at
    # most 160 vectors (wider blocks run chunk by chunk)
    cells_per_launch = ctx.n_cells / 8.0
    flops_per_launch = 2.0 * ctx.nloc ** 2 * min(N, COL_CHUNK) * cells_per_launch
    avg_cell_s = cell_ms * 1e-3 / max(ncell_l, 1)
    achieved = flops_per_launch / avg_cell_s
    peak = PEAK[args.prec]
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
        "dtype": {"fp64": "f64", "fp32": "f32 cell GEMM / f64", "bf16": "bf16 cell GEMM / f64"}[
            args.prec],
        "data": "synthetic",
        "config": {"workload": f"{w['name']}: {len(w['xyz'])}-atom jittered cubic Gaussian-"
                               f"pseudopotential cluster, {w['ncell'][0]}^3 cells p={w['p']}, "
                               f"N={N} vectors, Chebyshev degree {deg}, residual filter, "
                               f"one SCF step per step",
                   "n_dof": ctx.n_dof, "rows": ctx.rows, "filter_precision": args.prec,
                   "filter_ms_per_pass": filt_ms / npass, "rr_ms": rr_ms / max(nrr, 1),
                   "h_apply_ms": app_ms / max(napp, 1),
                   "recurrence_ms": rec_ms / max(nrec, 1), "step_breakdown_ms": breakdown},
        "roofline": {"bound": "mfma", "kernel": CELL_KERNEL[args.prec] + " (one colour pass)",
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(CELL_KERNEL[args.prec]),
                     "launch_ms": avg_cell_s * 1e3, "flops_per_launch": flops_per_launch},
    }
    if not args.no_scf:
        out["time_to_scf"] = time_to_scf(args, w, new_run, on_pass)
    if not args.no_cpu:
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
