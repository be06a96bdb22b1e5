"""Benchmark of the EFE residual-Chebyshev hot path on one MI355X.

Default workload: the 500-atom cluster (30^3 cells, p = 6, 5.93e6 rows,
5,739,839 DoF, N = 1200 vectors, Chebyshev degree 50).  One step = one
residual Chebyshev filter pass (efe_cheb_filter: G = H V - M V Lambda, 49
recurrence applies of M~^-1 H, V_out) of degree 50 over one 160-column chunk
of the block, the width the filter processes at a time; a pass over the whole
1200-vector block is 7.5 such chunks back to back (the filter acts on every
column on its own).  The chunk is the seeded start block after one
Rayleigh-Ritz (its Ritz values and a Lanczos bound set the filter interval);
each step filters a fresh copy of it.

Headline value: DoF * vector * degree / s over the timed steps (DoF =
interior CFE nodes + enrichment rows), whole-job wall time of the K steps.
Also reported: the roofline of the dominant kernel (the cell GEMM colour
pass, timed with HIP events on the library stream), per-kernel times, and
the CPU oracle on a bounded sample (extrapolated to the full apply).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp64|fp32|bf16]
                    [--workload c500|c64] [--no-cpu]
    python bench.py --scf-only --workload c500 ...   time-to-SCF runs
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
STEP_TIMERS = ("t_filter_ms", "t_rr_ms", "t_poisson_ms", "t_density_ms", "t_operators_ms",
               "t_bound_ms", "t_energy_ms", "t_other_ms")
COL_CHUNK = 160   # column chunk of the filter and of one cell GEMM launch
CELL_KERNEL = {"fp64": "k_cell3<double, 1, 10, true>", "fp32": "k_cell3<float, 2, 10, true>",
               "bf16": "k_cell_bf16<32>"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summary (rocprofv3 FETCH_SIZE and WRITE_SIZE runs, each scaled by
    the same counter's reading for a 1 GiB device copy), or None when the
    summary is missing or was taken from a different source of the kernel."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"cell_gemm_{workload}_traffic.json")
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
    """The oracle's H^E apply (one Chebyshev degree step) of 8 vectors, on a
    bounded sample, extrapolated to the whole workload.  The oracle's apply
    is the CFE cell sums (two per apply: H X^C and H C^T X^E, every cell)
    plus the sparse enrichment and projector products (per atom).  Timed:
    the cell sums over a block of cells, and the sparse products of the atoms
    within 9 bohr of the corner atom; scaled by cells and atoms.  One BLAS
    thread (the sparse products are single-threaded anyway)."""
    from threadpoolctl import threadpool_limits
    from oracle import enrich, fe, psp
    from paper_2607_06848_amd import workloads as wl
    nvec = 8
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
        ic = wl.corner_atom(w)
        sub, keep = wl.subcluster(w, np.asarray(w["xyz"])[ic], 9.0)
        s = enrich.EFESystem(mesh, sub)
        cells = np.arange(min(mesh.n_cells, 400))
        X = mesh.quad_coords()
        vq = np.zeros(X.shape[:2])
        for R in np.asarray(sub["xyz"]):
            vq += psp.v_local(np.linalg.norm(X - R, axis=-1), w["Z"], w["loc_rc"],
                              w["loc_amp"], w["loc_rg"])
        s.set_potential(vq)
        V = wl.random_block(s.rows, nvec, 5)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        mesh.cfe_apply(vq, V[:s.n_nodes], cells=cells)
        t_cells = time.perf_counter() - t0
        t0 = time.perf_counter()
        s.apply_H(V, cells=np.zeros(0, np.int64))
        t_sparse = time.perf_counter() - t0
    t_full = 2 * t_cells * mesh.n_cells / len(cells) + t_sparse * len(w["xyz"]) / len(keep)
    n_dof = int(len(mesh.interior) + len(w["xyz"]) * s.nf)
    return {"value": n_dof * nvec / t_full, "unit": "DoF*vec*deg/s", "cores": 1, "kind": "oracle",
            "extrapolated": True,
            "sample": f"oracle H^E apply of {nvec} vectors on the {w['name']} mesh, FP64 "
                      f"NumPy/SciPy on one thread: CFE cell sums over {len(cells)} of "
                      f"{mesh.n_cells} cells ({t_cells:.2f} s, x2 per apply), sparse enrichment "
                      f"and projector products of {len(keep)} of {len(w['xyz'])} atoms "
                      f"({t_sparse:.2f} s); extrapolated apply {t_full:.1f} s; setup "
                      f"{t_setup:.1f} s excluded"}


def profile_applies(w, prec, k):
    """A short program for hardware-counter runs: K H^E applies of one column
    chunk of the workload's block (its first min(N, 160) columns: the width
    one cell-GEMM launch takes) under the local pseudopotential, then one
    plain device copy of 1 GiB."""
    import torch
    from paper_2607_06848_amd import efe
    from paper_2607_06848_amd import workloads as wl
    ctx = efe.Context(w)
    vq = ctx.local_potential()
    ctx.set_potential(vq, precisions=(1 << efe.EFE_FP32) | (1 << efe.EFE_BF16))
    N = min(w["nvec"], COL_CHUNK)
    X = torch.empty(ctx.rows, N, dtype=torch.float64, device="cuda")
    for r0, blk in wl.random_block_rows(ctx.rows, N, w["v0_seed"], 1 << 18):
        X[r0:r0 + len(blk)].copy_(torch.from_numpy(blk))
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
        hist = efe.scf_run(ctx, V, lam, v0, deg, tol=args.scf_tol, rho_tol=args.scf_tol,
                           max_iter=args.max_scf_steps,
                           prec=prec_k, passes_first=args.passes_first, passes=1,
                           tau=args.tau, max_passes=args.max_passes, kerker_k0=args.kerker,
                           mix_beta=args.mix_beta, mix_history=args.mix_history,
                           progress=on_pass,
                           log=lambda i, r: log(f" {name} step {i}: E {r['E']:.8f} "
                                                f"dE {r['dE']:.2e} drho {r['drho']:.2e} "
                                                f"passes {r['passes']} max occ res "
                                                f"{r['max_occ_res']:.2e} "
                                                f"at {time.perf_counter() - t0:.1f} s; ms: "
                                                + " ".join(f"{k[2:-3]} {r[k]:.0f}" for k in
                                                           STEP_TIMERS)))
        torch.cuda.synchronize()
        t_scf = time.perf_counter() - t0
        ctx.close()
        # the next run allocates its own block: free this one first
        del V, lam, v0
        torch.cuda.empty_cache()
        res[name] = {"seconds": t_scf, "steps": len(hist),
                     "filter_passes": sum(h["passes"] for h in hist), "E_Ha": hist[-1]["E"],
                     "converged": len(hist) > 1
                     and abs(hist[-1]["dE"]) / len(w["xyz"]) < args.scf_tol
                     and hist[-1]["drho"] / hist[-1]["n_el"] < args.scf_tol,
                     "last_dE_per_atom": abs(hist[-1]["dE"]) / len(w["xyz"]),
                     "last_drho_per_electron": hist[-1]["drho"] / hist[-1]["n_el"],
                     "guess": "learned" if mdl is not None and not fb else "superposition",
                     "filter_precision": "fp64" if prec_k == 0 else "fp32",
                     "max_occ_res": [h["max_occ_res"] for h in hist],
                     "E_per_step": [h["E"] for h in hist],
                     "tau": args.tau, "kerker_k0": args.kerker, "scf_tol": args.scf_tol,
                     "mix_beta": args.mix_beta, "mix_history": args.mix_history}
        log(f"SCF {name}: {len(hist)} steps, {t_scf:.1f} s, E {hist[-1]['E']:.8f}")
    for other in ("fp32_learned", "fp64_learned", "fp32_sad"):
        if other in res and "fp64_sad" in res:
            a, b = res["fp64_sad"], res[other]
            res[f"speedup_{other}"] = a["seconds"] / b["seconds"]
            res[f"dE_per_atom_{other}"] = abs(a["E_Ha"] - b["E_Ha"]) / len(w["xyz"])
    res["tol_Ha_per_atom"] = 1e-5
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp64", choices=sorted(PREC))
    ap.add_argument("--workload", default="c500")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--scf-runs", default="fp64_sad,fp32_learned",
                    help="time-to-SCF runs, comma separated <fp64|fp32>_<sad|learned>")
    ap.add_argument("--profile-applies", type=int, default=0, metavar="K",
                    help="profiling mode: set up the workload with its local pseudopotential, "
                         "run K H^E applies of one 160-column chunk in --prec, copy a 1 GiB buffer "
                         "once (a plain copy of known size for counter calibration), print "
                         "timings and exit without the JSON line")
    ap.add_argument("--prec-error", action="store_true",
                    help="one SCF step (Rayleigh-Ritz + first-step passes) in FP64 and in FP32 "
                         "from the same start; print the eigenvalue, density and energy "
                         "differences as one JSON line and exit")
    ap.add_argument("--tau", type=float, default=1e-3,
                    help="time-to-SCF runs: filter passes continue while the largest occupied "
                         "residual exceeds tau")
    ap.add_argument("--max-passes", type=int, default=12,
                    help="time-to-SCF runs: cap of the filter passes per SCF step")
    ap.add_argument("--passes-first", type=int, default=4,
                    help="time-to-SCF runs: minimum passes of the first SCF step")
    ap.add_argument("--kerker", type=float, default=0.0,
                    help="time-to-SCF runs: Kerker k0 of the mixing (0: plain Anderson)")
    ap.add_argument("--mix-beta", type=float, default=0.3,
                    help="time-to-SCF runs: Anderson mixing parameter")
    ap.add_argument("--mix-history", type=int, default=8,
                    help="time-to-SCF runs: Anderson history depth")
    ap.add_argument("--scf-tol", type=float, default=1e-5,
                    help="time-to-SCF runs: stop when |dE| per atom and the density change "
                         "per electron are both below this")
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

    def on_pass(i, tf, tr):
        log(f"  pass {i}: filter {tf:.0f} ms, Rayleigh-Ritz {tr:.0f} ms")

    if args.scf_only:
        print(json.dumps({"workload": w["name"], "natoms": len(w["xyz"]), "vectors": N,
                          "degree": deg, "time_to_scf": time_to_scf(args, w, new_run, on_pass)}),
              flush=True)
        return
    print(json.dumps(filter_bench(args, w)), flush=True)


def filter_bench(args, w):
    """The timed filter passes over one column chunk (the headline)."""
    import torch
    from paper_2607_06848_amd import efe
    from paper_2607_06848_amd import workloads as wl
    deg = w["degree"]
    prec = PREC[args.prec]
    n = min(w["nvec"], COL_CHUNK)
    t0 = time.perf_counter()
    ctx = efe.Context(w)
    ctx.set_potential(ctx.local_potential(), 0 if prec == 0 else (1 << prec))
    V0 = torch.empty(ctx.rows, n, dtype=torch.float64, device="cuda")
    for r0, blk in wl.random_block_rows(ctx.rows, n, w["v0_seed"], 1 << 18):
        V0[r0:r0 + len(blk)].copy_(torch.from_numpy(blk))
    lam, _ = ctx.rayleigh_ritz(V0)
    b = ctx.spectrum_upper_bound(torch.from_numpy(wl.random_vector(ctx.rows, 7)).cuda(), 20)
    lh = lam.cpu().numpy()
    V = torch.empty_like(V0)
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t0:.1f} s: rows {ctx.rows} dof {ctx.n_dof} enr "
        f"{ctx.n_enr} cells {ctx.n_cells}; Ritz values [{lh[0]:.4f}, {lh[-1]:.4f}], bound {b:.2f}")

    def step():
        V.copy_(V0)
        ctx.cheb_filter(V, lam, deg, lh[-1], b, lh[0], prec=prec)

    for i in range(args.warmup):
        ta = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i}: {1e3 * (time.perf_counter() - ta):.0f} ms")
    ctx.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        if i % 5 == 4:
            torch.cuda.synchronize()
            log(f"step {i + 1} of {args.steps} at {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timers = {k: ctx.timing_get(k) for k in ("cell", "pre", "post", "recur", "apply")}
    names = {"cell": "cell GEMM colour pass", "pre": "projector pass + Y^C start values",
             "post": "enrichment rows", "recur": "recurrence step (fused apply)",
             "apply": "plain H apply (G)"}
    ctx.timing(False)
    amp = ctx.amplification()
    ncp, maxe = ctx.coupling()
    ctx.close()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = ctx.n_dof * n * deg * args.steps / (t1 - t0)
    kernels = {names[k]: {"launches": c, "ms_avg": ms / max(c, 1), "ms_per_step": ms / args.steps}
               for k, (c, ms) in timers.items()}
    log(f"step {ms_step:.1f} ms; " + ", ".join(f"{k} {v['ms_avg']:.3f} ms x {v['launches']}"
                                              for k, v in kernels.items()))
    # roofline of the cell GEMM colour pass: one launch multiplies one
    # colour's cells (n_cells / 8 on average) into the chunk's columns: the
    # cell Hamiltonians (2 nloc^2 per cell and vector) and the coupling blocks
    # E_c and E_c^T (4 nf nloc per coupling pair and vector)
    ncell_l, cell_ms = timers["cell"]
    nf = ctx.n_enr // max(ctx.natoms, 1)
    flops_per_launch = (2.0 * ctx.nloc ** 2 * ctx.n_cells + 4.0 * nf * ctx.nloc * ncp) * n / 8.0
    avg_cell_s = cell_ms * 1e-3 / max(ncell_l, 1)
    achieved = flops_per_launch / avg_cell_s
    peak = PEAK[args.prec]
    full_pass_s = (t1 - t0) / args.steps * w["nvec"] / n
    return {
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
                               f"{w['nvec']} vectors, Chebyshev degree {deg}; one step = one "
                               f"residual filter pass over a {n}-column chunk",
                   "n_dof": ctx.n_dof, "rows": ctx.rows, "vectors_per_step": n,
                   "filter_precision": args.prec, "enrichment_amplification": amp,
                   "coupling_pairs": ncp, "max_enrichment_per_cell": maxe,
                   "full_block_pass_s": full_pass_s,
                   "full_block_pass_rule": f"{w['nvec']} / {n} chunk passes back to back",
                   "kernels": kernels},
        "roofline": {"bound": "mfma", "kernel": CELL_KERNEL[args.prec] + " (one colour pass)",
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(CELL_KERNEL[args.prec], w["name"]),
                     "launch_ms": avg_cell_s * 1e3, "flops_per_launch": flops_per_launch,
                     "share_of_step": cell_ms / ((t1 - t0) * 1e3)},
        **({} if args.no_cpu else {"cpu_baseline": _cpu(w)}),
    }


def _cpu(w):
    log("timing the oracle on a bounded sample")
    return cpu_baseline(w)


if __name__ == "__main__":
    main()
