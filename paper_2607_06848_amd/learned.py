"""Learned initial SCF density: training data, training driver and guess.

A small MLP proposes the initial SCF density as a correction to the
superposition of atomic densities (SAD), from rotation-invariant descriptors
of the 16 nearest atoms at every Gauss point.  Everything numeric runs in
the library's kernels (efe_descriptors, efe_mlp_forward, efe_mlp_loss_grad,
efe_mlp_backward, efe_mlp_adam, efe_density_guess); this module only
arranges the data:

  generate  converged SCF densities of perturbed 64-atom clusters, sampled
            at Gauss points (half uniform, half where the SAD density is
            above 1e-4), with importance weights that make the sampled loss
            an unbiased estimate of the quadrature-weighted loss;
  train     Adam on the quadrature-weighted squared error of the predicted
            correction against rho_* - rho_SAD;
  Model     the trained parameters with the input standardization and the
            target scale, saved as .npz.

The converged SCF decides the answer: the guess changes where the SCF
starts, never where it ends.

    python -m paper_2607_06848_amd.learned generate --seeds 100:118 --out DIR
    python -m paper_2607_06848_amd.learned train --data DIR --out model.npz
"""
import argparse
import glob
import json
import os
import time

import numpy as np

N_IN = 25          # 8 radial Gaussians x l = 0..2 power spectrum + log rho_SAD
HIDDEN = 128
N_PARAMS = HIDDEN * N_IN + HIDDEN + 2 * (HIDDEN * HIDDEN + HIDDEN) + HIDDEN + 1
DENSE = 1e-4       # SAD density above which half of the samples are drawn


def _log(*a):
    print("[learned]", *a, flush=True)


def perturbed_c64(seed, sigma=0.3):
    """The 64-atom cluster with every atom moved by N(0, sigma^2) per axis."""
    from . import workloads as wl
    w = wl.make("c64")
    w["xyz"] = wl.perturb(np.asarray(w["xyz"]), sigma, seed)
    w["name"] = f"c64-perturbed-{seed}"
    return w


def sample_points(rho_sad, n, seed):
    """Mixture sample (with replacement) of Gauss-point indices: half uniform
    over all points, half uniform over points with rho_SAD > DENSE.  Returns
    the indices and 1 / (n p(q)), the factor that turns the quadrature weight
    into the weight of an unbiased sampled sum."""
    rng = np.random.default_rng(seed)
    nq = len(rho_sad)
    dense = np.flatnonzero(rho_sad > DENSE)
    if not len(dense):
        return rng.integers(0, nq, n), np.full(n, nq / n)
    uniform = rng.random(n) < 0.5
    idx = np.where(uniform, rng.integers(0, nq, n), dense[rng.integers(0, len(dense), n)])
    p = 0.5 / nq + (0.5 / len(dense)) * (rho_sad[idx] > DENSE)
    return idx.astype(np.int64), 1.0 / (n * p)


def generate(seeds, out, nsamp=32768, prec=1, tol=1e-5, max_iter=60):
    import torch
    from . import efe
    from . import workloads as wl
    os.makedirs(out, exist_ok=True)
    for seed in seeds:
        t0 = time.perf_counter()
        w = perturbed_c64(seed)
        ctx = efe.Context(w)
        N = w["nvec"]
        V = torch.from_numpy(wl.random_block(ctx.rows, N, w["v0_seed"])).cuda()
        lam = torch.zeros(N, dtype=torch.float64, device="cuda")
        v0 = torch.from_numpy(wl.random_vector(ctx.rows, 7)).cuda()
        hist = efe.scf_run(ctx, V, lam, v0, w["degree"], tol=tol, max_iter=max_iter, prec=prec)
        rho_star = ctx.get_density(1)
        rho_sad = ctx.get_density(2)
        _, wq = ctx.quadrature()
        drho = (rho_star - rho_sad).cpu().numpy()
        sad = rho_sad.cpu().numpy()
        wq = wq.cpu().numpy()
        ctx.close()
        idx, fac = sample_points(sad, nsamp, seed)
        conv = len(hist) < max_iter
        np.savez_compressed(os.path.join(out, f"geom_{seed}.npz"), xyz=np.asarray(w["xyz"]),
                            idx=idx.astype(np.int32), w=(wq[idx] * fac).astype(np.float32),
                            rho_sad=sad[idx].astype(np.float32),
                            drho=drho[idx].astype(np.float32), steps=len(hist),
                            E=hist[-1]["E"], converged=conv)
        _log(f"seed {seed}: {len(hist)} SCF steps, E {hist[-1]['E']:.8f}, converged {conv}, "
             f"{time.perf_counter() - t0:.1f} s")
        del V, lam, v0
        torch.cuda.empty_cache()


class Model:
    """Trained density network: flat FP32 parameters, the feature
    standardization (shift, scale) and the target scale s_t."""

    def __init__(self, params, shift, scale, target_scale, meta=None):
        self.params = np.asarray(params, np.float32)
        self.shift = np.asarray(shift, np.float32)
        self.scale = np.asarray(scale, np.float32)
        self.target_scale = float(target_scale)
        self.meta = meta or {}

    @property
    def norm(self):
        return np.concatenate([self.shift, self.scale, [self.target_scale]]).astype(np.float32)

    def save(self, path):
        np.savez(path, params=self.params, shift=self.shift, scale=self.scale,
                 target_scale=self.target_scale, meta=json.dumps(self.meta))

    @classmethod
    def load(cls, path):
        z = np.load(path, allow_pickle=False)
        return cls(z["params"], z["shift"], z["scale"], float(z["target_scale"]),
                   json.loads(str(z["meta"])))

    def apply(self, ctx):
        """Set ctx's next input density to the learned guess; returns
        (used_fallback, factor)."""
        import torch
        p = torch.from_numpy(self.params).cuda()
        return ctx.density_guess(p, self.norm)


def init_params(seed):
    """W, b ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) per layer (FP32)."""
    rng = np.random.default_rng(seed)
    out = []
    for fan_out, fan_in in ((HIDDEN, N_IN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (1, HIDDEN)):
        b = 1.0 / np.sqrt(fan_in)
        out.append(rng.uniform(-b, b, size=fan_out * fan_in))
        out.append(rng.uniform(-b, b, size=fan_out))
    return np.concatenate(out).astype(np.float32)


def _load_samples(files, xq):
    """Device inputs of the descriptor kernel (points, atoms, SAD density),
    targets and per-geometry normalized weights of every file's samples;
    xq holds the mesh's Gauss points on the host."""
    import torch
    feats, drho, wts = [], [], []
    for f in files:
        z = np.load(f, allow_pickle=False)
        pts = torch.from_numpy(np.ascontiguousarray(xq[z["idx"].astype(np.int64)])).cuda()
        sad = torch.from_numpy(z["rho_sad"].astype(np.float64)).cuda()
        xyz = torch.from_numpy(np.ascontiguousarray(z["xyz"], np.float64)).cuda()
        feats.append((pts, xyz, sad))
        drho.append(z["drho"].astype(np.float64))
        w = z["w"].astype(np.float64)
        wts.append(w / w.sum())
    return feats, drho, wts


def train(data_dir, out, epochs=30, batch=65536, lr=1e-3, n_val=2, seed=6, shuffle_seed=7):
    import torch
    from . import efe
    files = sorted(glob.glob(os.path.join(data_dir, "geom_*.npz")),
                   key=lambda f: int(f.rsplit("_", 1)[1].split(".")[0]))
    if len(files) <= n_val:
        raise RuntimeError(f"need more than {n_val} geometries in {data_dir}")
    t0 = time.perf_counter()
    ctx = efe.Context(perturbed_c64(0))          # the mesh's Gauss points
    xq = ctx.quadrature()[0].cpu().numpy()
    ctx.close()
    geo, drho, wts = _load_samples(files, xq)
    # standardization from the raw training features
    F = np.concatenate([efe.efe_descriptors(p, x, s).cpu().numpy()
                        for (p, x, s) in geo[:-n_val]]).astype(np.float64)
    shift_h = F.mean(0).astype(np.float32)
    scale_h = (F.std(0) + 1e-6).astype(np.float32)
    del F
    shift = torch.from_numpy(shift_h).cuda()
    scale = torch.from_numpy(scale_h).cuda()
    dtr = np.concatenate(drho[:-n_val])
    wtr = np.concatenate(wts[:-n_val])
    s_t = float(np.sqrt(np.sum(wtr * dtr ** 2) / np.sum(wtr)))

    def stack(sel):
        X = torch.cat([efe.efe_descriptors(p, x, s, shift, scale) for (p, x, s) in sel])
        return X

    Xtr = stack(geo[:-n_val]).cpu().numpy()
    Xva = stack(geo[-n_val:])
    ttr = (dtr / s_t).astype(np.float32)
    tva_h = (np.concatenate(drho[-n_val:]) / s_t).astype(np.float32)
    wva_h = np.concatenate(wts[-n_val:]).astype(np.float32)
    sad_only = float(np.sum(wva_h * tva_h.astype(np.float64) ** 2) / np.sum(wva_h))
    tva = torch.from_numpy(tva_h).cuda()
    wva = torch.from_numpy(wva_h).cuda()
    wtr = wtr.astype(np.float32)
    n = len(ttr)
    _log(f"{len(files) - n_val} training geometries ({n} points), {n_val} validation; "
         f"target scale {s_t:.3e}; setup {time.perf_counter() - t0:.1f} s")
    P = torch.from_numpy(init_params(seed)).cuda()
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    nb = min(batch, n)
    acts = torch.empty(3 * nb * HIDDEN, dtype=torch.float32, device="cuda")
    work = torch.empty(2 * nb * HIDDEN, dtype=torch.float32, device="cuda")
    grads = torch.empty_like(P)
    rng = np.random.default_rng(shuffle_seed)
    step, hist = 0, []
    for ep in range(epochs):
        perm = rng.permutation(n)
        Xe = torch.from_numpy(Xtr[perm]).cuda()
        te = torch.from_numpy(ttr[perm]).cuda()
        we = torch.from_numpy(wtr[perm]).cuda()
        tl, tw = 0.0, 0.0
        for b0 in range(0, n - nb + 1, nb):
            X, t, w = Xe[b0:b0 + nb], te[b0:b0 + nb], we[b0:b0 + nb]
            y = efe.efe_mlp_forward(P, X, acts)
            dy, sums = efe.efe_mlp_loss_grad(y, t, w)
            efe.efe_mlp_backward(P, X, acts, dy, grads, work)
            step += 1
            efe.efe_mlp_adam(P, grads, m, v, step, lr)
            s = sums.cpu().numpy()
            tl += s[1]
            tw += s[0]
        yv = efe.efe_mlp_forward(P, Xva)
        _, sv = efe.efe_mlp_loss_grad(yv, tva, wva)
        sv = sv.cpu().numpy()
        hist.append((tl / tw, sv[1] / sv[0]))
        _log(f"epoch {ep}: train {tl / tw:.4e} validation {sv[1] / sv[0]:.4e} "
             f"(SAD alone: {sad_only:.4e})")
    seeds = [int(f.rsplit("_", 1)[1].split(".")[0]) for f in files]
    model = Model(P.cpu().numpy(), shift_h, scale_h, s_t,
                  dict(train_seeds=seeds[:-n_val], val_seeds=seeds[-n_val:], epochs=epochs,
                       batch=nb, lr=lr, init_seed=seed, shuffle_seed=shuffle_seed,
                       loss_history=hist, points=n, train_seconds=time.perf_counter() - t0))
    model.save(out)
    _log(f"saved {out} after {time.perf_counter() - t0:.1f} s")
    return model


def compare(model_path, seeds, prec=1, tol=1e-5, max_iter=60):
    """SCF from the superposition guess and from the learned guess on the
    given perturbed geometries; returns per-geometry steps, times, energies."""
    import torch
    from . import efe
    from . import workloads as wl
    model = Model.load(model_path)
    rows = []
    for seed in seeds:
        w = perturbed_c64(seed)
        rec = {"seed": seed}
        for guess in ("sad", "learned"):
            ctx = efe.Context(w)
            N = w["nvec"]
            V = torch.from_numpy(wl.random_block(ctx.rows, N, w["v0_seed"])).cuda()
            lam = torch.zeros(N, dtype=torch.float64, device="cuda")
            v0 = torch.from_numpy(wl.random_vector(ctx.rows, 7)).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fb, fac = model.apply(ctx) if guess == "learned" else ctx.density_guess(None)
            hist = efe.scf_run(ctx, V, lam, v0, w["degree"], tol=tol, max_iter=max_iter,
                               prec=prec)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            passes = sum(h["passes"] for h in hist)
            rec[guess] = dict(steps=len(hist), passes=passes, seconds=dt, E=hist[-1]["E"],
                              fallback=fb, factor=fac,
                              drho0=hist[0]["drho"])
            _log(f"seed {seed} {guess}: {len(hist)} steps, {passes} filter passes, "
                 f"{dt:.1f} s, E {hist[-1]['E']:.8f}, fallback {fb}, factor {fac:.4f}, "
                 f"first-step density residual {hist[0]['drho']:.3e}")
            ctx.close()
            del V, lam, v0
            torch.cuda.empty_cache()
        rows.append(rec)
    return rows


def _seeds(s):
    if ":" in s:
        a, b = s.split(":")
        return list(range(int(a), int(b)))
    return [int(x) for x in s.split(",")]


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--seeds", required=True)
    g.add_argument("--out", required=True)
    g.add_argument("--nsamp", type=int, default=32768)
    g.add_argument("--prec", type=int, default=1)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=30)
    t.add_argument("--batch", type=int, default=65536)
    t.add_argument("--lr", type=float, default=1e-3)
    c = sub.add_parser("compare")
    c.add_argument("--model", required=True)
    c.add_argument("--seeds", required=True)
    c.add_argument("--prec", type=int, default=1)
    c.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "generate":
        generate(_seeds(a.seeds), a.out, a.nsamp, a.prec)
    elif a.cmd == "train":
        train(a.data, a.out, a.epochs, a.batch, a.lr)
    else:
        rows = compare(a.model, _seeds(a.seeds), a.prec)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
