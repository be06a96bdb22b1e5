"""Oracle of the learned initial density (test infrastructure only).

Plain FP64 NumPy restatement of the learned-density guess: descriptors of
the 16 nearest atoms at a point, the 25 -> 128 -> 128 -> 128 -> 1 SiLU MLP,
its quadrature-weighted squared-error loss and gradient, one Adam step, and
the guess rho_0 = max(rho_SAD + dRho, 0) renormalized to the electron count
with the superposition of atomic densities as fallback.  The paper starts
its SCF from atomic densities and has no learned part; this component
follows the project's own definition, stated here:

  descriptors  For a point x, the 16 nearest atoms I (ties by the lower atom
               index), d_I = |x - R_I|, u_I = (x - R_I)/d_I; radial Gaussians
               g_n(d) = exp(-(d - n)^2 / 2), n = 0..7; real spherical
               harmonics Y_lm, l = 0..2; power spectrum
               P_nl = sum_m (sum_I g_n(d_I) Y_lm(u_I))^2, stored as feature
               3 n + l; feature 24 is log(max(rho_SAD, 1e-12)).  Features are
               standardized as (f - shift) / scale.
  MLP          h_k = silu(W_k h_{k-1} + b_k) for k = 1..3, y = W_4 h_3 + b_4;
               parameters in one flat array: W1 (128 x 25), b1, W2 (128 x 128),
               b2, W3, b3, W4 (1 x 128), b4 (1), row-major.
  loss         L = sum_q w_q (y_q - t_q)^2 / sum_q w_q, t = (rho_* - rho_SAD)/s_t.
  Adam         m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
               theta -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
  guess        rho_0 = max(rho_SAD + s_t y, 0) scaled by N_e / int rho_0;
               fall back to rho_SAD when a value is not finite or the
               scale factor leaves [0.9, 1.1].

Pins (tests/test_oracle_learned.py): the power spectrum equals its
Legendre addition-theorem form; rotation and atom-permutation invariance;
nearest-atom ties; a one-path network against silu(silu(silu(x)));
central-difference gradients of the loss; Adam's first step against
lr sign(g); renormalization and both fallbacks.
"""
import numpy as np

NRAD = 8
LMAX = 2
KNEAR = 16
N_IN = NRAD * (LMAX + 1) + 1
HIDDEN = 128
RHO_FLOOR = 1e-12


def nearest_atoms(x, xyz, k=KNEAR):
    """Indices (npts, min(k, natoms)) of the nearest atoms, ties broken by the
    lower index.  Squared distances are summed x, y, z in that order."""
    dx = x[:, None, 0] - xyz[None, :, 0]
    dy = x[:, None, 1] - xyz[None, :, 1]
    dz = x[:, None, 2] - xyz[None, :, 2]
    d2 = (dx * dx + dy * dy) + dz * dz
    order = np.argsort(d2, axis=1, kind="stable")
    return order[:, :min(k, len(xyz))]


def real_sph_harm(u):
    """Real spherical harmonics Y_lm (l = 0..2) of unit vectors u (n, 3), in
    the order Y00 | Y1,-1 Y10 Y11 (y z x) | xy yz (3z^2-1) xz (x^2-y^2).
    Rows with u = 0 (a point on an atom) get 0 for l > 0."""
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    c0 = 0.5 / np.sqrt(np.pi)
    c1 = np.sqrt(3.0 / (4.0 * np.pi))
    c2 = 0.5 * np.sqrt(15.0 / np.pi)
    c20 = 0.25 * np.sqrt(5.0 / np.pi)
    c22 = 0.25 * np.sqrt(15.0 / np.pi)
    Y = np.stack([np.full_like(x, c0), c1 * y, c1 * z, c1 * x,
                  c2 * x * y, c2 * y * z, c20 * (3 * z * z - 1.0), c2 * x * z,
                  c22 * (x * x - y * y)], 1)
    Y[np.all(u == 0, axis=1), 1:] = 0.0
    return Y


LSLICE = [slice(0, 1), slice(1, 4), slice(4, 9)]


def descriptors(pts, xyz, rho_sad, shift=None, scale=None):
    """(npts, 25) features of the points (see module docstring)."""
    pts = np.asarray(pts, np.float64)
    xyz = np.asarray(xyz, np.float64)
    nb = nearest_atoms(pts, xyz)
    F = np.zeros((len(pts), N_IN))
    if len(xyz):
        vec = pts[:, None, :] - xyz[nb]                       # (npts, k, 3)
        d = np.sqrt(np.sum(vec * vec, axis=2))
        with np.errstate(invalid="ignore", divide="ignore"):
            u = np.where(d[..., None] > 0, vec / d[..., None], 0.0)
        Y = real_sph_harm(u.reshape(-1, 3)).reshape(len(pts), nb.shape[1], 9)
        for n in range(NRAD):
            g = np.exp(-0.5 * (d - n) ** 2)                   # (npts, k)
            A = np.einsum("pk,pkm->pm", g, Y)                 # (npts, 9)
            for l in range(LMAX + 1):
                F[:, 3 * n + l] = np.sum(A[:, LSLICE[l]] ** 2, axis=1)
    F[:, 24] = np.log(np.maximum(np.asarray(rho_sad, np.float64), RHO_FLOOR))
    if shift is not None:
        F = (F - shift) / scale
    return F


# ------------------------------------------------------------------ MLP
SHAPES = [(HIDDEN, N_IN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,),
          (1, HIDDEN), (1,)]
N_PARAMS = int(sum(np.prod(s) for s in SHAPES))


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], np.float64).reshape(s))
        o += n
    return out


def pack(arrs):
    return np.concatenate([np.asarray(a, np.float64).ravel() for a in arrs])


def init_params(seed):
    """W, b ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), rounded to FP32."""
    rng = np.random.default_rng(seed)
    arrs = []
    for W, b in zip(SHAPES[0::2], SHAPES[1::2]):
        bound = 1.0 / np.sqrt(W[1])
        arrs.append(rng.uniform(-bound, bound, size=W).astype(np.float32))
        arrs.append(rng.uniform(-bound, bound, size=b).astype(np.float32))
    return pack(arrs)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X):
    """y (npts,) and the pre-activations (z1, z2, z3)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    z1 = X @ W1.T + b1
    z2 = silu(z1) @ W2.T + b2
    z3 = silu(z2) @ W3.T + b3
    y = silu(z3) @ W4[0] + b4[0]
    return y, (z1, z2, z3)


def loss(y, t, w):
    return float(np.sum(w * (y - t) ** 2) / np.sum(w))


def loss_grad(y, t, w):
    """dL/dy of the weighted squared error."""
    return 2.0 * w * (y - t) / np.sum(w)


def backward(theta, X, cache, dy):
    """Gradient (flat, same layout as theta) of sum_q dy_q y_q."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    z1, z2, z3 = cache
    h1, h2, h3 = silu(z1), silu(z2), silu(z3)
    gW4 = (dy @ h3)[None, :]
    gb4 = np.array([dy.sum()])
    dz3 = np.outer(dy, W4[0]) * dsilu(z3)
    gW3, gb3 = dz3.T @ h2, dz3.sum(0)
    dz2 = (dz3 @ W3) * dsilu(z2)
    gW2, gb2 = dz2.T @ h1, dz2.sum(0)
    dz1 = (dz2 @ W2) * dsilu(z1)
    gW1, gb1 = dz1.T @ X, dz1.sum(0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


def adam_step(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def density_guess(rho_sad, wq, y, target_scale, n_el, lo=0.9, hi=1.1):
    """(rho_0, used_fallback, factor) of the learned guess."""
    rho = np.maximum(rho_sad + target_scale * y, 0.0)
    if not np.all(np.isfinite(rho)):
        return np.array(rho_sad, copy=True), True, float("nan")
    total = float(np.sum(wq * rho))
    fac = n_el / total if total > 0 else float("inf")
    if not (np.isfinite(fac) and lo <= fac <= hi):
        return np.array(rho_sad, copy=True), True, fac
    return fac * rho, False, fac
