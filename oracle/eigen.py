"""Chebyshev-filtered subspace iteration (oracle; test infrastructure).

Sec. III.B of the paper.  The scaled filter C_m(x) = T_m(L(x)) / T_m(L(a_min))
with L(x) = (x - c)/e, c = (a + b)/2, e = (b - a)/2, obeys the three-term
recurrence of Eq. (ChebyRecur) with sigma_1 = e / (a_min - c) and
sigma_k = 1 / (2/sigma_1 - sigma_{k-1}).

Residual filter (Eqs. residual, residualapprox).  The printed recurrence has
three misprints; the reading used here follows from inserting Eq. (ChebyRecur)
into the definition Z_k = M~ (C_k(A) V - V C_k(Lambda)):
    G    = H V - M V Lambda
    Z_0  = 0,  Z_1 = (sigma_1 / e) G
    Z_k  = (2 sigma_k / e) H (M~^-1 Z_{k-1}) - (2 c sigma_k / e) Z_{k-1}
           - sigma_{k-1} sigma_k Z_{k-2} + (2 sigma_k / e) G C_{k-1}(Lambda)
    Vout = M~^-1 Z_m + V C_m(Lambda)
(coefficient of Z_{k-2} is sigma_{k-1} sigma_k, the forcing term carries
C_{k-1}(Lambda), and the output adds V C_m(Lambda)).  With M~ = M this equals
the standard filter C_m(M^-1 H) V exactly.

Rayleigh-Ritz (Eq. projectedKSEig) uses the exact M^E.
"""
import numpy as np
import scipy.linalg as sla


# ---------------------------------------------------------------- scalars
def cheb_params(a, b, a_min):
    c = 0.5 * (a + b)
    e = 0.5 * (b - a)
    sigma1 = e / (a_min - c)
    return c, e, sigma1


def sigmas(a, b, a_min, m):
    """sigma_1 .. sigma_m (index 0 unused)."""
    c, e, s1 = cheb_params(a, b, a_min)
    s = np.zeros(m + 1)
    s[1] = s1
    for k in range(2, m + 1):
        s[k] = 1.0 / (2.0 / s1 - s[k - 1])
    return s


def cheb_scalar(x, a, b, a_min, m):
    """C_0(x) .. C_m(x) by the recurrence of Eq. (ChebyRecur); shape (m+1, ...)."""
    x = np.asarray(x, float)
    c, e, _ = cheb_params(a, b, a_min)
    s = sigmas(a, b, a_min, m)
    out = np.zeros((m + 1,) + x.shape)
    out[0] = 1.0
    if m >= 1:
        out[1] = s[1] * (x - c) / e
    for k in range(2, m + 1):
        out[k] = (2 * s[k] / e) * (x - c) * out[k - 1] - s[k - 1] * s[k] * out[k - 2]
    return out


def cheb_closed(x, a, b, a_min, m):
    """T_m(L(x)) / T_m(L(a_min)) from cos / cosh (definition of C_m)."""
    x = np.asarray(x, float)
    c, e, _ = cheb_params(a, b, a_min)

    def T(y):
        y = np.asarray(y, float)
        inside = np.abs(y) <= 1
        yi = np.clip(y, -1, 1)
        yo = np.where(inside, 2.0, np.abs(y))
        out_in = np.cos(m * np.arccos(yi))
        out_out = np.cosh(m * np.arccosh(yo)) * np.where(y < 0, (-1.0) ** m, 1.0)
        return np.where(inside, out_in, out_out)

    return T((x - c) / e) / T((a_min - c) / e)


# ---------------------------------------------------------------- filters
def standard_filter(apply_A, V, a, b, a_min, m):
    """V_out = C_m(A) V by the three-term recurrence (Eq. ChebyRecur)."""
    c, e, _ = cheb_params(a, b, a_min)
    s = sigmas(a, b, a_min, m)
    Yp = V.copy()
    Y = (s[1] / e) * (apply_A(V) - c * V)
    for k in range(2, m + 1):
        Yn = (2 * s[k] / e) * (apply_A(Y) - c * Y) - s[k - 1] * s[k] * Yp
        Yp, Y = Y, Yn
    return Y


def residual_filter(apply_H, apply_M, apply_Minv_tilde, V, lam, a, b, a_min, m):
    """Residual Chebyshev filter (Eqs. residual, residualapprox; reading in
    the module docstring).  ``lam`` are the Ritz values paired with V."""
    c, e, _ = cheb_params(a, b, a_min)
    s = sigmas(a, b, a_min, m)
    Cl = cheb_scalar(lam, a, b, a_min, m)          # (m+1, N)
    G = apply_H(V) - apply_M(V) * lam[None, :]
    Zp = np.zeros_like(V)
    Z = (s[1] / e) * G
    for k in range(2, m + 1):
        HY = apply_H(apply_Minv_tilde(Z))
        Zn = ((2 * s[k] / e) * HY - (2 * c * s[k] / e) * Z - s[k - 1] * s[k] * Zp
              + (2 * s[k] / e) * G * Cl[k - 1][None, :])
        Zp, Z = Z, Zn
    return apply_Minv_tilde(Z) + V * Cl[m][None, :]


# ---------------------------------------------------------------- RR
def rayleigh_ritz(apply_H, apply_M, V, active_mask=None):
    """Project on span(V): S = V^T M V, Hp = V^T H V, solve Hp d = eps S d,
    rotate V <- V D (Eq. projectedKSEig).  Returns (V, lam, resnorm) with
    resnorm_j = || H v_j - lam_j M v_j ||_2 on the coefficient vector."""
    HV = apply_H(V)
    MV = apply_M(V)
    S = V.T @ MV
    Hp = V.T @ HV
    S = 0.5 * (S + S.T)
    Hp = 0.5 * (Hp + Hp.T)
    lam, Q = sla.eigh(Hp, S)
    Vn = V @ Q
    R = HV @ Q - (MV @ Q) * lam[None, :]
    if active_mask is not None:
        Vn = Vn * active_mask[:, None]
        R = R * active_mask[:, None]
    return Vn, lam, np.linalg.norm(R, axis=0)


# ---------------------------------------------------------------- bounds
def lanczos_upper_bound(apply_H, apply_Mt, apply_Mt_inv, v0, k=20):
    """Upper bound of the spectrum of M~^-1 H by k Lanczos steps in the M~
    inner product: theta_max(T_k) + |beta_k| (reading of 'a_min <= eps_min',
    '(a, b)' in Sec. III.B: b must bound the operator being filtered).
    Each new vector is orthogonalized once more against all earlier ones
    (classical Gram-Schmidt in the M~ inner product): without it the basis
    loses orthogonality at a rate set by the conditioning of M~, and two
    roundings of the same run give different bounds."""
    v = v0 / np.sqrt(v0 @ apply_Mt(v0))
    v_prev = np.zeros_like(v)
    beta_prev = 0.0
    alphas, betas = [], []
    basis = []
    for j in range(k):
        basis.append(v)
        w = apply_Mt_inv(apply_H(v))
        alpha = w @ apply_Mt(v)
        w = w - alpha * v - beta_prev * v_prev
        Q = np.stack(basis, 1)
        w = w - Q @ (Q.T @ apply_Mt(w))
        beta = np.sqrt(w @ apply_Mt(w))
        alphas.append(alpha)
        betas.append(beta)
        v_prev, v = v, w / beta
        beta_prev = beta
    T = np.diag(alphas) + np.diag(betas[:-1], 1) + np.diag(betas[:-1], -1)
    theta = np.linalg.eigvalsh(T)
    return float(theta[-1] + abs(betas[-1])), float(theta[-1]), np.array(betas)


# ---------------------------------------------------------------- driver
def eigensolve(sys, V0, degree, passes, b, mode="residual", b_margin=1.0):
    """Fixed-potential multi-pass solve (Sec. III.B): one Rayleigh-Ritz of the
    start block (not counted), then ``passes`` times {filter with a = lam_N,
    a_min = lam_1; Rayleigh-Ritz}.  Returns the Ritz values and residual
    norms after every pass and the final block."""
    mask = np.zeros(sys.rows)
    mask[sys.active()] = 1.0
    V, lam, res = rayleigh_ritz(sys.apply_H, sys.apply_M, V0 * mask[:, None], mask)
    hist = [(lam.copy(), res.copy())]
    for _ in range(passes):
        a, a_min = lam[-1], lam[0]
        if mode == "residual":
            Vf = residual_filter(sys.apply_H, sys.apply_M, sys.apply_Minv_tilde, V, lam,
                                 a, b * b_margin, a_min, degree)
        elif mode == "standard":
            Vf = standard_filter(lambda X: sys.apply_Minv_tilde(sys.apply_H(X)), V,
                                 a, b * b_margin, a_min, degree)
        elif mode == "standard_exact":
            Vf = standard_filter(lambda X: sys.apply_Minv_exact(sys.apply_H(X)), V,
                                 a, b * b_margin, a_min, degree)
        else:
            raise ValueError(mode)
        V, lam, res = rayleigh_ritz(sys.apply_H, sys.apply_M, Vf, mask)
        hist.append((lam.copy(), res.copy()))
    return V, lam, res, hist


def dense_ghep(sys, k=None):
    """Reference: all (or the lowest k) eigenvalues of H^E x = eps M^E x over
    the active DoFs, by a dense generalized symmetric solve (Eq.
    lineigensolveghep).  Tiny meshes only."""
    H = sys.dense_HE()
    M = sys.dense_ME()
    H = 0.5 * (H + H.T)
    if k is None:
        return sla.eigh(H, M, eigvals_only=True)
    return sla.eigh(H, M, eigvals_only=True, subset_by_index=[0, k - 1])
