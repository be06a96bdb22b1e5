"""Radial Kohn-Sham problem of one isolated synthetic atom and the pristine
enrichment functions built from it (oracle; test infrastructure).

Sec. II.B: the enrichment functions are the Kohn-Sham eigenfunctions of the
isolated atom, a radial function times a real spherical harmonic, with the
radial part from a one-dimensional problem.  Each is truncated by the smooth
cutoff h(r, r0, t) (Eq. eqnCutoffProperties, t = 0.33), with r0 the smallest
radius that (i) lies at or beyond the last turning point of the radial
solution, (ii) keeps the truncated function's norm within 5e-3 of one and
(iii) sits in the tail, |dR/dr(r0)| < 5e-3; r0 is at most 10 bohr.

Readings (the paper gives no discretization or SCF details):
  * u(r) = r R(r) on the uniform grid r_i = i h (i = 1..n), u = 0 at r = 0
    and at r = (n+1) h.  Channel l:
        (H_l u)_i = -(u_{i+1} - 2 u_i + u_{i-1}) / (2 h^2)
                    + (l(l+1) / (2 r_i^2) + v_eff(r_i)) u_i
    plus, in the s channel, the Kleinman-Bylander term D |beta><beta| of the
    synthetic pseudopotential, <beta|psi> = sqrt(4 pi) int beta(r) r u(r) dr
    (the 3-D projector is s-type with unit norm).  In the vector
    w = sqrt(h) u the matrix is symmetric tridiagonal (+ D q q^T with
    q_i = sqrt(4 pi h) r_i beta(r_i)); eigenvectors are normalized to
    h sum u_i^2 = 1 with the largest |u_i| positive.
  * Rank-one term: the eigenpairs of T + D q q^T follow from those of the
    tridiagonal T by the secular equation 1 + D sum_j z_j^2/(lambda_j - mu)
    = 0, z = Q^T q (the rank-one modification of a symmetric eigenproblem);
    each root is bisected in its interval between poles.
  * Hartree: w = r v_H solves w'' = -4 pi r rho by the same three-point
    difference, w(0) = 0, w((n+1) h) = Q, Q = 4 pi h sum r_i^2 rho_i.
  * Exchange-correlation: PW92 LDA (the functional of the 3-D solver).
  * Occupations: Fermi-Dirac at the 3-D solver's kT, each (n, l) level
    holding 2 (2l + 1) electrons, mu by bisection for the atom's Z.
  * SCF: rho_in <- rho_in + beta (rho_out - rho_in), beta = 0.5, until the
    radial L2 norm sqrt(4 pi h sum r^2 (rho_out - rho_in)^2) < tol.
  * Last turning point: the last interior grid extremum of u (the largest i
    with (u_{i+1} - u_i)(u_i - u_{i-1}) <= 0).
  * Table: f_l(r) = u(r) / r^{l+1} = R(r) / r^l on r_i = i h (i = 0..n),
    f_l(0) = (4 f_l(h) - f_l(2h)) / 3 (f_l is even in r for a regular
    solution), slopes by central differences (one-sided at the ends,
    0 at r = 0); the 3-D enrichment function is S_lm(x) f_l(r) h(r) with
    the solid harmonics of the Gaussian enrichment, f_l by cubic Hermite
    interpolation of the table.
  * Atomic fields (Sec. III.C, one species): rho^(I) = the atom's output
    density and phi^(I) the potential of rho^(I) + b^(I) (b the Gaussian
    smeared charge), tabulated like f_l; the pair energies <n_I, n_J> by
    radial-angular quadrature (trapezoid over the table points, 64-point
    Gauss-Legendre in the angle), zero beyond the tables.
"""
import numpy as np
from scipy.linalg import eigh_tridiagonal, solve_banded

from . import enrich, psp, scf

T_CUTOFF = 0.33
R0_MAX = 10.0
NORM_TOL = 5e-3
SLOPE_TOL = 5e-3


def grid(n, h):
    return h * np.arange(1, n + 1, dtype=float)


def channel(l, v, r, h):
    """Diagonal and off-diagonal of the tridiagonal part of H_l."""
    d = 1.0 / (h * h) + l * (l + 1) / (2.0 * r * r) + v
    e = np.full(len(r) - 1, -0.5 / (h * h))
    return d, e


def kb_vector(r, h, width, rcut):
    """q with <beta|psi> = q . (sqrt(h) u)."""
    return np.sqrt(4.0 * np.pi * h) * r * psp.kb_beta(r, width, rcut)


def _sign_and_norm(w, h):
    """u from the scaled vector w: h sum u^2 = 1, largest |u| positive."""
    u = w / np.sqrt(h)
    u = u / np.sqrt(h * np.sum(u * u))
    k = np.argmax(np.abs(u))
    return u if u[k] > 0 else -u


def eig_channel(l, v, r, h, k, D=0.0, q=None):
    """The k lowest eigenpairs of channel l: values and u (n x k)."""
    d, e = channel(l, v, r, h)
    if D == 0.0 or q is None or l != 0:
        lam, W = eigh_tridiagonal(d, e, select="i", select_range=(0, k - 1))
    else:
        lam0, Q = eigh_tridiagonal(d, e)
        z = Q.T @ q
        lam = np.empty(k)
        W = np.empty((len(d), k))
        for j in range(k):
            lo, hi = lam0[j], lam0[j + 1]
            # f(mu) = 1 + D sum z^2 / (lam0 - mu) increases from -inf to +inf
            for _ in range(200):
                mu = 0.5 * (lo + hi)
                if mu <= lo or mu >= hi:
                    break
                if 1.0 + D * np.sum(z * z / (lam0 - mu)) < 0.0:
                    lo = mu
                else:
                    hi = mu
            mu = 0.5 * (lo + hi)
            lam[j] = mu
            W[:, j] = Q @ (z / (lam0 - mu))
    U = np.stack([_sign_and_norm(W[:, j], h) for j in range(k)], 1)
    return lam, U


def hartree(rho, r, h):
    """v_H from w'' = -4 pi r rho, w(0) = 0, w(R) = Q (three-point rule)."""
    n = len(r)
    Q = 4.0 * np.pi * h * np.sum(r * r * rho)
    rhs = -4.0 * np.pi * h * h * r * rho
    rhs[-1] -= Q
    ab = np.zeros((3, n))
    ab[0, 1:] = 1.0
    ab[1, :] = -2.0
    ab[2, :-1] = 1.0
    w = solve_banded((1, 1), ab, rhs)
    return w / r


def _density(U, occ, r):
    """Spherical density sum occ u^2 / (4 pi r^2) over the channels' levels
    (occ per channel, with the 2 (2l+1) factor)."""
    rho = np.zeros_like(r)
    for Ul, fl in zip(U, occ):
        rho += (Ul * Ul) @ fl
    return rho / (4.0 * np.pi * r * r)


def occupations(eps, Z, kT):
    """Occupations 2 (2l+1) f(eps_nl, mu) per channel, mu for Z electrons."""
    flat = np.concatenate([np.repeat(e, 2 * l + 1) for l, e in enumerate(eps)])
    mu, _ = scf.fermi_level(flat, Z, kT)
    return mu, [2.0 * (2 * l + 1) * scf.occupations(e, mu, kT) for l, e in enumerate(eps)]


def solve_atom(p, n=2000, h=0.02, lmax=1, nstates=2, kT=500 * 3.166811563e-6, beta=0.5,
               tol=1e-10, maxit=300, rho0=None):
    """Self-consistent isolated synthetic atom.  p: workload parameters (Z,
    loc_rc, loc_amp, loc_rg, kb_width, kb_D, kb_rcut, rho_alpha).  Returns a
    dict: r, h, eps (list per l), u (list of n x nstates), occ, mu, rho,
    v_eff, iterations, residual."""
    r = grid(n, h)
    Z = float(p["Z"])
    vloc = psp.v_local(r, Z, p["loc_rc"], p["loc_amp"], p["loc_rg"])
    q = kb_vector(r, h, p["kb_width"], p["kb_rcut"]) if p["kb_width"] > 0 else None
    D = float(p["kb_D"]) if q is not None else 0.0
    rho_in = psp.rho_atom(r, Z, p["rho_alpha"]) if rho0 is None else np.asarray(rho0, float)
    res = np.inf
    for it in range(1, maxit + 1):
        v = vloc + hartree(rho_in, r, h) + scf.lda_pw92(rho_in)[1]
        eps, U = [], []
        for l in range(lmax + 1):
            lam, Ul = eig_channel(l, v, r, h, nstates, D, q)
            eps.append(lam)
            U.append(Ul)
        mu, occ = occupations(eps, Z, kT)
        rho_out = _density(U, occ, r)
        d = rho_out - rho_in
        res = np.sqrt(4.0 * np.pi * h * np.sum(r * r * d * d))
        if res < tol:
            break
        rho_in = rho_in + beta * d
    return dict(r=r, h=h, eps=eps, u=U, occ=occ, mu=mu, rho=rho_out, v_eff=v, iterations=it,
                residual=res)


# ---------------------------------------------------------------- r0 rules
def last_turning_point(u, r):
    """Radius of the last interior extremum of u (0 if there is none)."""
    du = np.diff(u)
    ext = np.flatnonzero(du[:-1] * du[1:] <= 0.0)
    return r[ext[-1] + 1] if ext.size else 0.0


def truncated_norm(u, r, h, r0, t=T_CUTOFF):
    """h sum (u h(r; r0, t))^2 for a function with h sum u^2 = 1."""
    hc, _ = enrich.cutoff(r, r0 * (1.0 + 1.0 / t), t)
    return h * np.sum((u * hc) ** 2)


def select_r0(u, r, h, t=T_CUTOFF, r0_max=R0_MAX, norm_tol=NORM_TOL, slope_tol=SLOPE_TOL):
    """Smallest grid radius meeting rules (i)-(iii), at most r0_max."""
    R = u / r
    dR = np.gradient(R, h)
    rt = last_turning_point(u, r)
    for i in np.flatnonzero((r >= rt) & (r <= r0_max)):
        if abs(dR[i]) < slope_tol and 1.0 - truncated_norm(u, r, h, r[i], t) <= norm_tol:
            return float(r[i])
    return float(r0_max)


# ---------------------------------------------------------------- table
def radial_table(u, r, h, l):
    """f_l = u / r^{l+1} on r_i = i h (i = 0..n) and its slopes."""
    f = np.empty(len(r) + 1)
    f[1:] = u / r ** (l + 1)
    f[0] = (4.0 * f[1] - f[2]) / 3.0
    df = np.empty_like(f)
    df[1:-1] = (f[2:] - f[:-2]) / (2.0 * h)
    df[0] = 0.0
    df[-1] = (f[-1] - f[-2]) / h
    return f, df


def hermite(f, df, dr, x):
    """Cubic Hermite interpolation of the table (f, df on x_i = i dr) at x
    (values and derivatives; zero beyond the table)."""
    x = np.asarray(x, float)
    s = x / dr
    i = np.clip(np.floor(s).astype(int), 0, len(f) - 2)
    t = s - i
    inside = x <= (len(f) - 1) * dr
    t2, t3 = t * t, t * t * t
    h00, h10 = 2 * t3 - 3 * t2 + 1, t3 - 2 * t2 + t
    h01, h11 = -2 * t3 + 3 * t2, t3 - t2
    val = h00 * f[i] + h10 * dr * df[i] + h01 * f[i + 1] + h11 * dr * df[i + 1]
    d00, d10 = (6 * t2 - 6 * t) / dr, 3 * t2 - 4 * t + 1
    d01, d11 = (-6 * t2 + 6 * t) / dr, 3 * t2 - 2 * t
    der = d00 * f[i] + d10 * df[i] + d01 * f[i + 1] + d11 * df[i + 1]
    return np.where(inside, val, 0.0), np.where(inside, der, 0.0)


def enrichment_tables(atom, lmax):
    """Per l <= lmax the lowest state's table and its cutoff: a dict with
    f (lmax+1, n+1), df, dr, r0 (per l), rc = r0 (1 + 1/t) (support end)."""
    r, h = atom["r"], atom["h"]
    F, DF, R0 = [], [], []
    for l in range(lmax + 1):
        u = atom["u"][l][:, 0]
        f, df = radial_table(u, r, h, l)
        F.append(f)
        DF.append(df)
        R0.append(select_r0(u, r, h))
    R0 = np.array(R0)
    return dict(f=np.array(F), df=np.array(DF), dr=h, r0=R0, rc=R0 * (1.0 + 1.0 / T_CUTOFF),
                t=T_CUTOFF)


def enrichment_tabulated(mesh, center, cells, lmax, table):
    """Unnormalized phi = S_k(d) f_l(r) h(r; rc_l, t) and its gradient at the
    Gauss points of ``cells`` (k of angular momentum l), from a table of
    enrichment_tables: shapes (nc, nq^3, nf) and (nc, nq^3, nf, 3).
    grad phi = grad S f h + S (f' h + f h') d / r."""
    X = mesh.quad_coords(cells)
    d = X - np.asarray(center, float)[None, None, :]
    r = np.sqrt(np.sum(d * d, -1))
    rs = np.where(r > 0, r, 1.0)
    S, dS = enrich.solid_harmonics(d, lmax)
    lof = np.concatenate([np.full(2 * l + 1, l) for l in range(lmax + 1)])
    rad, drad = [], []
    for l in range(lmax + 1):
        f, fp = hermite(table["f"][l], table["df"][l], table["dr"], r)
        hc, dh = enrich.cutoff(r, table["rc"][l], table["t"])
        rad.append(f * hc)
        drad.append((fp * hc + f * dh) / rs)
    rad = np.stack(rad, -1)[..., lof]
    drad = np.stack(drad, -1)[..., lof]
    phi = S * rad
    grad = dS * rad[..., None] + (S * drad)[..., None] * d[..., None, :]
    return phi, grad


# ---------------------------------------------------------------- atomic fields
def atomic_tables(atom, p):
    """The isolated atom's density rho^(I) and the potential phi^(I) of
    rho^(I) + b^(I) (the neutral atom: b the Gaussian smeared nuclear charge
    of width r_b = loc_rc), Sec. III.C, tabulated at r = i h (i = 0..n) with
    slopes, in the form of radial_table: rho from the last output density;
    phi = v_H[rho] - Z erf(r / r_b) / r with v_H by the three-point rule
    (hartree); both even in r, so their r = 0 values come from
    (4 f(h) - f(2h)) / 3.  Returns dict(rho=(f, df), phi=(f, df), dr)."""
    r, h = atom["r"], atom["h"]
    rho = atom["rho"]
    phi = hartree(rho, r, h) - float(p["Z"]) * psp.erf_over_r(r, p["loc_rc"])

    def tab(v):
        f = np.empty(len(r) + 1)
        f[1:] = v
        f[0] = (4.0 * f[1] - f[2]) / 3.0
        df = np.empty_like(f)
        df[1:-1] = (f[2:] - f[:-2]) / (2.0 * h)
        df[0] = 0.0
        df[-1] = (f[-1] - f[-2]) / h
        return f, df
    return dict(rho=tab(rho), phi=tab(phi), dr=h)


def pair_coulomb(tabI, tabJ, Z, rb, R, nmu=64):
    """<n_I, n_J> = int n_I(x) phi_J(|x - R|) d^3x for spherical n_I = rho_I +
    b_I (b the Gaussian smeared charge -Z) and phi_J the potential of n_J:
    2 pi sum_i w_i r_i^2 n_I(r_i) sum_k w_k phi_J(d_ik), d_ik^2 = r_i^2 + R^2 -
    2 r_i R mu_k, over the table points r_i (trapezoid weights) and nmu
    Gauss-Legendre nodes mu_k; phi_J by cubic Hermite interpolation, zero
    beyond its table.  R = 0 gives the self term 4 pi int n phi r^2 dr."""
    dr = tabI["dr"]
    f = tabI["rho"][0]
    ri = dr * np.arange(len(f))
    wi = np.full(len(f), dr)
    wi[0] = wi[-1] = 0.5 * dr
    n_i = f + psp.b_smear(ri, Z, rb)
    mu, wm = np.polynomial.legendre.leggauss(nmu)
    d = np.sqrt(np.maximum(ri[:, None] ** 2 + R * R - 2.0 * ri[:, None] * R * mu[None, :], 0.0))
    phij, _ = hermite(tabJ["phi"][0], tabJ["phi"][1], tabJ["dr"], d)
    return float(2.0 * np.pi * np.sum(wi * ri * ri * n_i * (phij @ wm)))
