"""Self-consistent field support (oracle; test infrastructure only).

Sec. II.A of the paper: density from the orbitals (Eq. rhocompute), Fermi
level from the electron count (Eq. electronconstraint), Kohn-Sham potential
v_KS = v_xc + v_el (Eq. vKS) with LDA exchange-correlation in the Perdew-Wang
1992 form, the local reformulation of the electrostatics (Eqs. EZZbsmear,
EellocReform, poisson), energies; Sec. III.C: electrostatic potential split
phi = phi^at + phi^rem with phi^rem from a Poisson problem for the smooth
Delta rho = rho - sum_I rho^(I) on the CFE mesh without enrichment; Sec. IV:
Fermi-Dirac smearing at 500 K and Anderson mixing.

Readings (the paper defers these details):
  * phi^rem solves -(1/4 pi) Lap phi^rem = Delta rho with homogeneous
    Dirichlet data on the box, by CG with a Jacobi preconditioner.
  * total energy at the output density (one more Poisson solve):
        E = E_band - int rho_out v_eff[rho_in] + E_xc[rho_out] + E_el[rho_out]
    with E_el = 1/2 sum_IJ <n_I, n_J> + int Drho phi^at + 1/2 int Drho phi^rem
              + int rho v_short - E_self + dE_ZZ,   n_I = rho^(I) + b^(I);
    free energy F = E - T S, S = -2 k_B sum[f ln f + (1-f) ln(1-f)].
  * Anderson mixing of rho at the Gauss points in the quadrature-weighted
    inner product, history depth m; optionally with a Kerker preconditioner
    (a reading beyond the paper, for charge sloshing in large clusters).
  * filter passes per SCF step: a minimum, then more until the largest
    occupied-state residual is below tau (Sec. III.B), up to a cap.
  * LDA terms vanish where rho <= 1e-14.

Pins (tests/test_oracle_scf.py, tests/test_oracle_energy.py): the band-energy
identity, E_el against Gaussian closed forms, the PW92 high-density limit
(A, c1 and beta_2 = 2 A beta_1^2).  Parity unpinned: the fitted PW92 constants
alpha_1, beta_3 and beta_4 (no closed form fixes them; the published table is
the only source) and the assembled total energy of a cluster.
"""
import numpy as np
from scipy.special import expit

from . import eigen, psp

KB_HA_PER_K = 3.166811563e-6

# Perdew-Wang 1992, unpolarized correlation (Phys. Rev. B 45, 13244, Table I)
PW92_A, PW92_A1 = 0.031091, 0.21370
PW92_B = (7.5957, 3.5876, 1.6382, 0.49294)


# ---------------------------------------------------------------- LDA
def lda_pw92(rho):
    """eps_xc(rho) (energy per electron) and v_xc = d(rho eps_xc)/d rho.
    A, beta_1 and beta_2 are pinned by the high-density expansion; alpha_1,
    beta_3 and beta_4 are fitted constants of the published table: parity
    unpinned."""
    rho = np.asarray(rho, float)
    pos = rho > 1e-14
    r = np.where(pos, rho, 1.0)
    ex = -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * np.cbrt(r)
    vx = 4.0 / 3.0 * ex
    rs = np.cbrt(3.0 / (4.0 * np.pi * r))
    A, a1 = PW92_A, PW92_A1
    b1, b2, b3, b4 = PW92_B
    srs = np.sqrt(rs)
    Q0 = -2.0 * A * (1.0 + a1 * rs)
    Q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs)
    Q1p = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs)
    L = np.log1p(1.0 / Q1)
    ec = Q0 * L
    dec = -2.0 * A * a1 * L - Q0 * Q1p / (Q1 * Q1 + Q1)
    vc = ec - rs / 3.0 * dec
    return np.where(pos, ex + ec, 0.0), np.where(pos, vx + vc, 0.0)


# ---------------------------------------------------------------- occupations
def occupations(eps, mu, kT):
    """Fermi-Dirac f(eps, mu) (Eq. rhocompute)."""
    return expit(-(np.asarray(eps) - mu) / kT)


def electron_excess(eps, mu, n_electrons, kT):
    """2 sum_i f(eps_i, mu) - N_e written as the integer 2 #{eps_i <= mu} - N_e
    plus the Fermi tails 2 (sum_{eps_i > mu} f_i - sum_{eps_i <= mu} (1 - f_i)),
    each tail term formed without cancellation (1 - f(x) = expit(x) for
    x = (eps - mu)/kT <= 0).  Inside a gap much wider than kT the plain sum is
    flat to rounding; this form keeps its sign resolved there."""
    x = (np.asarray(eps, float) - mu) / kT
    below = x <= 0.0
    tails = np.sum(expit(-x[~below])) - np.sum(expit(x[below]))
    return (2.0 * np.count_nonzero(below) - n_electrons) + 2.0 * tails


def fermi_level(eps, n_electrons, kT, iters=200):
    """mu with 2 sum_i f(eps_i, mu) = N_e by bisection (Eq. electronconstraint)."""
    eps = np.asarray(eps, float)
    lo = eps.min() - 50.0 * kT - 1.0
    hi = eps.max() + 50.0 * kT + 1.0
    for _ in range(iters):
        mu = 0.5 * (lo + hi)
        if electron_excess(eps, mu, n_electrons, kT) < 0.0:
            lo = mu
        else:
            hi = mu
    mu = 0.5 * (lo + hi)
    return mu, occupations(eps, mu, kT)


def entropy_term(f, kT):
    """T S = -2 kT sum [f ln f + (1-f) ln(1-f)]."""
    f = np.asarray(f, float)
    g = np.where((f > 0) & (f < 1), f * np.log(np.where(f > 0, f, 1)) +
                 (1 - f) * np.log(np.where(f < 1, 1 - f, 1)), 0.0)
    return -2.0 * kT * g.sum()


# ---------------------------------------------------------------- density
def density(sys, V, f, chunk=16):
    """rho(q) = 2 sum_j f_j psi_j(q)^2 at every Gauss point (Eq. rhocompute),
    psi = sum_j N^C_j Vhat_j + sum_k phi_k V^E_k with Vhat = V^C - C^T V^E (the
    CFE coefficients of the orthogonalized expansion)."""
    mesh = sys.mesh
    n = sys.n_nodes
    rho = np.zeros((mesh.n_cells, mesh.nqp))
    f = np.asarray(f, float)
    cols = np.flatnonzero(f > 1e-14)
    for s in range(0, cols.size, chunk):
        cc = cols[s:s + chunk]
        Vc = V[:n, cc] * sys.intr[:, None]
        VE = V[n:, cc]
        if sys.nf:
            Vc = Vc - sys.C.T @ VE
        psi = np.einsum('ql,clj->cqj', mesh.N3, Vc[mesh.cell_to_global], optimize=True)
        for I in range(sys.natoms if sys.nf else 0):
            psi[sys.supp[I]] += np.einsum('cqk,kj->cqj', sys.phi[I],
                                          VE[I * sys.nf:(I + 1) * sys.nf])
        rho += 2.0 * np.einsum('cqj,j->cq', psi * psi, f[cc])
    return rho


def integrate(mesh, fq):
    """Gauss-rule integral of a field given at the Gauss points."""
    return float(np.sum(fq * mesh.W3[None, :]))


# ---------------------------------------------------------------- electrostatics
class Electrostatics:
    """Atomic parts at the Gauss points and the Poisson problem for phi^rem
    (Sec. III.C)."""

    def __init__(self, mesh, xyz, Z, prm):
        self.mesh = mesh
        self.xyz = np.asarray(xyz, float).reshape(-1, 3)
        self.Z = np.asarray(Z, float)
        self.prm = prm
        X = mesh.quad_coords()
        self.rho_at = np.zeros(X.shape[:2])
        self.phi_at = np.zeros(X.shape[:2])
        self.v_short = np.zeros(X.shape[:2])
        a, rb = prm["rho_alpha"], prm["loc_rc"]
        # atomic densities and potentials: Gaussian forms, or (atom_table, one
        # species) the isolated atom's radial solution (radial.atomic_tables)
        self.tab = prm.get("atom_table")
        if self.tab is not None:
            from . import radial
        for R, Z in zip(self.xyz, self.Z):
            r = np.linalg.norm(X - R, axis=-1)
            if self.tab is None:
                self.rho_at += psp.rho_atom(r, Z, a)
                self.phi_at += psp.phi_atom(r, Z, a, rb)
            else:
                self.rho_at += radial.hermite(*self.tab["rho"], self.tab["dr"], r)[0]
                self.phi_at += radial.hermite(*self.tab["phi"], self.tab["dr"], r)[0]
            self.v_short += psp.v_short(r, prm["loc_amp"], prm["loc_rg"])
        K = mesh.stiffness_cell()
        d = np.zeros(mesh.n_nodes)
        np.add.at(d, mesh.cell_to_global.ravel(), np.tile(np.diag(K), mesh.n_cells))
        self.Kdiag = np.where(mesh.boundary == 0, d, 1.0)
        self.m_int = mesh.lumped_mass() * (1 - mesh.boundary)

    def K(self, x, shift=0.0):
        """(K + shift diag(m)) x on the interior nodes."""
        y = self.mesh.cfe_apply(None, x, kinetic=1.0)
        return y + shift * self.m_int * x if shift else y

    def solve(self, drho_q, x0=None, rtol=1e-12, maxit=5000, scale=4.0 * np.pi, shift=0.0):
        """phi^rem at the nodes: K phi = 4 pi int Drho N (interior nodes), by
        Jacobi-preconditioned CG from x0.  Returns (phi, iterations).  With
        scale and shift: (K + shift diag(m)) x = scale int f N."""
        b = scale * self.mesh.load_vector(drho_q)
        x = np.zeros_like(b) if x0 is None else x0 * (1 - self.mesh.boundary)
        diag = np.where(self.mesh.boundary == 0, self.Kdiag + shift * self.m_int, 1.0)
        r = b - self.K(x, shift)
        z = r / diag
        p = z.copy()
        rz = r @ z
        bn = np.sqrt(b @ b)
        it = 0
        if bn == 0.0:            # zero source: zero potential
            return np.zeros_like(b), 0
        while np.sqrt(r @ r) > rtol * bn and it < maxit:
            Ap = self.K(p, shift)
            alpha = rz / (p @ Ap)
            x += alpha * p
            r -= alpha * Ap
            z = r / diag
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
            it += 1
        return x, it

    def kerker(self, F, k0, rtol=1e-12):
        """Kerker preconditioner of the mixing residual F (at the Gauss points):
        F - u with u the CFE solution of (K + k0^2 diag(m)) u = k0^2 int F N,
        i.e. F scaled by q^2 / (q^2 + k0^2) in Fourier terms.  Not in the
        paper, which names Anderson mixing only."""
        u, it = self.solve(F, None, rtol, scale=k0 * k0, shift=k0 * k0)
        return F - self.mesh.gather_quad(u), it

    def pair_energy(self):
        """1/2 sum_IJ <n_I, n_J> with n_I = rho^(I) + b^(I), in closed form from
        Gaussian-Gaussian Coulomb integrals (the I = J terms included); with
        tabulated atoms by radial.pair_coulomb."""
        if self.tab is not None:
            from . import radial
            rb = self.prm["loc_rc"]
            e = 0.0
            for i in range(len(self.Z)):
                for j in range(len(self.Z)):
                    R = float(np.linalg.norm(self.xyz[i] - self.xyz[j]))
                    e += 0.5 * radial.pair_coulomb(self.tab, self.tab, self.Z[i], rb, R)
            return e
        a = self.prm["rho_alpha"]
        ab = 1.0 / self.prm["loc_rc"] ** 2
        e = 0.0
        for i in range(len(self.Z)):
            for j in range(len(self.Z)):
                R = np.linalg.norm(self.xyz[i] - self.xyz[j])
                g = (psp.gauss_coulomb(R, a, a) - 2.0 * psp.gauss_coulomb(R, a, ab)
                     + psp.gauss_coulomb(R, ab, ab))
                e += 0.5 * self.Z[i] * self.Z[j] * float(g)
        return e

    def constant_energy(self):
        """Geometry-only part of E_el: 1/2 sum <n_I, n_J> - E_self + dE_ZZ."""
        rb = self.prm["loc_rc"]
        return (self.pair_energy() - psp.self_energy(self.Z, rb)
                + psp.delta_ezz(self.xyz, self.Z, rb))


# ---------------------------------------------------------------- mixing
class Anderson:
    """Anderson mixing of x = rho at the Gauss points (Sec. IV): with the
    residuals F = x_out - x_in of the last m+1 steps,
        gamma = argmin || F_k - dF gamma ||_W,  x_bar = x_k - dX gamma,
        F_bar = F_k - dF gamma,  x_next = x_bar + beta F_bar,
    dX, dF the differences of consecutive inputs and residuals, W the
    quadrature weights."""

    def __init__(self, w, beta=0.3, m=8):
        self.w = np.asarray(w, float).ravel()
        self.beta = beta
        self.m = m
        self.X, self.F = [], []

    def step(self, x_in, x_out, precond=None):
        """Next input; with precond, x_next = x_bar + beta P(F_bar) where
        P maps a residual of the input's shape to a preconditioned one."""
        x = np.asarray(x_in, float).ravel()
        F = np.asarray(x_out, float).ravel() - x
        self.X.append(x.copy())
        self.F.append(F.copy())
        if len(self.X) > self.m + 1:
            self.X.pop(0)
            self.F.pop(0)
        k = len(self.X) - 1
        P = ((lambda v: np.asarray(precond(v.reshape(np.shape(x_in))), float).ravel())
             if precond is not None else (lambda v: v))
        if k == 0:
            return (x + self.beta * P(F)).reshape(np.shape(x_in))
        dX = np.stack([self.X[i + 1] - self.X[i] for i in range(k)], 1)
        dF = np.stack([self.F[i + 1] - self.F[i] for i in range(k)], 1)
        A = dF.T @ (self.w[:, None] * dF)
        rhs = dF.T @ (self.w * F)
        gamma = np.linalg.solve(A, rhs)
        xb = x - dX @ gamma
        Fb = F - dF @ gamma
        return (xb + self.beta * P(Fb)).reshape(np.shape(x_in))


# ---------------------------------------------------------------- driver
def effective_potential(es, rho_in, phi_rem_nodes):
    """v_eff = phi^at + phi^rem + v_short + v_xc at the Gauss points (Eq. vKS
    with the split of Sec. III.C)."""
    _, vxc = lda_pw92(rho_in)
    return es.phi_at + es.mesh.gather_quad(phi_rem_nodes) + es.v_short + vxc


def total_energy(sys, es, lam, f, rho_out, v_in, kT, phi0=None, rtol=1e-12):
    """Energies at the output density (reading in the module docstring).
    Parity unpinned as a whole: its parts (band sum, PW92 LDA, Gaussian
    self and pair energies, the Poisson solve) are pinned, and the converged
    SCF energy is pinned to be independent of the start, but the assembled
    total of a cluster has no closed form."""
    mesh = sys.mesh
    e_band = 2.0 * float(np.sum(f * lam))
    exc, _ = lda_pw92(rho_out)
    drho = rho_out - es.rho_at
    phi_rem, it = es.solve(drho, phi0, rtol)
    pq = mesh.gather_quad(phi_rem)
    e_xc = integrate(mesh, rho_out * exc)
    e_el = (es.constant_energy() + integrate(mesh, drho * es.phi_at)
            + 0.5 * integrate(mesh, drho * pq) + integrate(mesh, rho_out * es.v_short))
    e_rv = integrate(mesh, rho_out * v_in)
    E = e_band - e_rv + e_xc + e_el
    TS = entropy_term(f, kT)
    return dict(E=E, F=E - TS, E_band=e_band, E_xc=e_xc, E_el=e_el, int_rho_v=e_rv,
                n_el=integrate(mesh, rho_out)), phi_rem


def max_occupied_residual(lam, res, n_electrons, kT):
    """Largest residual among the states occupied (f > 1e-14) at the Fermi
    level of the Ritz values lam."""
    _, f = fermi_level(lam, n_electrons, kT)
    occ = f > 1e-14
    return float(np.max(res[occ])) if np.any(occ) else 0.0


def scf(sys, es, V0, v0, nvec, degree, n_electrons, kT, beta=0.3, m=8, tol=1e-5,
        max_iter=50, passes_first=4, passes=1, lanczos=20, rho0=None, rtol=1e-12,
        tau=0.0, max_passes=0, kerker_k0=0.0):
    """SCF iterations (CS of Sec. II.A with the filter of Sec. III.B):
    rho_in -> Poisson for phi^rem -> v_eff -> bound -> filter passes and
    Rayleigh-Ritz -> mu -> rho_out -> energy -> Anderson.  Each step runs at
    least passes_first (first step) or passes filter + Rayleigh-Ritz passes,
    then more while the largest occupied-state residual exceeds tau, up to
    max_passes (Sec. III.B: filter until the eigen-residual is below a
    tolerance; tau <= 0 keeps the minimum).  kerker_k0 > 0 preconditions the
    Anderson update with Electrostatics.kerker.  Converged when
    |E_k - E_{k-1}| / N_atoms < tol.  Returns a list of per-step records."""
    mesh = sys.mesh
    mask = np.zeros(sys.rows)
    mask[sys.active()] = 1.0
    rho_in = es.rho_at.copy() if rho0 is None else np.array(rho0, float)
    mix = Anderson(np.tile(mesh.W3, mesh.n_cells), beta, m)
    V = V0 * mask[:, None]
    lam = None
    phi = None
    hist = []
    E_prev = None
    for it in range(max_iter):
        phi, cg_it = es.solve(rho_in - es.rho_at, phi, rtol)
        v_in = effective_potential(es, rho_in, phi)
        sys.set_potential(v_in)
        b, _, _ = eigen.lanczos_upper_bound(sys.apply_H, sys.apply_Mtilde, sys.apply_Minv_tilde,
                                            v0 * mask, lanczos)
        nmin = passes_first if it == 0 else passes
        nmax = max(nmin, max_passes if tau > 0 else nmin)
        if it == 0:
            V, lam, res = eigen.rayleigh_ritz(sys.apply_H, sys.apply_M, V, mask)
        npass = 0
        while npass < nmax:
            Vf = eigen.residual_filter(sys.apply_H, sys.apply_M, sys.apply_Minv_tilde, V, lam,
                                       lam[-1], b, lam[0], degree)
            V, lam, res = eigen.rayleigh_ritz(sys.apply_H, sys.apply_M, Vf, mask)
            npass += 1
            occ_res = max_occupied_residual(lam, res, n_electrons, kT)
            if npass >= nmin and not (tau > 0 and occ_res > tau):
                break
        mu, f = fermi_level(lam, n_electrons, kT)
        rho_out = density(sys, V, f)
        en, _ = total_energy(sys, es, lam, f, rho_out, v_in, kT, phi, rtol)
        drho = np.sqrt(integrate(mesh, (rho_out - rho_in) ** 2))
        rec = dict(iter=it, mu=mu, lam=lam.copy(), res=res.copy(), drho=drho, cg=cg_it, b=b,
                   passes=npass, max_occ_res=occ_res, **en)
        hist.append(rec)
        if E_prev is not None and abs(en["E"] - E_prev) / len(es.Z) < tol:
            break
        E_prev = en["E"]
        pre = (lambda F: es.kerker(F, kerker_k0, rtol)[0]) if kerker_k0 > 0 else None
        rho_in = mix.step(rho_in, rho_out, pre)
    return hist, V
