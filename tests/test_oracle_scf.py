"""Pins of the oracle's SCF layer against closed forms, derivatives,
independent one-dimensional integrals and invariants."""
import numpy as np
import pytest
from scipy import integrate as si

from oracle import enrich, fe, psp, scf
from paper_2607_06848_amd import workloads as wl


def test_lda_exchange_closed_form_and_derivative():
    rho = np.array([1e-4, 1e-2, 0.1, 1.0, 5.0])
    exc, vxc = scf.lda_pw92(rho)
    # uniform-gas exchange -(3/4)(3 rho / pi)^(1/3) is the rs -> 0 limit
    ex = -0.75 * (3 * rho / np.pi) ** (1 / 3)
    assert np.all(exc < ex)                 # correlation is negative
    # v_xc = d(rho eps_xc)/d rho by central differences
    h = 1e-6 * rho
    fp = (rho + h) * scf.lda_pw92(rho + h)[0]
    fm = (rho - h) * scf.lda_pw92(rho - h)[0]
    assert np.allclose(vxc, (fp - fm) / (2 * h), rtol=1e-7)
    e0, v0 = scf.lda_pw92(np.array([0.0, -1e-3]))
    assert np.all(e0 == 0) and np.all(v0 == 0)


def test_correlation_high_density_limit():
    """PW92 tends to the Gell-Mann--Brueckner form eps_c = c0 ln rs - c1 as
    rs -> 0 with c0 = A (the exact 0.0311)."""
    rs = np.array([1e-4, 2e-4])
    rho = 3.0 / (4 * np.pi * rs ** 3)
    exc, _ = scf.lda_pw92(rho)
    ec = exc + 0.75 * (3 * rho / np.pi) ** (1 / 3)
    slope = (ec[1] - ec[0]) / np.log(2.0)
    assert abs(slope - 0.031091) < 3e-4


def test_fermi_level():
    eps = np.array([-1.0, -0.5, -0.49, 0.2, 0.3, 1.0])
    for ne in (2.0, 5.0, 7.3):
        mu, f = scf.fermi_level(eps, ne, 500 * scf.KB_HA_PER_K)
        assert abs(2 * f.sum() - ne) < 1e-12
    mu, f = scf.fermi_level(eps, 4.0, 1e-6)        # T -> 0: aufbau
    assert np.allclose(f, [1, 1, 0, 0, 0, 0], atol=1e-12)


def test_fermi_level_inside_a_wide_gap():
    """Gap of 3 Ha at kT = 1e-2 Ha: 2 sum f is flat to rounding across it
    (tails near 1e-65), yet mu is fixed by the tails.  Two states at -1 (full)
    and one at +2 (empty), N_e = 4: the tails balance when
    exp(-(2 - mu)/kT) = 2 exp(-(mu + 1)/kT), i.e. mu = 1/2 + kT ln(2)/2; a
    symmetric gap puts mu in its middle."""
    kT = 1e-2
    mu, f = scf.fermi_level(np.array([-1.0, -1.0, 2.0]), 4.0, kT)
    assert mu == pytest.approx(0.5 + 0.5 * kT * np.log(2.0), abs=1e-12)
    mu, _ = scf.fermi_level(np.array([-1.0] * 4 + [1.0] * 4), 8.0, kT)
    assert abs(mu) < 1e-12


def _radial(fn, a=0.0, b=np.inf):
    return si.quad(fn, a, b, limit=400, epsabs=1e-14, epsrel=1e-13)[0]


def test_self_energy_by_radial_integral():
    rb, Z = 0.8, 4.0
    # 1/2 int b v_sm over R^3, b and v_sm of one smeared charge
    val = _radial(lambda r: 0.5 * 4 * np.pi * r * r * psp.b_smear(r, Z, rb)
                  * (-Z * psp.erf_over_r(r, rb)))
    assert abs(val - psp.self_energy([Z], rb)) < 1e-11


@pytest.mark.parametrize("R", [0.0, 0.7, 2.5])
def test_gaussian_coulomb_by_radial_integral(R):
    """<g_a, g_b>(R) against the spherical average of the potential of g_b
    over the shell of radius s around the centre of g_a."""
    a, b = 1.2, 1.0 / 0.64
    ga = lambda r: (a / np.pi) ** 1.5 * np.exp(-a * r * r)

    def shell(s):
        if R == 0.0:
            return 4 * np.pi * s * s * ga(s) * psp.erf_over_r(s, 1 / np.sqrt(b))
        mu = np.linspace(-1, 1, 401)
        d = np.sqrt(np.maximum(s * s + R * R - 2 * s * R * mu, 0.0))
        return 2 * np.pi * s * s * ga(s) * np.trapezoid(psp.erf_over_r(d, 1 / np.sqrt(b)), mu)

    val = _radial(shell, 0.0, 12.0)
    tol = 1e-10 if R == 0.0 else 1e-5
    assert abs(val - float(psp.gauss_coulomb(R, a, b))) < tol


def test_poisson_neutral_gaussian_pair():
    """-(1/4pi) Lap phi = g_a - g_b (same centre): phi = erf(sqrt a r)/r -
    erf(sqrt b r)/r, which vanishes at the box walls to round-off.  The nodal
    error falls at the spectral-element rate under refinement."""
    L = 16.0
    a, b = 1.0, 0.5
    errs = []
    for nc in (4, 6):
        mesh = fe.Mesh((0,) * 3, (L,) * 3, (nc,) * 3, 6, 7)
        es = scf.Electrostatics(mesh, np.zeros((0, 3)), np.zeros(0),
                                dict(rho_alpha=1.0, loc_rc=0.8, loc_amp=0.0, loc_rg=1.0))
        c = L / 2
        r = np.linalg.norm(mesh.quad_coords() - c, axis=-1)
        q = (a / np.pi) ** 1.5 * np.exp(-a * r * r) - (b / np.pi) ** 1.5 * np.exp(-b * r * r)
        phi, it = es.solve(q, rtol=1e-12)
        rn = np.linalg.norm(mesh.node_coords() - c, axis=-1)
        exact = psp.erf_over_r(rn, 1 / np.sqrt(a)) - psp.erf_over_r(rn, 1 / np.sqrt(b))
        errs.append(np.abs(phi - exact * (1 - mesh.boundary)).max() / np.abs(exact).max())
        assert it < 400
    assert errs[0] < 5e-3
    assert errs[1] < errs[0] / 4


def test_anderson_finite_termination_on_linear_map():
    """For an affine contraction x -> A x + c, Anderson with full history and
    beta = 1 is a Krylov method: it reaches the fixed point in n + 1 steps."""
    rng = np.random.default_rng(0)
    n = 6
    A = 0.5 * rng.normal(size=(n, n)) / np.sqrt(n)
    c = rng.normal(size=n)
    xstar = np.linalg.solve(np.eye(n) - A, c)
    mix = scf.Anderson(np.ones(n), beta=1.0, m=10)
    x = np.zeros(n)
    for _ in range(n + 2):
        x = mix.step(x, A @ x + c)
    assert np.abs(x - xstar).max() < 1e-9
    # history 0 is plain linear mixing
    lin = scf.Anderson(np.ones(n), beta=0.3, m=0)
    x0 = rng.normal(size=n)
    assert np.allclose(lin.step(x0, A @ x0 + c), x0 + 0.3 * (A @ x0 + c - x0))


def test_density_of_exactly_represented_functions():
    """A CFE polynomial and an enrichment function give rho = 2 f psi^2 at the
    Gauss points with psi evaluated directly."""
    w = wl.make("eig2")
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    s = enrich.EFESystem(mesh, w)
    Xn = mesh.node_coords()
    L = 10.0
    qn = Xn[:, 0] * (L - Xn[:, 0]) * Xn[:, 1] * (L - Xn[:, 1]) * Xn[:, 2] * (L - Xn[:, 2]) / L ** 6
    V = np.zeros((s.rows, 2))
    V[:s.n_nodes, 0] = qn * s.intr
    e = np.zeros(s.n_enr)
    e[1] = 1.0
    V[:s.n_nodes, 1] = s.C.T @ e
    V[s.n_nodes:, 1] = e
    rho = scf.density(s, V, np.array([0.5, 0.0]))
    Xq = mesh.quad_coords()
    qq = (Xq[..., 0] * (L - Xq[..., 0]) * Xq[..., 1] * (L - Xq[..., 1]) * Xq[..., 2]
          * (L - Xq[..., 2]) / L ** 6)
    assert np.abs(rho - qq * qq).max() < 1e-13
    rho = scf.density(s, V, np.array([0.0, 0.5]))
    I, k = 0, 1
    cells = s.supp[I]
    ref = np.zeros_like(rho)
    ref[cells] = s.phi[I][:, :, k] ** 2
    assert np.abs(rho - ref).max() < 1e-12 * ref.max()


def test_scf_converges_and_is_guess_independent():
    """The 2-atom system converges to the same energy from the superposition
    guess and from a perturbed guess (the converged SCF judges the guess)."""
    w = wl.make("eig2")
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    s = enrich.EFESystem(mesh, w)
    es = scf.Electrostatics(mesh, w["xyz"], w["Zs"], w)
    V0 = wl.random_block(s.rows, w["nvec"], 5)
    v0 = wl.random_vector(s.rows, 7)
    kT = 500 * scf.KB_HA_PER_K
    h1, _ = scf.scf(s, es, V0, v0, w["nvec"], w["degree"], 8.0, kT, tol=1e-8, max_iter=40)
    rho0 = es.rho_at * (1 + 0.2 * np.sin(mesh.quad_coords()[..., 0]))
    h2, _ = scf.scf(s, es, V0, v0, w["nvec"], w["degree"], 8.0, kT, tol=1e-8, max_iter=40,
                    rho0=rho0)
    assert len(h1) < 40 and len(h2) < 40
    assert abs(h1[-1]["E"] - h2[-1]["E"]) < 2e-6
    assert abs(h1[-1]["F"] - h1[-1]["E"]) < 1e-3


def test_kerker_on_a_dirichlet_mode():
    """The lowest Dirichlet mode of the box, sin(pi x/L) sin(pi y/L) sin(pi z/L),
    is an eigenfunction of -Lap with q^2 = 3 pi^2 / L^2: the preconditioner
    scales it by q^2 / (q^2 + k0^2) (to the discretization error), and leaves
    a field of much shorter wavelength nearly unchanged."""
    L = 10.0
    mesh = fe.Mesh((0,) * 3, (L,) * 3, (4,) * 3, 6, 7)
    es = scf.Electrostatics(mesh, np.zeros((0, 3)), np.zeros(0),
                            dict(rho_alpha=1.0, loc_rc=0.8, loc_amp=0.0, loc_rg=1.0))
    X = mesh.quad_coords()
    F = np.prod(np.sin(np.pi * X / L), axis=-1)
    q2 = 3 * np.pi ** 2 / L ** 2
    for k0 in (0.5, 1.0, 2.0):
        PF, it = es.kerker(F, k0)
        ratio = scf.integrate(mesh, PF * F) / scf.integrate(mesh, F * F)
        assert ratio == pytest.approx(q2 / (q2 + k0 ** 2), rel=1e-5)
        assert np.abs(PF - ratio * F).max() < 1e-4
    Fh = np.prod(np.sin(7 * np.pi * X / L), axis=-1)
    PF, _ = es.kerker(Fh, 0.5)
    q2h = 3 * (7 * np.pi) ** 2 / L ** 2
    ratio = scf.integrate(mesh, PF * Fh) / scf.integrate(mesh, Fh * Fh)
    assert ratio == pytest.approx(q2h / (q2h + 0.25), abs=2e-3)


def test_tau_controlled_passes_reach_the_tolerance():
    """With tau the first step keeps filtering until every occupied residual
    is below tau (Sec. III.B); its Ritz values then agree with the dense
    generalized eigensolve of the same potential."""
    from oracle import eigen
    w = wl.make("eig2")
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    s = enrich.EFESystem(mesh, w)
    es = scf.Electrostatics(mesh, w["xyz"], w["Zs"], w)
    V0 = wl.random_block(s.rows, w["nvec"], 5)
    v0 = wl.random_vector(s.rows, 7)
    kT = 500 * scf.KB_HA_PER_K
    tau = 1e-9
    h, _ = scf.scf(s, es, V0, v0, w["nvec"], w["degree"], 8.0, kT, max_iter=1,
                   passes_first=1, tau=tau, max_passes=40)
    r = h[0]
    assert 1 < r["passes"] < 40
    assert r["max_occ_res"] < tau
    ev = eigen.dense_ghep(s, 8)
    assert np.abs(r["lam"][:4] - ev[:4]).max() < 1e-9
    # without tau the minimum is run
    h1, _ = scf.scf(s, es, V0, v0, w["nvec"], w["degree"], 8.0, kT, max_iter=1, passes_first=2)
    assert h1[0]["passes"] == 2 and h1[0]["max_occ_res"] > tau
