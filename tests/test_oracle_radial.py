"""Pins of the oracle's radial single-atom solver and of the pristine
enrichment built from it (Sec. II.B): closed-form spectra, a brute-force
dense eigensolve, the Coulomb potential of a Gaussian charge, charge and
self-consistency of the atom, the r0 rules on a hydrogen orbital, exactness of
the table interpolation, and the 3-D enrichment from the table against the
analytic function it tabulates."""
import numpy as np
import pytest

from oracle import fe, psp, radial
from paper_2607_06848_amd import workloads as wl


def _levels(v, h, n, l, k):
    r = radial.grid(n, h)
    return radial.eig_channel(l, v(r), r, h, k)[0]


@pytest.mark.parametrize("l", [0, 1, 2])
def test_hydrogenic_levels_converge_at_second_order(l):
    """-1/r: eps_nl = -1/(2 n^2), n = n_r + l + 1; the three-point rule's
    error falls by 4 when h halves."""
    exact = np.array([-0.5 / (k + l + 1) ** 2 for k in range(2)])
    e1 = _levels(lambda r: -1.0 / r, 0.02, 3000, l, 2) - exact
    e2 = _levels(lambda r: -1.0 / r, 0.01, 6000, l, 2) - exact
    assert np.all(np.abs(e2) < 2e-5)
    ratio = np.abs(e1[0] / e2[0])
    assert 3.6 < ratio < 4.4


@pytest.mark.parametrize("l", [0, 1, 2])
def test_oscillator_levels(l):
    """v = w^2 r^2 / 2: eps = w (2 n_r + l + 3/2)."""
    w = 1.3
    exact = w * (2 * np.arange(3) + l + 1.5)
    e1 = _levels(lambda r: 0.5 * w * w * r * r, 0.02, 1000, l, 3) - exact
    e2 = _levels(lambda r: 0.5 * w * w * r * r, 0.01, 2000, l, 3) - exact
    assert np.all(np.abs(e2) < 4e-4)
    assert np.all((np.abs(e1 / e2) > 3.6) & (np.abs(e1 / e2) < 4.4))


def test_projector_channel_matches_dense_eigensolve():
    """s channel with the rank-one projector term against numpy's dense
    eigensolver of the assembled matrix (brute force at n = 300)."""
    h, n = 0.05, 300
    r = radial.grid(n, h)
    p = wl.PSP
    v = psp.v_local(r, p["Z"], p["loc_rc"], p["loc_amp"], p["loc_rg"])
    q = radial.kb_vector(r, h, p["kb_width"], p["kb_rcut"])
    lam, U = radial.eig_channel(0, v, r, h, 3, p["kb_D"], q)
    d, e = radial.channel(0, v, r, h)
    A = np.diag(d) + np.diag(e, 1) + np.diag(e, -1) + p["kb_D"] * np.outer(q, q)
    lw, W = np.linalg.eigh(A)
    assert np.abs(lam - lw[:3]).max() < 1e-12 * np.abs(lw).max()
    for j in range(3):
        u = W[:, j] / np.sqrt(h)
        u *= np.sign(u[np.argmax(np.abs(u))])
        assert np.abs(U[:, j] - u).max() < 1e-9
    # the projector raises the s levels (D > 0) and the plain channel is below
    lam0, _ = radial.eig_channel(0, v, r, h, 3)
    assert np.all(lam > lam0)


def test_hartree_of_a_gaussian_charge():
    """rho = Z (a/pi)^{3/2} e^{-a r^2}: v_H = Z erf(sqrt(a) r) / r; second
    order in h."""
    Z, a = 4.0, 1.2
    errs = []
    for h, n in ((0.04, 1000), (0.02, 2000)):
        r = radial.grid(n, h)
        vh = radial.hartree(psp.rho_atom(r, Z, a), r, h)
        errs.append(np.abs(vh - Z * psp.erf_over_r(r, 1.0 / np.sqrt(a))).max())
    assert errs[1] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


@pytest.fixture(scope="module")
def atom():
    return radial.solve_atom(wl.PSP, n=1000, h=0.04, lmax=2, nstates=2)


def test_atom_is_self_consistent(atom):
    """Z electrons in the density; the output density's potential reproduces
    the bound levels; s and p hold two electrons each, d is empty (its levels
    are box states above zero)."""
    r, h = atom["r"], atom["h"]
    assert atom["residual"] < 1e-10
    assert abs(4 * np.pi * h * np.sum(r * r * atom["rho"]) - wl.PSP["Z"]) < 1e-10
    p = wl.PSP
    v = (psp.v_local(r, p["Z"], p["loc_rc"], p["loc_amp"], p["loc_rg"])
         + radial.hartree(atom["rho"], r, h) + radial.scf.lda_pw92(atom["rho"])[1])
    q = radial.kb_vector(r, h, p["kb_width"], p["kb_rcut"])
    for l in range(2):
        lam, _ = radial.eig_channel(l, v, r, h, 1, p["kb_D"], q)
        assert abs(lam[0] - atom["eps"][l][0]) < 1e-8
    assert np.all(atom["eps"][2] > 0)
    assert abs(atom["occ"][0][0] - 2) < 1e-9 and abs(atom["occ"][1][0] - 2) < 1e-9
    assert atom["occ"][2].sum() < 1e-9
    # the p shell holds 2 of 6 electrons: f = 1/3, so mu = eps_p - kT ln 2
    kT = 500 * 3.166811563e-6
    assert atom["eps"][0][0] < atom["eps"][1][0] < 0
    assert abs(atom["mu"] - (atom["eps"][1][0] - kT * np.log(2.0))) < 1e-6


def test_r0_rules_on_a_hydrogen_orbital():
    """R = 2 e^{-r}: u = 2 r e^{-r} turns at r = 1; |R'| = 2 e^{-r} drops below
    5e-3 at ln 400; the cutoff there keeps the norm within 5e-3.  So r0 is
    the first grid point beyond ln 400.  A function still too steep at 10
    bohr gets the cap."""
    h, n = 0.01, 6000
    r = radial.grid(n, h)
    u = 2 * r * np.exp(-r)
    assert abs(radial.last_turning_point(u, r) - 1.0) <= h
    r0 = radial.select_r0(u, r, h)
    first = r[np.flatnonzero(r > np.log(400.0))[0]]
    assert abs(r0 - first) < 1.5 * h
    assert 1 - radial.truncated_norm(u, r, h, r0) <= 5e-3
    wide = np.sqrt(2 * 0.05 ** 3) * 2 * r * np.exp(-0.05 * r)
    wide /= np.sqrt(h * np.sum(wide ** 2))
    assert radial.select_r0(wide, r, h) == 10.0


def test_hermite_table_is_exact_for_cubics():
    dr = 0.1
    x = np.arange(0, 51) * dr
    c = (0.3, -1.2, 0.7, 0.05)
    f = c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
    df = c[1] + 2 * c[2] * x + 3 * c[3] * x ** 2
    t = np.linspace(0, 4.99, 777)
    val, der = radial.hermite(f, df, dr, t)
    assert np.abs(val - (c[0] + c[1] * t + c[2] * t ** 2 + c[3] * t ** 3)).max() < 1e-12
    assert np.abs(der - (c[1] + 2 * c[2] * t + 3 * c[3] * t ** 2)).max() < 1e-11
    v, d = radial.hermite(f, df, dr, np.array([5.0 + 1e-9, 7.0]))
    assert np.all(v == 0) and np.all(d == 0)


def test_tabulated_enrichment_matches_the_function_it_tabulates():
    """A table of f(r) = e^{-a r^2} (exact values and slopes, fine spacing)
    gives the Gaussian enrichment of the same cutoff: values and gradients at
    the Gauss points within the interpolation error (fourth order)."""
    from oracle import enrich
    mesh = fe.Mesh((0.0,) * 3, (8.0,) * 3, (2, 2, 2), 4, 5)
    a, rc, t, dr = 0.6, 6.0, 0.33, 0.005
    x = np.arange(0, int(7.0 / dr) + 1) * dr
    table = dict(f=np.tile(np.exp(-a * x * x), (3, 1)),
                 df=np.tile(-2 * a * x * np.exp(-a * x * x), (3, 1)),
                 dr=dr, rc=np.full(3, rc), t=t)
    c = np.array([3.9, 4.2, 4.05])
    cells = np.arange(mesh.n_cells)
    p1, g1 = radial.enrichment_tabulated(mesh, c, cells, 2, table)
    p0, g0 = enrich.enrichment_raw(mesh, c, cells, 2, a, rc, t)
    assert np.abs(p1 - p0).max() < 1e-9 * np.abs(p0).max()
    assert np.abs(g1 - g0).max() < 1e-7 * np.abs(g0).max()


def test_enrichment_tables_of_the_synthetic_atom(atom):
    """Tables reproduce u / r^{l+1} at the grid points; r0 obeys the three
    rules and the cap; the cutoff radius is r0 (1 + 1/t)."""
    tab = radial.enrichment_tables(atom, 1)
    r, h = atom["r"], atom["h"]
    for l in range(2):
        u = atom["u"][l][:, 0]
        val, _ = radial.hermite(tab["f"][l], tab["df"][l], tab["dr"], r)
        assert np.abs(val * r ** (l + 1) - u).max() < 1e-12 * np.abs(u).max()
        r0 = tab["r0"][l]
        assert r0 <= 10.0
        assert r0 >= radial.last_turning_point(u, r)
        if r0 < 10.0:
            R = u / r
            i = int(round(r0 / h)) - 1
            assert abs(np.gradient(R, h)[i]) < 5e-3
            assert 1 - radial.truncated_norm(u, r, h, r0) <= 5e-3
        assert tab["rc"][l] == pytest.approx(r0 * (1 + 1 / 0.33))


def _gaussian_atom_tables(h=0.04, n=1000):
    """Tables of the Gaussian atomic density and its neutral potential with
    exact slopes (psp's closed forms), in the layout of atomic_tables."""
    from scipy.special import erf
    p = wl.PSP
    Z, a, rb = p["Z"], p["rho_alpha"], p["loc_rc"]
    x = h * np.arange(n + 1)
    rho = psp.rho_atom(x, Z, a)
    phi = psp.phi_atom(x, Z, a, rb)
    xs = np.where(x > 0, x, 1.0)

    def g(s):   # d/dr erf(s r) / r, r > 0
        return (2 / np.sqrt(np.pi)) * s * np.exp(-(s * xs) ** 2) / xs - erf(s * xs) / xs ** 2
    dphi = np.where(x > 0, Z * (g(np.sqrt(a)) - g(1 / rb)), 0.0)
    return dict(rho=(rho, -2 * a * x * rho), phi=(phi, dphi), dr=h)


def test_pair_coulomb_reproduces_gaussian_closed_forms():
    """<n_I, n_J> by the radial-angular quadrature of pair_coulomb against the
    Gaussian-Gaussian Coulomb closed forms (self term and three separations)."""
    p = wl.PSP
    Z, a, rb = p["Z"], p["rho_alpha"], p["loc_rc"]
    tab = _gaussian_atom_tables()
    ab = 1 / rb ** 2
    for R in (0.0, 1.5, 3.0, 6.0):
        ex = Z * Z * (psp.gauss_coulomb(R, a, a) - 2 * psp.gauss_coulomb(R, a, ab)
                      + psp.gauss_coulomb(R, ab, ab))
        assert abs(radial.pair_coulomb(tab, tab, Z, rb, R) - float(ex)) < 1e-9


def test_tabulated_electrostatics_match_the_gaussian_forms():
    """Electrostatics with Gaussian atom tables gives the analytic atomic
    density, potential and geometry energy of the Gaussian atoms, to the
    cubic Hermite error h^4 max|f^(4)| / 384 (about 1.2e-7 of rho(0) for the
    density at h = 0.04)."""
    from oracle import scf
    w = wl.make("eig2")
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    es0 = scf.Electrostatics(mesh, w["xyz"], w["Zs"], w)
    es1 = scf.Electrostatics(mesh, w["xyz"], w["Zs"], dict(w, atom_table=_gaussian_atom_tables()))
    assert np.abs(es1.rho_at - es0.rho_at).max() < 2e-7 * np.abs(es0.rho_at).max()
    assert np.abs(es1.phi_at - es0.phi_at).max() < 2e-7 * np.abs(es0.phi_at).max()
    assert abs(es1.constant_energy() - es0.constant_energy()) < 1e-8


def test_atomic_tables_of_the_synthetic_atom(atom):
    """The density table integrates to Z; w = r (phi + Z erf(r/r_b)/r) solves
    the three-point Poisson equation w'' = -4 pi r rho at every interior
    point; the neutral atom's potential vanishes at the end of the table."""
    p = wl.PSP
    tab = radial.atomic_tables(atom, p)
    h = tab["dr"]
    x = h * np.arange(len(tab["rho"][0]))
    wq = np.full(len(x), h)
    wq[0] = wq[-1] = h / 2
    assert abs(4 * np.pi * np.sum(wq * x * x * tab["rho"][0]) - p["Z"]) < 1e-9
    r = x[1:]
    wv = r * tab["phi"][0][1:] + p["Z"] * r * psp.erf_over_r(r, p["loc_rc"])
    res = (wv[2:] - 2 * wv[1:-1] + wv[:-2]) / h ** 2 + 4 * np.pi * r[1:-1] * tab["rho"][0][2:-1]
    assert np.abs(res).max() < 1e-9 * np.abs(4 * np.pi * r * tab["rho"][0][1:]).max()
    assert abs(tab["phi"][0][-1]) < 1e-9
