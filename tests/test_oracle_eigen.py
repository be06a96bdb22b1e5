"""Pins of the oracle's enrichment and eigensolver layers.

Enrichment wiring is pinned through quantities with an independent value:
the energy and norm of functions that the EFE space represents exactly,
computed by a separate fine tensor Gauss rule over the box.  The eigensolver
is pinned by Chebyshev identities, the equivalence of the residual and
standard filters when the overlap inverse is exact, the fixed point of the
residual filter, the stagnation contrast of Sec. III.B, and agreement with a
dense generalized eigensolve."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import eigen, enrich, fe, psp
from paper_2607_06848_amd import workloads as wl

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


# ---------------------------------------------------------------- helpers
def fine_box_rule(L, n=48):
    x, w = np.polynomial.legendre.leggauss(n)
    x = (x + 1) * L / 2
    w = w * L / 2
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1), W


def ho_system(lmax=1, kb=0.0, p=4, nq=10, L=10.0):
    mesh = fe.Mesh((0,) * 3, (L,) * 3, (4,) * 3, p, nq)
    c = L / 2
    prm = dict(xyz=[[c, c, c]], enr_lmax=lmax, enr_alpha=0.5, enr_rcut=40.0, enr_t=0.33,
               kb_width=1.0 if kb else 0.0, kb_D=kb, kb_rcut=40.0)
    s = enrich.EFESystem(mesh, prm)
    s.set_potential(0.5 * np.sum((mesh.quad_coords() - c) ** 2, -1))
    return s


def enrich_vector(s, k, cfe=None):
    """Coefficients of (cfe + phi_k): X^C = cfe + C^T e_k, X^E = e_k."""
    e = np.zeros(s.n_enr)
    e[k] = 1.0
    X = np.zeros(s.rows)
    X[:s.n_nodes] = (s.C.T @ e) + (0 if cfe is None else cfe)
    X[s.n_nodes:] = e
    return X


# ---------------------------------------------------------------- enrichment
def test_cutoff_properties():
    r = np.linspace(0, 7, 701)
    h, dh = enrich.cutoff(r, 6.0, 0.33)
    r0 = 6.0 * 0.33 / 1.33
    assert np.all(h[r <= r0] == 1.0) and np.all(h[r >= 6.0] == 0.0)
    inner = (r > r0) & (r < 6.0)
    assert np.all((h[inner] >= 0) & (h[inner] <= 1))
    assert np.all(h[(r > r0 + 0.5) & (r < 6.0)] < 1)   # below 1 once exp(-1/x) is resolvable
    assert np.all(np.diff(h) <= 1e-15)
    # derivative against central differences
    rr = np.linspace(r0 + 0.05, 5.95, 50)
    e = 1e-6
    fd = (enrich.cutoff(rr + e, 6.0, 0.33)[0] - enrich.cutoff(rr - e, 6.0, 0.33)[0]) / (2 * e)
    assert np.allclose(enrich.cutoff(rr, 6.0, 0.33)[1], fd, atol=1e-7)


def test_solid_harmonic_gradients():
    d = np.random.default_rng(0).normal(size=(20, 3))
    S, G = enrich.solid_harmonics(d, 2)
    e = 1e-6
    for ax in range(3):
        dp = d.copy()
        dp[:, ax] += e
        dm = d.copy()
        dm[:, ax] -= e
        fd = (enrich.solid_harmonics(dp, 2)[0] - enrich.solid_harmonics(dm, 2)[0]) / (2 * e)
        assert np.allclose(G[..., ax], fd, atol=1e-8)


@pytest.fixture(scope="module")
def ho():
    return ho_system(lmax=1)


def test_enrichment_normalized(ho):
    for k in range(ho.n_enr):
        v = enrich_vector(ho, k)
        assert abs(v @ ho.apply_M(v) - 1.0) < 1e-12


def test_oscillator_energy_of_enrichment(ho):
    """The s and p enrichment functions are the oscillator's eigenfunctions;
    their EFE coefficient vectors have Rayleigh quotients 3/2 and 5/2."""
    g = GOLD["harmonic_oscillator_w1"]["levels"]
    for k, want in zip(range(4), (g[0], g[1], g[2], g[3])):
        v = enrich_vector(ho, k)
        rq = (v @ ho.apply_H(v)) / (v @ ho.apply_M(v))
        assert abs(rq - want) < 1e-8, (k, rq)
    # H-orthogonality of the exact eigenfunctions
    vs = enrich_vector(ho, 0)
    vp = enrich_vector(ho, 2)
    assert abs(vs @ ho.apply_H(vp)) < 1e-9


def test_projector_shifts_ground_level():
    g = GOLD["oscillator_ground_state_plus_projector"]
    s = ho_system(lmax=1, kb=g["D"])
    for k, want in ((0, g["s"]), (3, g["p"])):
        v = enrich_vector(s, k)
        rq = (v @ s.apply_H(v)) / (v @ s.apply_M(v))
        assert abs(rq - want) < 1e-8, (k, rq)


def test_cfe_enrichment_cross_terms(ho):
    """<q + phi_s | H | q + phi_s> and the M^E norm for a polynomial q that
    the CFE space holds exactly, against a 48^3-point Gauss rule."""
    L = 10.0
    mesh = ho.mesh
    Xn = mesh.node_coords()

    def qf(X):
        return 64 * X[:, 0] * (L - X[:, 0]) * X[:, 1] * (L - X[:, 1]) * X[:, 2] * (L - X[:, 2]) / L ** 6

    def gq(X):
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        a, b, c = x * (L - x), y * (L - y), z * (L - z)
        return 64 / L ** 6 * np.stack([(L - 2 * x) * b * c, a * (L - 2 * y) * c, a * b * (L - 2 * z)], 1)

    q = qf(Xn) * (1 - mesh.boundary)
    v = enrich_vector(ho, 0, cfe=q)
    P, W = fine_box_rule(L)
    d = P - 5.0
    r2 = np.sum(d * d, 1)
    g0 = np.exp(-r2 / 2)
    phi = g0 / np.sqrt(np.sum(W * g0 * g0))
    gphi = -d * phi[:, None]
    u = qf(P) + phi
    gu = gq(P) + gphi
    E = np.sum(W * (0.5 * np.sum(gu * gu, 1) + 0.5 * r2 * u * u))
    assert abs(v @ ho.apply_H(v) - E) < 1e-8 * abs(E)
    # M^E norm: lumped int q^2 (exact here) + 2 int q phi + int phi^2
    N = np.sum(W * u * u)
    assert abs(v @ ho.apply_M(v) - N) < 1e-8 * N


def test_explicit_blocks_match_transformed_hamiltonian():
    w = wl.make("eig2")
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    s = enrich.EFESystem(mesh, w)
    vq = sum(psp.v_local(np.linalg.norm(mesh.quad_coords() - R, axis=-1), w["Z"],
                         w["loc_rc"], w["loc_amp"], w["loc_rg"]) for R in w["xyz"])
    s.set_potential(vq)
    H = s.dense_HE()
    assert np.abs(H - s.dense_T_Hhat_T()).max() < 1e-12 * np.abs(H).max()
    act = s.active()
    X = np.zeros((s.rows, 3))
    X[act] = np.random.default_rng(0).normal(size=(act.size, 3))
    assert np.abs(s.apply_H(X)[act] - H @ X[act]).max() < 1e-12 * np.abs(H).max()
    # M^E is block diagonal and SPD
    M = s.dense_ME()
    assert np.linalg.eigvalsh(s.Mee).min() > 0


def test_single_atom_tilde_is_exact():
    w = wl.make("eig2")
    w["xyz"] = w["xyz"][:1]
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    s = enrich.EFESystem(mesh, w)
    X = np.random.default_rng(1).normal(size=(s.rows, 2))
    assert np.allclose(s.apply_Minv_tilde(s.apply_M(X))[s.active()], X[s.active()], atol=1e-10)


# ---------------------------------------------------------------- Chebyshev
def test_cheb_recurrence_matches_closed_form():
    a, b, amin, m = 1.0, 30.0, -4.0, 25
    x = np.concatenate([np.linspace(-4, 30, 200), [-3.99, 0.5, 29.9]])
    C = eigen.cheb_scalar(x, a, b, amin, m)
    for k in (1, 2, 7, 25):
        ref = eigen.cheb_closed(x, a, b, amin, k)
        assert np.allclose(C[k], ref, rtol=1e-11, atol=1e-14)
    inside = (x >= amin) & (x <= b)
    assert np.all(np.abs(C[m][inside]) <= 1 + 1e-12)
    assert abs(eigen.cheb_scalar(np.array([amin]), a, b, amin, m)[m][0] - 1.0) < 1e-12


@pytest.fixture(scope="module")
def dense_pair():
    rng = np.random.default_rng(3)
    n = 60
    A = rng.normal(size=(n, n))
    H = A + A.T
    B = rng.normal(size=(n, n))
    M = B @ B.T / n + np.eye(n)
    return H, M


def test_residual_equals_standard_with_exact_inverse(dense_pair):
    H, M = dense_pair
    Mi = np.linalg.inv(M)
    lam, V = sla.eigh(H, M)
    rng = np.random.default_rng(4)
    Vin = V[:, :6] + 1e-2 * rng.normal(size=(60, 6))
    Vin, lam_in, _ = eigen.rayleigh_ritz(lambda X: H @ X, lambda X: M @ X, Vin)
    a, b, amin, m = lam_in[-1], lam[-1] * 1.01, lam_in[0] - 0.1, 12
    out_r = eigen.residual_filter(lambda X: H @ X, lambda X: M @ X, lambda X: Mi @ X,
                                  Vin, lam_in, a, b, amin, m)
    out_s = eigen.standard_filter(lambda X: Mi @ (H @ X), Vin, a, b, amin, m)
    assert np.abs(out_r - out_s).max() < 1e-12 * np.abs(out_s).max()


def test_residual_filter_fixed_point(dense_pair):
    H, M = dense_pair
    lam, V = sla.eigh(H, M)
    Mt_inv = np.diag(1.0 / np.diag(M))            # deliberately inexact
    a, b, amin, m = lam[5], lam[-1] * 1.01, lam[0] - 0.1, 15
    out = eigen.residual_filter(lambda X: H @ X, lambda X: M @ X, lambda X: Mt_inv @ X,
                                V[:, :6], lam[:6], a, b, amin, m)
    ref = V[:, :6] * eigen.cheb_scalar(lam[:6], a, b, amin, m)[m][None, :]
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------- solver
@pytest.fixture(scope="module")
def eig2():
    w = wl.make("eig2")
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    s = enrich.EFESystem(mesh, w)
    vq = sum(psp.v_local(np.linalg.norm(mesh.quad_coords() - R, axis=-1), w["Z"],
                         w["loc_rc"], w["loc_amp"], w["loc_rg"]) for R in w["xyz"])
    s.set_potential(vq)
    ev = eigen.dense_ghep(s)
    v0 = wl.random_vector(s.rows, 7)
    mask = np.zeros(s.rows)
    mask[s.active()] = 1
    b, _, _ = eigen.lanczos_upper_bound(s.apply_H, s.apply_Mtilde, s.apply_Minv_tilde, v0 * mask, 20)
    return w, s, ev, b


def test_lanczos_bound_covers_filtered_operator(eig2):
    w, s, ev, b = eig2
    act = s.active()
    Mt = np.zeros((s.rows, s.rows))
    Mt[act, act] = 1.0
    Mt = s.apply_Mtilde(np.eye(s.rows))[np.ix_(act, act)]
    top = sla.eigh(s.dense_HE(), Mt, eigvals_only=True)[-1]
    assert b >= top
    assert b < 2 * top


def test_stagnation_contrast(eig2):
    """Sec. III.B: with the approximate inverse the standard filter stalls,
    the residual filter converges to round-off; the standard filter with the
    exact inverse also converges."""
    w, s, ev, b = eig2
    V0 = wl.random_block(s.rows, w["nvec"], w["v0_seed"])
    res = {}
    for mode in ("residual", "standard", "standard_exact"):
        V, lam, r, hist = eigen.eigensolve(s, V0, w["degree"], 12, b, mode=mode)
        res[mode] = (r[:4].max(), np.abs(lam[:4] - ev[:4]).max(), V, lam)
    assert res["standard"][0] > 1e-5
    assert res["residual"][0] < 1e-10
    assert res["standard_exact"][0] < 1e-10
    assert res["residual"][1] < 1e-12
    V, lam = res["residual"][2], res["residual"][3]
    S = V.T @ s.apply_M(V)
    assert np.abs(S - np.eye(S.shape[0])).max() < 1e-12


def test_five_pass_solve(eig2):
    """The fixed-potential workload: 5 passes of degree 20 lower every Ritz
    value monotonically and bring the lowest states close to the dense
    solution."""
    w, s, ev, b = eig2
    V0 = wl.random_block(s.rows, w["nvec"], w["v0_seed"])
    V, lam, r, hist = eigen.eigensolve(s, V0, w["degree"], w["passes"], b)
    for (l0, _), (l1, _) in zip(hist[:-1], hist[1:]):
        assert np.all(l1 <= l0 + 1e-12)
    assert np.all(lam >= ev[:w["nvec"]] - 1e-10)
    assert np.abs(lam[:2] - ev[:2]).max() < 1e-3


def test_rayleigh_ritz_on_a_pencil_with_known_spectrum():
    """A pencil built with known eigenvalues d: H = M^(1/2) Q diag(d) Q^T M^(1/2).
    On a mixed basis of an invariant subspace, Rayleigh-Ritz returns exactly
    those eigenvalues, an M-orthonormal basis and zero residuals; on a random
    subspace its Ritz values lie above the eigenvalues of the same index
    (Courant-Fischer)."""
    rng = np.random.default_rng(11)
    n, k = 40, 6
    B = rng.standard_normal((n, n))
    M = B @ B.T + n * np.eye(n)
    w, U = np.linalg.eigh(M)
    Mh = U @ np.diag(np.sqrt(w)) @ U.T
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = np.sort(rng.uniform(-3.0, 5.0, n))
    H = Mh @ Q @ np.diag(d) @ Q.T @ Mh
    X = np.linalg.solve(Mh, Q)          # H X = M X diag(d), X^T M X = I
    V = X[:, :k] @ rng.standard_normal((k, k))
    Vr, lam, res = eigen.rayleigh_ritz(lambda Y: H @ Y, lambda Y: M @ Y, V)
    np.testing.assert_allclose(lam, d[:k], rtol=0, atol=1e-10 * np.abs(d).max())
    np.testing.assert_allclose(Vr.T @ M @ Vr, np.eye(k), atol=1e-10)
    assert res.max() < 1e-8 * np.linalg.norm(H)
    _, lam_r, _ = eigen.rayleigh_ritz(lambda Y: H @ Y, lambda Y: M @ Y,
                                      rng.standard_normal((n, k)))
    assert np.all(lam_r >= d[:k] - 1e-10)
