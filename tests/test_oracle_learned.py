"""Pins of the learned-density oracle against mathematics it must obey."""
import numpy as np
import pytest
from scipy.special import eval_legendre

from oracle import learned as L


def _cluster(seed, natoms=24, box=10.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, box, size=(natoms, 3)), rng.uniform(-1, 11, size=(40, 3))


def test_power_spectrum_addition_theorem():
    """P_nl = (2l+1)/(4 pi) sum_IJ g_n(d_I) g_n(d_J) P_l(u_I . u_J) over the 16
    nearest atoms, found here by a plain sort of (distance, index)."""
    xyz, pts = _cluster(3)
    F = L.descriptors(pts, xyz, np.ones(len(pts)))
    for p, x in enumerate(pts):
        order = sorted(range(len(xyz)), key=lambda i: (float(np.sum((x - xyz[i]) ** 2)), i))[:16]
        vec = x - xyz[order]
        d = np.linalg.norm(vec, axis=1)
        u = vec / d[:, None]
        cos = np.clip(u @ u.T, -1, 1)
        for n in range(8):
            g = np.exp(-0.5 * (d - n) ** 2)
            for l in range(3):
                ref = (2 * l + 1) / (4 * np.pi) * g @ eval_legendre(l, cos) @ g
                assert F[p, 3 * n + l] == pytest.approx(ref, rel=1e-11, abs=1e-14)
    assert np.all(F[:, 24] == 0.0)


def test_rotation_and_permutation_invariance():
    xyz, pts = _cluster(4)
    rho = np.exp(-np.random.default_rng(0).uniform(0, 40, len(pts)))
    F = L.descriptors(pts, xyz, rho)
    Q, _ = np.linalg.qr(np.random.default_rng(1).normal(size=(3, 3)))
    c = np.array([5.0, 5.0, 5.0])
    Fr = L.descriptors((pts - c) @ Q.T + c, (xyz - c) @ Q.T + c, rho)
    np.testing.assert_allclose(Fr, F, rtol=1e-10, atol=1e-13)
    perm = np.random.default_rng(2).permutation(len(xyz))
    Fp = L.descriptors(pts, xyz[perm], rho)
    np.testing.assert_allclose(Fp, F, rtol=1e-12, atol=1e-14)
    assert F[:, 24] == pytest.approx(np.log(np.maximum(rho, 1e-12)))


def test_nearest_atom_ties_by_index():
    # 6 atoms at distance 1, 12 at sqrt(2), 8 at sqrt(3) from the origin, in a
    # shuffled order: the 16 nearest are the 6 + the 10 lowest-index of the 12
    shells = []
    for v in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).reshape(3, -1).T:
        if np.any(v):
            shells.append(v.astype(float))
    xyz = np.array(shells)[np.random.default_rng(5).permutation(26)]
    nb = L.nearest_atoms(np.zeros((1, 3)), xyz)[0]
    d2 = np.sum(xyz ** 2, axis=1)
    want = list(np.flatnonzero(d2 == 1)) + list(np.flatnonzero(d2 == 2)[:10])
    assert list(nb) == want
    assert len(L.nearest_atoms(np.zeros((1, 3)), xyz[:5])[0]) == 5


def test_point_on_atom_and_few_atoms():
    xyz = np.array([[0.0, 0, 0], [2.0, 0, 0]])
    F = L.descriptors(np.array([[0.0, 0, 0]]), xyz, np.array([1.0]))
    # on atom 0 only its l = 0 part survives; atom 1 at d = 2 along x
    for n in range(8):
        g0, g1 = np.exp(-0.5 * n * n), np.exp(-0.5 * (2 - n) ** 2)
        assert F[0, 3 * n] == pytest.approx((g0 + g1) ** 2 / (4 * np.pi))
        assert F[0, 3 * n + 1] == pytest.approx(3 / (4 * np.pi) * g1 ** 2)
        assert F[0, 3 * n + 2] == pytest.approx(5 / (4 * np.pi) * g1 ** 2)


def test_standardization():
    xyz, pts = _cluster(6)
    F = L.descriptors(pts, xyz, np.ones(len(pts)))
    sh, sc = F.mean(0), F.std(0) + 1.0
    np.testing.assert_allclose(L.descriptors(pts, xyz, np.ones(len(pts)), sh, sc),
                               (F - sh) / sc, rtol=0, atol=1e-14)


def test_one_path_network():
    th = np.zeros(L.N_PARAMS)
    W1, b1, W2, b2, W3, b3, W4, b4 = L.unpack(th)
    W1[0, 3] = 1.0
    W2[0, 0] = 1.0
    W3[0, 0] = 1.0
    W4[0, 0] = 2.0
    b4[0] = 0.25
    th = L.pack([W1, b1, W2, b2, W3, b3, W4, b4])
    X = np.random.default_rng(0).normal(size=(9, 25)) * 3
    y, _ = L.forward(th, X)

    def s(z):
        return z / (1.0 + np.exp(-z))
    np.testing.assert_allclose(y, 2 * s(s(s(X[:, 3]))) + 0.25, rtol=1e-14, atol=1e-15)
    assert L.N_PARAMS == 128 * 25 + 128 + 2 * (128 * 128 + 128) + 128 + 1


def test_dsilu_matches_difference_quotient():
    z = np.linspace(-8, 8, 33)
    h = 1e-6
    np.testing.assert_allclose(L.dsilu(z), (L.silu(z + h) - L.silu(z - h)) / (2 * h),
                               rtol=1e-8, atol=1e-10)


def test_gradient_central_differences():
    rng = np.random.default_rng(7)
    th = L.init_params(3)
    X = rng.normal(size=(11, 25))
    t = rng.normal(size=11)
    w = rng.uniform(0.1, 2.0, size=11)

    def f(th_):
        return L.loss(L.forward(th_, X)[0], t, w)
    y, cache = L.forward(th, X)
    g = L.backward(th, X, cache, L.loss_grad(y, t, w))
    offs = np.cumsum([0] + [int(np.prod(s)) for s in L.SHAPES])
    picks = np.concatenate([rng.integers(offs[i], offs[i + 1], 6) for i in range(8)])
    h = 1e-6
    for i in picks:
        e = np.zeros_like(th)
        e[i] = h
        fd = (f(th + e) - f(th - e)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_adam_constant_gradient():
    """With a constant gradient the bias-corrected moments are g and g^2, so
    every step moves theta by lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    m = np.zeros(4)
    v = np.zeros(4)
    for step in range(1, 6):
        new, m, v = L.adam_step(th, g, m, v, step, lr=0.01)
        np.testing.assert_allclose(new - th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)
        th = new


def test_density_guess_renormalizes_and_falls_back():
    rng = np.random.default_rng(9)
    sad = rng.uniform(0, 1, 50)
    wq = rng.uniform(0.1, 1, 50)
    n_el = float(np.sum(wq * sad))
    y = rng.normal(size=50) * 0.05
    rho, fb, fac = L.density_guess(sad, wq, y, 1.0, n_el)
    assert not fb
    assert np.sum(wq * rho) == pytest.approx(n_el, rel=1e-14)
    assert np.all(rho >= 0)
    y2 = y.copy()
    y2[3] = -10.0                                   # clamped to zero
    rho2, fb2, _ = L.density_guess(sad, wq, y2, 1.0, n_el)
    assert not fb2 and rho2[3] == 0.0
    y3 = y.copy()
    y3[0] = np.nan
    rho3, fb3, _ = L.density_guess(sad, wq, y3, 1.0, n_el)
    assert fb3 and np.array_equal(rho3, sad)
    rho4, fb4, fac4 = L.density_guess(sad, wq, np.ones(50), 1.0, n_el)
    assert fb4 and fac4 < 0.9 and np.array_equal(rho4, sad)
