"""Pins of the oracle's finite-element layer against mathematics that does not
come from the oracle itself: quadrature exactness, interpolation identities,
closed-form Laplacian and oscillator spectra, table invariants."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fe

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_gll_rule_exactness(p):
    x, w = fe.gll_rule(p)
    assert x[0] == -1.0 and x[-1] == 1.0
    assert np.allclose(x, -x[::-1], atol=1e-15)
    for k in range(2 * p):            # exact through degree 2p-1
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14
    k = 2 * p                          # not exact at degree 2p
    assert abs(np.sum(w * x ** k) - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("n", [3, 5, 7, 10])
def test_gauss_rule_exactness(n):
    x, w = fe.gauss_rule(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14


@pytest.mark.parametrize("p", [4, 6])
def test_lagrange_identities(p):
    xg, _ = fe.gll_rule(p)
    V, D = fe.lagrange_basis(xg, xg)
    assert np.allclose(V, np.eye(p + 1), atol=1e-14)
    t = np.linspace(-1, 1, 17)
    V, D = fe.lagrange_basis(xg, t)
    assert np.allclose(V.sum(1), 1.0, atol=1e-13)
    assert np.allclose(D.sum(1), 0.0, atol=1e-11)
    for k in range(p + 1):             # interpolation of x^k is exact
        assert np.allclose(V @ xg ** k, t ** k, atol=1e-12)
        assert np.allclose(D @ xg ** k, k * t ** max(k - 1, 0) if k else 0 * t, atol=1e-10)


def test_mesh_tables_invariants():
    m = fe.Mesh((0, 0, 0), (3.0, 4.0, 5.0), (3, 4, 5), 3, 4)
    n1 = np.array([10, 13, 16])
    assert m.n_nodes == np.prod(n1)
    assert m.cell_to_global.shape == (60, 64)
    # multiplicity: every node is shared by 1, 2, 4 or 8 cells
    cnt = np.bincount(m.cell_to_global.ravel(), minlength=m.n_nodes)
    assert set(np.unique(cnt)) <= {1, 2, 4, 8}
    assert cnt.sum() == 60 * 64
    # each colour class is conflict-free (brute force)
    for col in range(8):
        cells = m.colour_order[m.colour_offsets[col]:m.colour_offsets[col + 1]]
        nodes = m.cell_to_global[cells].ravel()
        assert np.unique(nodes).size == nodes.size
        assert np.all(m.cell_colour[cells] == col)
        assert np.all(np.diff(cells) > 0)
    assert m.colour_offsets[-1] == 60
    assert int(m.boundary.sum()) == np.prod(n1) - np.prod(n1 - 2)
    # node (i,j,k) of cell (cx,cy,cz), local (a,b,c)
    cx, cy, cz, a, b, c = 2, 1, 3, 1, 3, 2
    cell = cx + 3 * (cy + 4 * cz)
    loc = a + 4 * (b + 4 * c)
    i, j, k = cx * 3 + a, cy * 3 + b, cz * 3 + c
    assert m.cell_to_global[cell, loc] == i + 10 * (j + 13 * k)


def test_lumped_mass_volume():
    m = fe.Mesh((0, 0, 0), (3.0, 4.0, 5.0), (3, 4, 5), 4, 5)
    assert abs(m.lumped_mass().sum() - 60.0) < 1e-11


def test_stiffness_kernel_and_quadratic_energy():
    L = 4.0
    m = fe.Mesh((0, 0, 0), (L, L, L), (2, 2, 2), 4, 5)
    K = m.stiffness_cell()
    assert np.abs(K.sum(1)).max() < 1e-12           # K . 1 = 0
    # q = x(L-x) + 2 y^2 - z: int |grad q|^2 over the box in closed form
    X = m.node_coords()
    q = X[:, 0] * (L - X[:, 0]) + 2 * X[:, 1] ** 2 - X[:, 2]
    # assemble K without the Dirichlet mask: sum over cells of q_c^T K q_c
    qc = q[m.cell_to_global]
    e_num = np.einsum('cl,lm,cm->', qc, K, qc)
    e_exact = (L ** 2 * (L ** 3 / 3.0)          # int (L - 2x)^2 = L^3/3, times L^2
               + 16 * L ** 2 * (L ** 3 / 3.0)    # int (4y)^2
               + L ** 3)                         # int 1
    assert abs(e_num - e_exact) < 1e-10 * e_exact


def _lowest_levels(mesh, vq, k):
    A = mesh.assemble_csr(vq)
    I = mesh.interior
    d = 1.0 / np.sqrt(mesh.lumped_mass()[I])
    S = sp.diags(d) @ A[I][:, I] @ sp.diags(d)
    return np.sort(spla.eigsh(S.tocsc(), k=k, sigma=-1.0, which="LM",
                              return_eigenvectors=False))


def test_box_laplacian_levels():
    g = GOLD["box_laplacian_L10"]
    mesh = fe.Mesh((0,) * 3, (g["L"],) * 3, (4,) * 3, 4, 5)
    ev = _lowest_levels(mesh, None, 5)
    assert abs(ev[0] - g["levels"][0]) < 1e-8
    assert np.allclose(ev[1:4], g["levels"][1:4], atol=1e-6)
    assert abs(ev[4] - g["levels"][4]) < 1e-5


def test_harmonic_oscillator_levels_converge():
    g = GOLD["harmonic_oscillator_w1"]
    errs = []
    for p in (4, 5):
        mesh = fe.Mesh((0,) * 3, (10.0,) * 3, (4,) * 3, p, p + 1)
        vq = 0.5 * np.sum((mesh.quad_coords() - 5.0) ** 2, -1)
        ev = _lowest_levels(mesh, vq, 4)
        errs.append(np.abs(ev - g["levels"][:4]).max())
    assert errs[1] < errs[0] / 5
    assert errs[1] < 1e-3


def test_support_cells_against_sampled_boxes():
    """Support cells of a sphere, checked cell by cell by the nearest of a
    dense grid of points in each cell box: a cell whose sampled distance is
    below r_c - (sampling error) must be listed, one whose sampled distance
    exceeds r_c + (sampling error) must not."""
    from oracle import enrich
    m = fe.Mesh([0.0, 0.0, 0.0], [10.0, 8.0, 9.0], [5, 4, 6], 2, 3)
    rng = np.random.default_rng(7)
    for _ in range(3):
        center = rng.uniform([1.0, 1.0, 1.0], [9.0, 7.0, 8.0])
        rc = rng.uniform(1.5, 4.0)
        got = set(enrich.support_cells(m, center, rc).tolist())
        s = np.linspace(0.0, 1.0, 21)
        P = np.stack(np.meshgrid(s, s, s, indexing="ij"), -1).reshape(-1, 3)
        err = 0.5 * np.linalg.norm(np.asarray(m.h, float)) / 20.0   # half a sample diagonal
        for cid in range(m.n_cells):
            cx = cid % 5
            cy = (cid // 5) % 4
            cz = cid // 20
            lo = np.asarray(m.lo, float) + np.array([cx, cy, cz]) * np.asarray(m.h, float)
            pts = lo + P * np.asarray(m.h, float)
            dmin = np.linalg.norm(pts - center, axis=1).min()
            if dmin < rc - err:
                assert cid in got, (cid, dmin, rc)
            if dmin - err > rc:
                assert cid not in got, (cid, dmin, rc)
