"""Spectral hexahedral finite elements (oracle; test infrastructure only).

The CFE basis of the paper (Sec. II.B) is a tensor-product Lagrange basis on
Gauss-Lobatto-Legendre (GLL) nodes; with the reduced GLL rule the CFE overlap
block is diagonal (Sec. III.A).  Integrals that contain a potential, a
gradient, an enrichment function or a projector use an n_q-point
Gauss-Legendre rule per axis (reading: n_q = 5 for p = 4, n_q = 7 for p = 6).

Index conventions (shared with the GPU tables, which must match bit for bit):
  node   (i, j, k)    -> i + n1x * (j + n1y * k),   n1 = ncell * p + 1
  cell   (cx, cy, cz) -> cx + ncx * (cy + ncy * cz)
  local  (a, b, c)    -> a + (p+1) * (b + (p+1) * c)
  quad   (qa, qb, qc) -> qa + nq * (qb + nq * qc)
  colour of a cell    =  (cx & 1) + 2 (cy & 1) + 4 (cz & 1)
Boundary nodes (any index at 0 or n1-1) carry homogeneous Dirichlet data.
"""
import numpy as np
from numpy.polynomial import legendre as npleg
import scipy.sparse as sp


# ---------------------------------------------------------------- 1-D rules
def gll_rule(p):
    """GLL nodes and weights on [-1, 1] for polynomial order p.

    Nodes: -1, the roots of P_p', +1; weights 2 / (p (p+1) P_p(x)^2)
    (spectral elements with the GLL rule, Sec. III.A).
    """
    cp = np.zeros(p + 1)
    cp[p] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(cp))) if p > 1 else np.zeros(0)
    # one Newton polish of the interior roots on P_p'
    dcp = npleg.legder(cp)
    d2cp = npleg.legder(dcp)
    for _ in range(3):
        if inner.size:
            inner = inner - npleg.legval(inner, dcp) / npleg.legval(inner, d2cp)
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (p * (p + 1) * npleg.legval(x, cp) ** 2)
    return x, w


def gauss_rule(n):
    """n-point Gauss-Legendre nodes and weights on [-1, 1]."""
    x, w = npleg.leggauss(n)
    return np.asarray(x, float), np.asarray(w, float)


def lagrange_basis(nodes, x):
    """Values V[i, a] = L_a(x_i) and derivatives D[i, a] = L_a'(x_i) of the
    Lagrange polynomials on ``nodes`` (plain product formula)."""
    nodes = np.asarray(nodes, float)
    x = np.asarray(x, float)
    n = nodes.size
    V = np.ones((x.size, n))
    D = np.zeros((x.size, n))
    for a in range(n):
        for b in range(n):
            if b != a:
                V[:, a] *= (x - nodes[b]) / (nodes[a] - nodes[b])
        for b in range(n):
            if b == a:
                continue
            t = np.full(x.size, 1.0 / (nodes[a] - nodes[b]))
            for c in range(n):
                if c != a and c != b:
                    t *= (x - nodes[c]) / (nodes[a] - nodes[c])
            D[:, a] += t
    return V, D


# ---------------------------------------------------------------- mesh
class Mesh:
    """Uniform hexahedral mesh of spectral elements on a box.

    Attributes mirror the integer tables of the method (DoF layout of
    Sec. II.B: the CFE nodes first, enrichment rows after).
    """

    def __init__(self, lo, hi, ncell, p, nq):
        self.lo = np.asarray(lo, float)
        self.hi = np.asarray(hi, float)
        self.ncell = np.asarray(ncell, dtype=np.int64)
        self.p = int(p)
        self.nq = int(nq)
        self.P = self.p + 1
        self.nloc = self.P ** 3
        self.nqp = self.nq ** 3
        self.h = (self.hi - self.lo) / self.ncell
        self.n1 = self.ncell * self.p + 1
        self.n_nodes = int(np.prod(self.n1))
        self.n_cells = int(np.prod(self.ncell))
        self._tables()
        self._reference()

    # integer tables ------------------------------------------------------
    def _tables(self):
        P, p = self.P, self.p
        ncx, ncy, ncz = (int(v) for v in self.ncell)
        n1x, n1y, _ = (int(v) for v in self.n1)
        cid = np.arange(self.n_cells, dtype=np.int64)
        cx = cid % ncx
        cy = (cid // ncx) % ncy
        cz = cid // (ncx * ncy)
        self.cell_ijk = np.stack([cx, cy, cz], 1)
        l = np.arange(self.nloc, dtype=np.int64)
        a = l % P
        b = (l // P) % P
        c = l // (P * P)
        gi = cx[:, None] * p + a[None, :]
        gj = cy[:, None] * p + b[None, :]
        gk = cz[:, None] * p + c[None, :]
        self.cell_to_global = (gi + n1x * (gj + n1y * gk)).astype(np.int32)
        colour = (cx & 1) + 2 * (cy & 1) + 4 * (cz & 1)
        self.cell_colour = colour.astype(np.int32)
        order = np.lexsort((cid, colour))          # by colour, then cell id
        self.colour_order = order.astype(np.int32)
        self.colour_offsets = np.searchsorted(colour[order], np.arange(9)).astype(np.int32)
        nid = np.arange(self.n_nodes, dtype=np.int64)
        i = nid % n1x
        j = (nid // n1x) % n1y
        k = nid // (n1x * n1y)
        bnd = ((i == 0) | (i == self.n1[0] - 1) | (j == 0) | (j == self.n1[1] - 1)
               | (k == 0) | (k == self.n1[2] - 1))
        self.boundary = bnd.astype(np.uint8)
        self.interior = np.flatnonzero(~bnd)

    def node_coords(self):
        """Physical coordinates of every node, shape (n_nodes, 3)."""
        xg, _ = gll_rule(self.p)
        nid = np.arange(self.n_nodes, dtype=np.int64)
        n1x, n1y = int(self.n1[0]), int(self.n1[1])
        idx = [nid % n1x, (nid // n1x) % n1y, nid // (n1x * n1y)]
        out = np.empty((self.n_nodes, 3))
        for d in range(3):
            cell = np.minimum(idx[d] // self.p, self.ncell[d] - 1)
            a = idx[d] - cell * self.p
            out[:, d] = self.lo[d] + cell * self.h[d] + (xg[a] + 1.0) * 0.5 * self.h[d]
        return out

    def quad_coords(self, cells=None):
        """Gauss-point coordinates, shape (len(cells), nq^3, 3)."""
        if cells is None:
            cells = np.arange(self.n_cells)
        cells = np.asarray(cells, dtype=np.int64)
        xq, _ = gauss_rule(self.nq)
        q = np.arange(self.nqp)
        qi = [q % self.nq, (q // self.nq) % self.nq, q // (self.nq * self.nq)]
        out = np.empty((cells.size, self.nqp, 3))
        for d in range(3):
            c = self.cell_ijk[cells, d]
            out[:, :, d] = (self.lo[d] + c[:, None] * self.h[d]
                            + (xq[qi[d]][None, :] + 1.0) * 0.5 * self.h[d])
        return out

    # reference element --------------------------------------------------
    def _reference(self):
        xg, wg = gll_rule(self.p)
        xq, wq = gauss_rule(self.nq)
        self.gll_x, self.gll_w = xg, wg
        self.gauss_x, self.gauss_w = xq, wq
        N1, D1 = lagrange_basis(xg, xq)            # (nq, P)
        self.N1, self.D1 = N1, D1
        hx, hy, hz = self.h
        # 3-D tables: row index q (qa fastest), column index l (a fastest)
        self.N3 = np.kron(N1, np.kron(N1, N1))
        self.Gx = np.kron(N1, np.kron(N1, D1)) * (2.0 / hx)
        self.Gy = np.kron(N1, np.kron(D1, N1)) * (2.0 / hy)
        self.Gz = np.kron(D1, np.kron(N1, N1)) * (2.0 / hz)
        self.jac = hx * hy * hz / 8.0
        self.W3 = np.kron(wq, np.kron(wq, wq)) * self.jac
        self.Wgll = np.kron(wg, np.kron(wg, wg)) * self.jac

    # ------------------------------------------------------------ operators
    def lumped_mass(self):
        """Diagonal CFE overlap from the GLL rule, summed over cells
        (spectral elements with the reduced GLL rule, Sec. III.A).
        Boundary entries are kept (they are the mass of the Dirichlet nodes)."""
        m = np.zeros(self.n_nodes)
        np.add.at(m, self.cell_to_global.ravel(),
                  np.tile(self.Wgll, self.n_cells))
        return m

    def stiffness_cell(self):
        """K_cell[l, l'] = int grad N_l . grad N_l' over one cell (Gauss rule);
        identical for every cell of the uniform mesh."""
        W = self.W3[:, None]
        return (self.Gx.T @ (W * self.Gx) + self.Gy.T @ (W * self.Gy)
                + self.Gz.T @ (W * self.Gz))

    def potential_cell(self, vq_cell):
        """V_cell[l, l'] = int v N_l N_l' over one cell, v given at its Gauss
        points."""
        return self.N3.T @ ((self.W3 * vq_cell)[:, None] * self.N3)

    def hamiltonian_cell(self, vq_cell, K=None):
        """Cell Hamiltonian 1/2 K_cell + V_cell of the Kohn-Sham operator
        (-1/2 Laplacian + local potential), Eq. (KS)."""
        if K is None:
            K = self.stiffness_cell()
        return 0.5 * K + self.potential_cell(vq_cell)

    def cells_of_nodes(self, nodes):
        """All cells that contain at least one of ``nodes``."""
        mark = np.zeros(self.n_nodes, bool)
        mark[np.asarray(nodes, dtype=np.int64)] = True
        return np.flatnonzero(mark[self.cell_to_global].any(1))

    def cell_matrices(self, vq, kinetic=0.5, cells=None):
        """kinetic K_cell + V_cell for every cell (or ``cells``)."""
        K = self.stiffness_cell()
        if cells is None:
            cells = np.arange(self.n_cells)
        Hc = np.broadcast_to(kinetic * K, (len(cells),) + K.shape).copy()
        if vq is not None:
            wv = self.W3[None, :] * vq[cells]
            Hc += np.einsum('ql,cq,qm->clm', self.N3, wv, self.N3, optimize=True)
        return Hc

    def cfe_apply(self, vq, X, cells=None, kinetic=0.5, chunk=64, Hc_all=None):
        """Y = sum_c P_c^T (kinetic K_cell + V_cell) P_c X: the assembled CFE
        operator applied cell by cell (definition of FE assembly).

        ``vq`` (n_cells, nq^3) potential at Gauss points (None: no potential);
        boundary rows/columns are dropped (homogeneous Dirichlet).  With
        ``cells`` only those cells are summed (rows of nodes whose cells are
        all included are exact)."""
        X = np.asarray(X, float)
        one = X.ndim == 1
        if one:
            X = X[:, None]
        Xm = X * (1 - self.boundary)[:, None]
        Y = np.zeros_like(Xm)
        if cells is None:
            cells = np.arange(self.n_cells)
        for s in range(0, len(cells), chunk):
            cc = np.asarray(cells[s:s + chunk])
            g = self.cell_to_global[cc]                       # (nc, nloc)
            Xc = Xm[g]                                        # (nc, nloc, N)
            if Hc_all is not None:
                Hc = Hc_all[cc]
            else:
                Hc = self.cell_matrices(vq, kinetic, cc)
            Yc = np.matmul(Hc, Xc)
            np.add.at(Y, g.ravel(), Yc.reshape(-1, Y.shape[1]))
        Y *= (1 - self.boundary)[:, None]
        return Y[:, 0] if one else Y

    def assemble_csr(self, vq, kinetic=0.5):
        """Assembled CFE operator (kinetic K + V) as a CSR matrix over all
        nodes, boundary rows and columns zero.  Small meshes only."""
        K = self.stiffness_cell()
        g = self.cell_to_global.astype(np.int64)
        Hc = np.broadcast_to(kinetic * K, (self.n_cells,) + K.shape).copy()
        if vq is not None:
            Hc += np.einsum('ql,cq,qm->clm', self.N3, self.W3[None, :] * vq, self.N3,
                            optimize=True)
        rows = np.broadcast_to(g[:, :, None], Hc.shape).ravel()
        cols = np.broadcast_to(g[:, None, :], Hc.shape).ravel()
        A = sp.coo_matrix((Hc.ravel(), (rows, cols)),
                          shape=(self.n_nodes, self.n_nodes)).tocsr()
        D = sp.diags((1 - self.boundary).astype(float))
        return (D @ A @ D).tocsr()

    def gather_quad(self, x_nodes):
        """Values at Gauss points of a CFE field given by nodal values,
        shape (n_cells, nq^3)."""
        xm = x_nodes * (1 - self.boundary)
        return xm[self.cell_to_global] @ self.N3.T

    def load_vector(self, fq):
        """f_j = int f N_j (Gauss rule) for a field given at Gauss points;
        boundary entries zero."""
        f = np.zeros(self.n_nodes)
        np.add.at(f, self.cell_to_global.ravel(),
                  ((fq * self.W3[None, :]) @ self.N3).ravel())
        return f * (1 - self.boundary)
