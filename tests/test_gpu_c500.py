"""500-atom cluster (30^3 cells, p = 6, 5.93e6 rows): one H^E apply of an
8-column chunk on the GPU against the oracle, element by element.

The oracle cannot hold the whole system (its enrichment tables took more than
55 GB at setup before it was stopped).  The apply is linear and local, so the
test feeds an input supported near one atom and gives the oracle only the
atoms that can reach it:
  X^C random on the interior nodes within 3 bohr of the corner atom,
  X^E random on the corner atom's rows, zero elsewhere.
Then (T X)^C lives on the corner atom's support and the ball; a projector
touches it only if its atom is within 6 + 5 bohr plus two cell diagonals
(16.7 bohr) of the corner atom.  With every atom within 18 bohr in the
oracle (64 atoms), H^E X is exact on every CFE row and on the enrichment rows
of those 64 atoms; the GPU runs the full 500-atom system.  The oracle's cell
sums run over the cells where (T X)^C is non-zero (exact, see
EFESystem.apply_H)."""
import numpy as np
import pytest

from paper_2607_06848_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-c500]", *a, flush=True)


def _potential(mesh, w, sub, center, radius=30.0):
    """Local pseudopotential of the oracle's atoms at the Gauss points of the
    cells within `radius` of `center`, zero elsewhere (an input shared by
    both sides)."""
    from oracle import psp
    vq = np.zeros((mesh.n_cells, mesh.nqp))
    cc = (mesh.cell_ijk + 0.5) * mesh.h[None, :] + mesh.lo[None, :]
    cells = np.flatnonzero(np.linalg.norm(cc - center, axis=1) < radius)
    X = mesh.quad_coords(cells)
    v = np.zeros(X.shape[:2])
    for R in sub["xyz"]:
        v += psp.v_local(np.linalg.norm(X - R, axis=-1), w["Z"], w["loc_rc"], w["loc_amp"],
                         w["loc_rg"])
    vq[cells] = v
    return vq


@pytest.mark.timeout(900)
def test_apply_c500_chunk():
    from oracle import enrich, fe
    from paper_2607_06848_amd import efe
    w = wl.make("c500")
    ic = wl.corner_atom(w)
    c = np.asarray(w["xyz"])[ic]
    sub, keep = wl.subcluster(w, c, 18.0)
    _say("oracle atoms", len(keep), "of", len(w["xyz"]))
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    s = enrich.EFESystem(mesh, sub)
    _say("oracle system built")
    vq = _potential(mesh, w, sub, c)
    s.set_potential(vq)
    # the input: random near the corner atom (seeded), zero elsewhere
    xn = mesh.node_coords()
    near = np.flatnonzero((np.linalg.norm(xn - c, axis=1) < 3.0) & (mesh.boundary == 0))
    rng = np.random.default_rng(17)
    ncols = 8
    XC = rng.uniform(-1.0, 1.0, (near.size, ncols))
    XEc = rng.uniform(-1.0, 1.0, (s.nf, ncols))
    j = int(np.flatnonzero(keep == ic)[0])
    Xo = np.zeros((s.rows, ncols))
    Xo[near] = XC
    Xo[s.n_nodes + j * s.nf:s.n_nodes + (j + 1) * s.nf] = XEc
    CtXE = s.C.T @ Xo[s.n_nodes:]
    nodes = np.union1d(near, np.flatnonzero(np.abs(CtXE).sum(1) > 0))
    cells = mesh.cells_of_nodes(nodes)
    _say("input nodes", nodes.size, "cells", cells.size)
    Yo = s.apply_H(Xo, cells=cells)
    _say("oracle apply done")
    ctx = efe.Context(w)
    nf = s.nf
    assert ctx.rows == mesh.n_nodes + len(w["xyz"]) * nf
    ctx.set_potential(torch.from_numpy(vq.ravel()).cuda())
    Xg = torch.zeros((ctx.rows, ncols), dtype=torch.float64, device="cuda")
    Xg[torch.from_numpy(near).cuda()] = torch.from_numpy(XC).cuda()
    Xg[ctx.n_nodes + ic * nf:ctx.n_nodes + (ic + 1) * nf] = torch.from_numpy(XEc).cuda()
    Yg = ctx.apply_H(Xg)
    torch.cuda.synchronize()
    YC = Yg[:ctx.n_nodes].cpu().numpy()
    rows_e = (ctx.n_nodes + keep[:, None] * nf + np.arange(nf)[None, :]).ravel()
    YE = Yg[torch.from_numpy(rows_e).cuda()].cpu().numpy()
    ctx.close()
    scale = np.abs(Yo).max()
    eC = np.abs(YC - Yo[:s.n_nodes]).max() / scale
    eE = np.abs(YE - Yo[s.n_nodes:]).max() / scale
    nzE = np.count_nonzero(np.abs(Yo[s.n_nodes:]).max(1) > 1e-12 * scale)
    _say("CFE rows rel err", eC, "enrichment rows rel err", eE, "non-zero enrichment rows",
         nzE, "non-zero CFE rows", np.count_nonzero(np.abs(Yo[:s.n_nodes]).max(1)))
    assert nzE > 9 * 8               # the input reaches many atoms' rows
    assert eC < 1e-12
    assert eE < 1e-12
