"""The seeded synthetic inputs have the shapes the workload recipe states:
atom counts, lattice spacing and jitter, vacuum, mesh sizes and node counts,
and the chunked block generator reproduces the whole-block one."""
import numpy as np
import pytest

from paper_2607_06848_amd import workloads as wl


def nodes(w):
    return int(np.prod([c * w["p"] + 1 for c in w["ncell"]]))


def test_two_atom_workload():
    w = wl.make("eig2")
    x = np.asarray(w["xyz"])
    assert x.shape == (2, 3)
    assert np.all((x >= 3.5) & (x <= 6.5))
    assert np.linalg.norm(x[0] - x[1]) >= 3.0
    assert w["hi"] == (10.0,) * 3 and w["ncell"] == (4, 4, 4) and w["p"] == 4 and w["nq"] == 5
    assert nodes(w) == 4913
    assert (w["nvec"], w["degree"], w["passes"], w["enr_lmax"]) == (8, 20, 5, 1)


@pytest.mark.parametrize("name,natoms,nside,ncell,n_nodes,nvec,degree",
                         [("c64", 64, 4, 16, 912673, 160, 40),
                          ("c500", 500, 8, 30, 5929741, 1200, 50)])
def test_clusters(name, natoms, nside, ncell, n_nodes, nvec, degree):
    w = wl.make(name)
    x = np.asarray(w["xyz"])
    assert x.shape == (natoms, 3)
    L = (nside - 1) * 4.2 + 20.0                    # 10 bohr of vacuum on each side
    assert w["hi"] == pytest.approx((L,) * 3)
    assert w["ncell"] == (ncell,) * 3 and w["p"] == 6 and w["nq"] == 7
    assert nodes(w) == n_nodes
    assert (w["nvec"], w["degree"], w["enr_lmax"]) == (nvec, degree, 2)
    # each atom sits within a few jitter widths of a lattice site 4.2 apart
    site = np.round((x - 10.0) / 4.2)
    d = x - (10.0 + 4.2 * site)
    assert np.all((site >= 0) & (site < nside))
    assert len({tuple(s) for s in site.astype(int)}) == natoms
    assert np.abs(d).max() < 5 * 0.15
    assert np.std(d) == pytest.approx(0.15, rel=0.2)
    assert np.all(w["Zs"] == 4.0)


def test_chunked_block_matches_whole_block():
    whole = wl.random_block(1000, 7, 5)
    parts = np.concatenate([b for _, b in wl.random_block_rows(1000, 7, 5, 128)])
    assert np.array_equal(whole, parts)
    assert whole.min() >= -1.0 and whole.max() < 1.0
