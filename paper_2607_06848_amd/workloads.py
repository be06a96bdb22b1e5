"""Seeded synthetic inputs shared by the GPU library's callers and the oracle.

This module only draws geometries and random arrays and states the workload
parameters; it holds none of the method's arithmetic.  Both the GPU path and
the CPU oracle receive the same arrays from here.

Workloads (synthetic Gaussian-pseudopotential clusters standing in for the
paper's ONCV-pseudopotential nanoparticles):
  eig2     fixed-potential eigensolve: 10 bohr cube, 4^3 cells p=4, 2 atoms
  c64      64-atom jittered cubic cluster, 16^3 cells p=6, N=160, degree 40
  c500     500-atom cluster (8^3 lattice minus 12 vacancies), 30^3 cells p=6,
           N=1200, degree 50
"""
import numpy as np

PSP = dict(Z=4.0, loc_rc=0.8, loc_amp=1.5, loc_rg=1.2,
           kb_width=0.9, kb_D=0.5, kb_rcut=5.0,
           enr_alpha=0.6, enr_rcut=6.0, enr_t=0.33,
           rho_alpha=1.2)


def two_atoms(seed=1, lo=3.5, hi=6.5, dmin=3.0):
    """Two atoms uniform in [lo, hi]^3, redrawn until at least dmin apart."""
    rng = np.random.default_rng(seed)
    while True:
        x = rng.uniform(lo, hi, size=(2, 3))
        if np.linalg.norm(x[0] - x[1]) >= dmin:
            return x


def jittered_lattice(nside, spacing, sigma, seed):
    """nside^3 simple-cubic lattice (origin at 0) with N(0, sigma^2) jitter."""
    rng = np.random.default_rng(seed)
    g = np.arange(nside) * spacing
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    return pts + rng.normal(0.0, sigma, size=pts.shape)


def remove_vacancies(xyz, nvac, seed):
    rng = np.random.default_rng(seed)
    drop = rng.choice(len(xyz), size=nvac, replace=False)
    keep = np.setdiff1d(np.arange(len(xyz)), drop)
    return xyz[keep]


def perturb(xyz, sigma, seed):
    rng = np.random.default_rng(seed)
    return xyz + rng.normal(0.0, sigma, size=xyz.shape)


def random_block(rows, ncols, seed):
    """V_0 ~ U[-1, 1), row-major (rows, ncols)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(rows, ncols))


def random_block_rows(rows, ncols, seed, chunk_rows):
    """The rows of random_block(rows, ncols, seed) in consecutive chunks of
    chunk_rows (same values: one generator drawn in row-major order)."""
    rng = np.random.default_rng(seed)
    for r0 in range(0, rows, chunk_rows):
        yield r0, rng.uniform(-1.0, 1.0, size=(min(chunk_rows, rows - r0), ncols))


def random_vector(rows, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=rows)


def cluster_box(nside, spacing, vacuum):
    """Cube enclosing the unjittered lattice plus vacuum on each side; the
    lattice is shifted so that the box is [0, L]^3."""
    L = (nside - 1) * spacing + 2 * vacuum
    return L, vacuum


def subcluster(w, center, radius):
    """The workload w restricted to its atoms within `radius` of `center`
    (same mesh and parameters; atoms kept in their original order).  Returns
    (workload, indices of the kept atoms)."""
    xyz = np.asarray(w["xyz"], float)
    keep = np.flatnonzero(np.linalg.norm(xyz - np.asarray(center, float), axis=1) < radius)
    sub = dict(w)
    sub["xyz"] = xyz[keep]
    sub["Zs"] = np.asarray(w["Zs"])[keep]
    return sub, keep


def corner_atom(w):
    """Index of the atom nearest the low corner of the box."""
    xyz = np.asarray(w["xyz"], float)
    return int(np.argmin(np.linalg.norm(xyz - np.asarray(w["lo"], float), axis=1)))


def make(name, **over):
    """Return a dict with mesh parameters, system parameters and solver
    sizes of a named workload."""
    if name == "eig2":
        xyz = two_atoms(over.pop("seed", 1))
        w = dict(lo=(0.0,) * 3, hi=(10.0,) * 3, ncell=(4, 4, 4), p=4, nq=5,
                 xyz=xyz, enr_lmax=1, nvec=8, degree=20, passes=5, v0_seed=5)
    elif name in ("c64", "c500"):
        if name == "c64":
            nside, nc, nvec, deg, seed = 4, 16, 160, 40, 2
        else:
            nside, nc, nvec, deg, seed = 8, 30, 1200, 50, 3
        L, shift = cluster_box(nside, 4.2, 10.0)
        xyz = jittered_lattice(nside, 4.2, 0.15, seed) + shift
        if name == "c500":
            xyz = remove_vacancies(xyz, 12, 4)
        w = dict(lo=(0.0,) * 3, hi=(L,) * 3, ncell=(nc,) * 3, p=6, nq=7,
                 xyz=xyz, enr_lmax=2, nvec=nvec, degree=deg, passes=1, v0_seed=5)
    elif name == "small":
        # a few-atom cluster on a small p=6 mesh: parity cases spanning
        # several tiles with a ragged column tail
        rng_seed = over.pop("seed", 11)
        natoms = over.pop("natoms", 3)
        L = over.pop("L", 12.0)
        nc = over.pop("ncell", 4)
        rng = np.random.default_rng(rng_seed)
        xyz = rng.uniform(0.35 * L, 0.65 * L, size=(natoms, 3))
        w = dict(lo=(0.0,) * 3, hi=(L,) * 3, ncell=(nc,) * 3, p=6, nq=7,
                 xyz=xyz, enr_lmax=2, nvec=37, degree=8, passes=2, v0_seed=5)
    else:
        raise KeyError(name)
    w.update(PSP)
    w.update(over)
    w["Zs"] = np.full(len(w["xyz"]), w["Z"])
    w["name"] = name
    return w
