"""Pins of the synthetic pseudopotential pieces of the oracle (Sec. II.A,
III.C) against what the mathematics fixes: normalizations by radial
quadrature, the radial Poisson equation by finite differences, the
long-range and short-range identities, and the point-charge sum recovered
from the smeared pair interaction; occupations and the entropy term at
their closed-form points."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import psp, scf

Z, RB, A_RHO, AMP, RG = 4.0, 0.8, 1.2, 1.5, 1.2


def radial(f, upper=40.0):
    return quad(lambda r: 4.0 * np.pi * r * r * f(r), 0.0, upper, limit=400,
                epsabs=1e-14, epsrel=1e-13)[0]


def test_atomic_density_and_smeared_charge_normalization():
    assert radial(lambda r: float(psp.rho_atom(r, Z, A_RHO))) == pytest.approx(Z, rel=1e-12)
    assert radial(lambda r: float(psp.b_smear(r, Z, RB))) == pytest.approx(-Z, rel=1e-12)


def test_projector_unit_norm_inside_its_cut():
    # exp(-r^2/w^2) at the 5-bohr cut is ~4e-14: the cut loses nothing measurable
    n = radial(lambda r: float(psp.kb_beta(r, 0.9, 5.0)) ** 2, upper=5.0)
    assert n == pytest.approx(1.0, abs=1e-11)
    assert float(psp.kb_beta(5.0, 0.9, 5.0)) == 0.0


def test_atomic_potential_solves_the_radial_poisson_equation():
    """-(1/r) d^2(r phi)/dr^2 = 4 pi (rho^(I) + b^(I)), by central differences."""
    h = 1e-3
    for r in (0.3, 0.7, 1.5, 3.0):
        u = lambda x: x * float(psp.phi_atom(x, Z, A_RHO, RB))
        lap = -(u(r + h) - 2.0 * u(r) + u(r - h)) / (h * h) / r
        src = 4.0 * np.pi * float(psp.rho_atom(r, Z, A_RHO) + psp.b_smear(r, Z, RB))
        assert lap == pytest.approx(src, rel=2e-5, abs=1e-8)
    # the pair is neutral: no Coulomb tail; finite value at the nucleus
    assert abs(float(psp.phi_atom(20.0, Z, A_RHO, RB))) < 1e-12
    phi0 = Z * (2.0 * np.sqrt(A_RHO / np.pi) - 2.0 / (RB * np.sqrt(np.pi)))
    assert float(psp.phi_atom(0.0, Z, A_RHO, RB)) == pytest.approx(phi0, rel=1e-12)


def test_local_potential_identities():
    r = np.array([0.05, 0.4, 1.0, 2.5, 6.0])
    v = psp.v_local(r, Z, RB, AMP, RG)
    v_sm = -Z * psp.erf_over_r(r, RB)
    np.testing.assert_allclose(v - v_sm, psp.v_short(r, AMP, RG), rtol=1e-13, atol=1e-15)
    # Coulomb tail of the ion
    assert float(psp.v_local(12.0, Z, RB, AMP, RG)) == pytest.approx(-Z / 12.0, rel=1e-14)


def test_point_charge_sum_from_smeared_pairs():
    """Two Gaussian smeared charges of width r_b interact through
    erf(R / (sqrt(2) r_b)) / R (gauss_coulomb with exponents 1/r_b^2); adding
    delta_ezz must give the point-charge sum for any geometry."""
    rng = np.random.default_rng(3)
    R = rng.uniform(0.0, 6.0, size=(5, 3))
    Zs = rng.uniform(1.0, 5.0, size=5)
    a = 1.0 / RB ** 2
    smeared = 0.0
    for i in range(5):
        for j in range(i + 1, 5):
            smeared += Zs[i] * Zs[j] * float(psp.gauss_coulomb(np.linalg.norm(R[i] - R[j]), a, a))
    assert smeared + psp.delta_ezz(R, Zs, RB) == pytest.approx(psp.ezz_point(R, Zs), rel=1e-13)


def test_occupations_and_entropy_closed_forms():
    kT, mu = 1e-3, -0.2
    assert float(scf.occupations(mu, mu, kT)) == pytest.approx(0.5, abs=1e-15)
    x = np.array([0.3, 1.0, 4.0]) * kT
    np.testing.assert_allclose(scf.occupations(mu + x, mu, kT),
                               1.0 - scf.occupations(mu - x, mu, kT), atol=1e-15)
    # half-filled levels carry k ln 2 each (x 2 for spin); full and empty none
    assert scf.entropy_term(np.full(3, 0.5), kT) == pytest.approx(6.0 * kT * np.log(2.0),
                                                                  rel=1e-14)
    assert scf.entropy_term(np.array([0.0, 1.0, 1.0]), kT) == 0.0
