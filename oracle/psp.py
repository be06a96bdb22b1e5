"""Synthetic Gaussian pseudopotential pieces (oracle; test infrastructure).

The paper uses ONCV pseudopotentials (Sec. IV), which are not available here;
the workloads use an analytic stand-in of the same structure (Sec. II.A):
  local part      v_loc(r) = -Z erf(r / r_c) / r + A exp(-(r / r_g)^2)
  smeared charge  b^(I)(r) = -Z exp(-r^2 / r_b^2) / (pi^{3/2} r_b^3),  r_b = r_c
                  (a normalized compact-in-practice unit charge, Eq. EZZbsmear)
  its potential   v_sm(r)  = -Z erf(r / r_b) / r
  so that         v_loc - v_sm = A exp(-(r / r_g)^2)  exactly
  atomic density  rho^(I)  = Z (a_rho / pi)^{3/2} exp(-a_rho r^2)
  atomic potential phi^(I) = Z [erf(sqrt(a_rho) r) - erf(r / r_b)] / r
                  (potential of rho^(I) + b^(I), Sec. III.C)
  KB projector    beta(r)  = (pi w^2)^{-3/4} exp(-r^2 / (2 w^2)), r < r_kb
                  with coupling D (one s channel per atom, Eq. KS v_nl).
"""
import numpy as np
from scipy.special import erf, erfc

SQRT_PI = np.sqrt(np.pi)


def erf_over_r(r, a):
    """erf(r / a) / r with its r -> 0 limit 2 / (a sqrt(pi))."""
    r = np.asarray(r, float)
    x = r / a
    small = x < 1e-6
    safe = np.where(small, 1.0, r)
    return np.where(small, (2.0 / (a * SQRT_PI)) * (1.0 - x * x / 3.0), erf(x) / safe)


def v_local(r, Z, rc, amp, rg):
    """Local pseudopotential of one atom."""
    return -Z * erf_over_r(r, rc) + amp * np.exp(-(np.asarray(r) / rg) ** 2)


def v_short(r, amp, rg):
    """v_loc - v_sm, the short-ranged remainder entering v_eff (Eq. EellocReform)."""
    return amp * np.exp(-(np.asarray(r) / rg) ** 2)


def b_smear(r, Z, rb):
    """Smeared nuclear charge b^(I) (negative, integrates to -Z)."""
    return -Z * np.exp(-(np.asarray(r) / rb) ** 2) / (SQRT_PI ** 3 * rb ** 3)


def rho_atom(r, Z, a_rho):
    """Isolated-atom density of the synthetic atom (integrates to Z)."""
    return Z * (a_rho / np.pi) ** 1.5 * np.exp(-a_rho * np.asarray(r) ** 2)


def phi_atom(r, Z, a_rho, rb):
    """Electrostatic potential of rho^(I) + b^(I) (Sec. III.C)."""
    return Z * (erf_over_r(r, 1.0 / np.sqrt(a_rho)) - erf_over_r(r, rb))


def kb_beta(r, w, rkb):
    """Gaussian s-type Kleinman-Bylander projector, unit L2 norm in R^3,
    set to zero at r >= rkb."""
    r = np.asarray(r, float)
    return np.where(r < rkb, (np.pi * w * w) ** -0.75 * np.exp(-r * r / (2 * w * w)), 0.0)


def gauss_coulomb(R, a, b):
    """Coulomb interaction of two unit-normalized Gaussian charges with
    exponents a, b (densities (a/pi)^{3/2} e^{-a r^2}) at separation R."""
    mu = np.sqrt(a * b / (a + b))
    return erf_over_r(R, 1.0 / mu)


def self_energy(Z, rb):
    """E_self = sum_I 1/2 <b^(I), b^(I)> for the Gaussian smeared charges
    (Eq. EZZbsmear)."""
    Z = np.asarray(Z, float)
    return float(np.sum(Z * Z / (np.sqrt(2 * np.pi) * rb)))


def delta_ezz(R, Z, rb):
    """Point-charge minus smeared-charge repulsion, sum_{I<J} Z_I Z_J
    erfc(R_IJ / (sqrt(2) r_b)) / R_IJ.  The Gaussian charges overlap, so this
    correction makes E_ZZ the point-charge sum of Eq. (Eel)."""
    R = np.asarray(R, float)
    Z = np.asarray(Z, float)
    e = 0.0
    for i in range(len(Z)):
        for j in range(i + 1, len(Z)):
            d = np.linalg.norm(R[i] - R[j])
            e += Z[i] * Z[j] * erfc(d / (np.sqrt(2) * rb)) / d
    return e


def ezz_point(R, Z):
    """Point-charge nuclear repulsion sum_{I<J} Z_I Z_J / R_IJ (Eq. Eel)."""
    R = np.asarray(R, float)
    Z = np.asarray(Z, float)
    e = 0.0
    for i in range(len(Z)):
        for j in range(i + 1, len(Z)):
            e += Z[i] * Z[j] / np.linalg.norm(R[i] - R[j])
    return e
