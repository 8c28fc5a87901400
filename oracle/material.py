"""Temperature-dependent material law (paper Section 2.1-2.2).

The thermal model is rho c dT/dt + chi rho d f_pc/dt - div(kappa grad T) = Q
(Section 2.1, the thermal-model equation).  Written in enthalpy form the two
time-derivative terms are dH/dt with

    H(T) = rho * int_{T_lo}^{T} c(s) ds + rho * chi * f_pc(T),

so H'(T) = rho c(T) + rho chi f_pc'(T).

Readings (the paper gives IN625 tables only as a stripped figure):
  * c(T) and kappa(T) are linear between T_lo and T_hi and constant outside
    that range; the paper states that values beyond its plotted range are
    held constant (Section 2.2).
  * f_pc is the sigmoid 1/2 [1 + tanh(S (T - T_m))], T_m = (T_sol+T_liq)/2,
    with sharpness S in 1/K.  The printed 2D formula (Section 5.1) has no T
    in it and reads like a derivative; the sigmoid behaviour it names
    (Section 2.1) is this function.
  * rho is constant (Section 2.2 takes a constant density).
"""
import numpy as np


def heat_capacity(T, mat):
    """c(T): linear from c_lo at T_lo to c_hi at T_hi, clamped outside."""
    Tc = np.clip(T, mat.T_lo, mat.T_hi)
    return mat.c_lo + (mat.c_hi - mat.c_lo) * (Tc - mat.T_lo) / (mat.T_hi - mat.T_lo)


def conductivity(T, mat):
    """kappa(T): linear from k_lo at T_lo to k_hi at T_hi, clamped outside."""
    Tc = np.clip(T, mat.T_lo, mat.T_hi)
    return mat.k_lo + (mat.k_hi - mat.k_lo) * (Tc - mat.T_lo) / (mat.T_hi - mat.T_lo)


def phase_fraction(T, mat):
    """f_pc(T) = 1/2 [1 + tanh(S (T - T_m))]."""
    if mat.pc_kind != 0:
        raise ValueError("only the tanh sigmoid phase-change law is supported")
    Tm = 0.5 * (mat.T_sol + mat.T_liq)
    return 0.5 * (1.0 + np.tanh(mat.sharpness * (T - Tm)))


def phase_fraction_slope(T, mat):
    """f_pc'(T) = S/2 [1 - tanh^2(S (T - T_m))]."""
    Tm = 0.5 * (mat.T_sol + mat.T_liq)
    th = np.tanh(mat.sharpness * (T - Tm))
    return 0.5 * mat.sharpness * (1.0 - th * th)


def sensible_integral(T, mat):
    """int_{T_lo}^{T} c(s) ds for the clamped linear c, piece by piece."""
    T = np.asarray(T, dtype=np.float64)
    slope = (mat.c_hi - mat.c_lo) / (mat.T_hi - mat.T_lo)
    below = mat.c_lo * (T - mat.T_lo)
    u = T - mat.T_lo
    inside = mat.c_lo * u + 0.5 * slope * u * u
    full = 0.5 * (mat.c_lo + mat.c_hi) * (mat.T_hi - mat.T_lo)
    above = full + mat.c_hi * (T - mat.T_hi)
    return np.where(T < mat.T_lo, below, np.where(T > mat.T_hi, above, inside))


def enthalpy(T, mat):
    """Volumetric enthalpy H(T) in J/m^3 (zero at T_lo apart from the tiny
    latent tail of the sigmoid)."""
    return mat.rho * (sensible_integral(T, mat) + mat.latent * phase_fraction(T, mat))


def enthalpy_slope(T, mat):
    """dH/dT = rho c(T) + rho chi f_pc'(T)."""
    return mat.rho * (heat_capacity(T, mat) + mat.latent * phase_fraction_slope(T, mat))
