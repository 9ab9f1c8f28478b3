"""The a0,eff distributions of Table 1 (Wide and Thin beams, any
synchronisation) and the energy distribution of Table 2 (Thin beam, classical
radiation reaction), per sample, as the paper prints them; shared by the oracle
pins and the GPU pins.  Distances in micrometres, a in units of a0.

Readings: z_pm = Delta_par +- L/4 with Delta_par the collision-centre offset
along the axis (c delay / 2); the Thin beam's Table 2 support is gamma_min <=
gamma <= gamma_z (the printed theta(gamma - gamma_z) has the inequality
reversed; the Table 1 support it is derived from fixes it).
"""
import math

import numpy as np
from scipy import integrate

C_SI = 299792458.0
R_E = 2.8179403262e-15


def a_of(z, zR):
    """On-axis a0,eff / a0 at axial distance z from the focus."""
    return 1.0 / math.sqrt(1.0 + (z / zR) ** 2)


def thin_density(a, zR, L, d_par):
    """Table 1, Thin beam: dN/da / N."""
    if not (0.0 < a < 1.0):
        return 0.0
    zp, zm = d_par + L / 4, d_par - L / 4
    ap, am = a_of(zp, zR), a_of(zm, zR)
    sign = 1.0 if d_par < L / 4 else -1.0
    th = (1.0 if a > ap else 0.0) + sign * (1.0 if a > am else 0.0)
    return 2.0 * zR / L / (a * a) / math.sqrt(1.0 - a * a) * th


def wide_density(a, zR, L, d_par, W0, R):
    """Table 1, Wide beam: dN/da / N with n_b = N / (pi R^2 L)."""
    if not (0.0 < a < 1.0):
        return 0.0
    zp, zm = d_par + L / 4, d_par - L / 4
    ap, am = a_of(zp, zR), a_of(zm, zR)
    sign = 1.0 if d_par < L / 4 else -1.0
    nb = 1.0 / (math.pi * R * R * L)

    def lin(z):
        return z / zR * (1.0 + (z / zR) ** 2 / 3.0)

    br = (lin(zp) * (1.0 if ap > a else 0.0) - lin(zm) * (1.0 if am > a else 0.0) +
          math.sqrt(1.0 - a * a) / (3.0 * a) * (2.0 + 1.0 / (a * a)) *
          ((1.0 if a > ap else 0.0) + sign * (1.0 if a > am else 0.0)))
    return 2.0 * math.pi * nb * W0 * W0 * zR / a * br


def c_rr_gauss(lambda_um, tau_fs):
    """eq. PWCRR's c_RR for theta = pi, e^2/(m c^2) = r_e and the Gaussian
    envelope of intensity FWHM tau (eta = (1/2) sqrt(pi / (4 ln 2)))."""
    w0 = 2 * math.pi * C_SI / (lambda_um * 1e-6)
    eta = 0.5 * math.sqrt(math.pi / (4 * math.log(2)))
    return 4.0 * eta / 3.0 * R_E * w0 ** 2 / C_SI * tau_fs * 1e-15


def thin_energy_density(g, g0, a0, c_rr, zR, L):
    """Table 2, Thin beam (synchronised): dN/dgamma / N on gamma_min <= gamma
    <= gamma_z."""
    g_min = g0 / (1 + c_rr * g0 * a0 ** 2)
    a_z = a0 * a_of(L / 4, zR)
    g_z = g0 / (1 + c_rr * g0 * a_z ** 2)
    if not (g_min < g < g_z):
        return 0.0
    q = c_rr * g * g0 * a0 ** 2 + g - g0
    return 2.0 * zR / L * g0 / (g0 - g) ** 1.5 * c_rr * g0 * a0 ** 2 / math.sqrt(q)


def expected_counts(dens, edges, n, breaks=()):
    """n times the integral of dens over each bin, split at the breakpoints
    (the densities' steps and integrable edges)."""
    out = np.zeros(len(edges) - 1)
    for k in range(len(edges) - 1):
        lo, hi = edges[k], edges[k + 1]
        pts = sorted(b for b in breaks if lo < b < hi)
        xs = [lo] + pts + [hi]
        out[k] = n * sum(integrate.quad(dens, xs[j], xs[j + 1], limit=400, epsabs=0,
                                        epsrel=1e-10)[0] for j in range(len(xs) - 1))
    return out
