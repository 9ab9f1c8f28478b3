"""Pins of the oracle's photon spectrum (Sec. 4: the LCFA quantum-synchrotron
spectrum of every (gamma, a) pair along the phase, integrated over it).

  - total photon number per unit chi at small chi: from the Mellin integrals
    Int_0^inf K_{2/3} = pi, Int_0^inf y K_{2/3} = 2 pi / (3 sqrt3),
    Int_0^inf Int_y^inf K_{1/3} = pi / 3, Int_0^inf y Int_y^inf K_{1/3} =
    4 pi / (9 sqrt3), the number Phi(1; chi) = (5 pi / 2) chi (1 - 8 chi / (5 sqrt3)
    + O(chi^2));
  - the soft end: Phi(xi; chi) -> 3 Gamma(2/3) (3 chi)^(2/3) xi^(1/3) as xi / chi -> 0
    (K_{2/3}(y) -> Gamma(2/3) / 2 (y/2)^(-2/3));
  - the first and second xi-moments of the spectrum are the Gaunt factor g
    and h of the drift and diffusion (their definitions), computed here from
    the CDF table, against the radiation-function table (a different
    quadrature of the same integrals);
  - in the classical model the emitted photon energy equals the electrons'
    energy loss exactly (the stage quadrature of the spectrum is the one that
    advances the mean energy);
  - bin masses are CDF differences: merging neighbouring bins of a finer
    histogram gives the coarser one.
"""
import math

import numpy as np
import pytest

from paper_2308_09348_amd import workloads


def test_photon_number_small_chi(oracle):
    for chi, tol in ((1e-6, 1e-9), (1e-5, 1e-8), (1e-4, 1e-7)):
        _, tot = oracle.photon_cdf(0.5, chi)
        expect = 5 * math.pi / 2 * chi * (1 - 8 * chi / (5 * math.sqrt(3)))
        assert abs(tot / expect - 1) <= tol, (chi, tot / expect - 1)


def test_photon_soft_end(oracle):
    for chi in (1e-3, 0.1, 3.0):
        for r in (1e-9, 1e-8):
            xi = r * chi
            phi, _ = oracle.photon_cdf(xi, chi)
            lead = 3 * math.gamma(2 / 3) * (3 * chi) ** (2 / 3) * xi ** (1 / 3)
            assert abs(phi / lead - 1) <= 50 * r ** (2 / 3), (chi, r, phi / lead)


def _moments(oracle, chi):
    """Int xi dPhi and Int xi^2 dPhi by parts over z = y^(1/3)."""
    zmax = 80.0 ** (1 / 3)
    z = np.linspace(0.0, zmax, 8193)
    y = z ** 3
    q = 2 + 3 * chi * y
    xi = 3 * chi * y / q
    dxi = 6 * chi / q ** 2 * 3 * z ** 2  # dxi/dz
    phi = np.array([oracle.photon_cdf(x, chi)[0] for x in xi])
    _, N = oracle.photon_cdf(0.5, chi)
    dz = z[1] - z[0]
    wts = np.full(z.size, 2.0)
    wts[1::2] = 4.0
    wts[0] = wts[-1] = 1.0
    simpson = lambda f: dz / 3 * np.dot(wts, f)
    xe = xi[-1]  # beyond y = 80 the CDF equals N
    m1 = N * xe - simpson(phi * dxi)
    m2 = N * xe ** 2 - 2 * simpson(phi * xi * dxi)
    return m1, m2


@pytest.mark.parametrize("chi", [1e-3, 0.05, 0.7, 4.0, 40.0])
def test_photon_moments_are_g_and_h(oracle, chi):
    m1, m2 = _moments(oracle, chi)
    g, _, _, h = oracle.radiation(chi)
    assert abs(m1 / (2 * math.pi * chi ** 2 / math.sqrt(3) * g) - 1) <= 1e-6, chi
    assert abs(m2 / (55 * math.pi * chi ** 3 / 24 * h) - 1) <= 1e-6, chi


def _photon_case(rr, amp, **kw):
    p = workloads.scaled(workloads.focused_3d(), n_samples=60, n_steps=256, rr_model=rr,
                         amp_mode=amp)
    p.update(kw)
    return p


@pytest.mark.parametrize("amp", ["local", "a0eff"])
def test_classical_photon_energy_is_electron_loss(oracle, amp):
    p = _photon_case("classical", amp)
    h, e = oracle.photons(p, 64, 0.0, 1.2 * p["gamma0"])
    assert e[0] > 0
    assert abs(e[0] - e[1]) <= 1e-12 * e[1], (e, e[0] / e[1] - 1)
    pw = workloads.scaled(workloads.plane_wave_1d(), n_samples=40, n_steps=256)
    h, e = oracle.photons(pw, 64, 0.0, 1.2 * pw["gamma0"])
    assert abs(e[0] - e[1]) <= 1e-12 * e[1]


def test_quantum_electron_loss_exceeds_photon_energy(oracle):
    """Quantum moments: the electron's mean loss adds -A''/2 sig2 > 0 to the
    drift that the spectrum integrates, a small positive excess."""
    p = _photon_case("quantum", "local")
    _, e = oracle.photons(p, 64, 0.0, 1.2 * p["gamma0"])
    assert 0 < e[1] - e[0] <= 5e-2 * e[0]


def test_photon_bins_merge(oracle):
    p = _photon_case("quantum", "local", n_samples=20)
    h1, _ = oracle.photons(p, 40, 5.0, 2405.0)
    h2, _ = oracle.photons(p, 80, 5.0, 2405.0)
    merged = h2[:80].reshape(40, 2).sum(1)
    assert np.allclose(merged, h1[:40], rtol=1e-12, atol=1e-15 * h1.sum())
    assert abs(h2[80] - h1[40]) <= 1e-12 * h1.sum() and abs(h2[81] - h1[41]) <= 1e-12 * h1.sum()


def test_photon_spectrum_energy(oracle):
    """The histogram's energy at bin centres approaches the emitted photon
    energy as the bins shrink; the error is dominated by the soft end, where
    dN/d(eps) ~ eps^(-2/3) puts an O(width^(4/3)) error in the first bin."""
    p = _photon_case("quantum", "local", n_samples=20)
    top = 1.01 * p["gamma0"] * 1.3
    errs = []
    for n in (3000, 12000):
        h, e = oracle.photons(p, n, 0.0, top)
        mid = (np.arange(n) + 0.5) * top / n
        assert h[n + 1] == 0.0  # no photon above the electron energy
        errs.append(np.dot(mid, h[:n]) / e[0] - 1)
    assert 0 < errs[1] <= 3e-4
    assert abs(errs[0] / errs[1] / 4 ** (4 / 3) - 1) <= 0.2, errs


def test_no_field_no_photons(oracle):
    p = _photon_case("quantum", "local", a0=0.0)
    h, e = oracle.photons(p, 32, 0.0, 3000.0)
    assert np.all(h == 0.0) and e[0] == 0.0 and e[1] == 0.0


# ---- Sec. 5.1: photon angular moments ---------------------------------------

def test_photon_angles_plane_wave_closed_form(oracle):
    """Classical plane wave, one energy: 1/mu(psi) = 1/gamma0 + K Int a^2 (the
    exact Landau-Lifshitz solution), photon number rate C_ph (5 pi / 2) (2|a|/a_S)
    (1 - 8 chi/(5 sqrt3)) (the small-chi number, chi ~ 2e-3 here), energy rate
    K a^2 mu^2; angles (a/mu, 0) with a 1/mu cone.  Fine Simpson quadrature in
    psi against the oracle's RK4 stage sums."""
    import math
    from scipy import integrate
    p = workloads.scaled(workloads.plane_wave_1d(), n_samples=4, n_steps=2048, sigma_gamma=0.0,
                         a0=2.0, gamma0=200.0)
    d = oracle.derived(p)
    aS, K, psim = d["aS"], d["K"], d["psi_max"]
    otau = d["omega0"] * p["tau_fs"]
    c_ph = 7.2973525693e-3 * aS / (2 * math.sqrt(3) * math.pi)
    psi = np.linspace(-psim, psim, 2_000_001)
    a = p["a0"] * np.exp(-2 * math.log(2) * (psi / otau) ** 2) * np.cos(psi)
    mu = 1.0 / (1.0 / p["gamma0"] + K * integrate.cumulative_trapezoid(a * a, psi, initial=0))
    chi = 2 * mu * np.abs(a) / aS
    dN = c_ph / mu * (5 * math.pi / 2) * chi * (1 - 8 * chi / (5 * math.sqrt(3)))
    dE = K * a * a * mu * mu
    x2, y2 = (a / mu) ** 2 + 1 / mu ** 2, 1 / mu ** 2
    N, E = integrate.simpson(dN, x=psi), integrate.simpson(dE, x=psi)
    ref = np.array([N, 1e3 * math.sqrt(integrate.simpson(dN * x2, x=psi) / N),
                    1e3 * math.sqrt(integrate.simpson(dN * y2, x=psi) / N), E,
                    1e3 * math.sqrt(integrate.simpson(dE * x2, x=psi) / E),
                    1e3 * math.sqrt(integrate.simpson(dE * y2, x=psi) / E)])
    o = oracle.photon_angles(p) / np.array([4, 1, 1, 4, 1, 1])  # per electron
    rel = np.abs(o - ref) / ref
    assert np.all(rel <= [3e-5, 1e-5, 1e-9, 1e-9, 1e-9, 1e-9]), rel
    # energy weighting: the emitted energy is the electron's loss
    r = oracle.sample(p, 0)
    assert abs(o[3] - (p["gamma0"] - r[oracle.S_MU])) <= 1e-10 * o[3]


def test_photon_angles_add_the_beam_direction(oracle):
    """Plane wave, one energy, 1 mrad divergence: every sample runs the same
    trajectory, so the y second moment is the samples' own mean theta_y^2 plus
    the cone of the divergence-free run exactly, and in x also up to the
    cross term 2 <theta_x> <a/mu>."""
    import math
    base = workloads.scaled(workloads.plane_wave_1d(), n_samples=400, n_steps=512,
                            sigma_gamma=0.0, a0=5.0, gamma0=1000.0)
    o0 = oracle.photon_angles(base)
    p = dict(base, div_mrad=1.0)
    o = oracle.photon_angles(p)
    rec = oracle.samples(dict(p, n_steps=1), range(p["n_samples"]))
    tx, ty = rec[:, oracle.S_THX], rec[:, oracle.S_THY]   # mrad
    for w in (0, 3):   # number-weighted, energy-weighted
        assert abs(o[w] - o0[w]) <= 1e-12 * o0[w]
        assert abs(o[w + 2] ** 2 - (np.mean(ty ** 2) + o0[w + 2] ** 2)) <= 1e-9 * o[w + 2] ** 2
        cross = 2 * abs(np.mean(tx)) * o0[w + 1]
        assert abs(o[w + 1] ** 2 - (np.mean(tx ** 2) + o0[w + 1] ** 2)) <= cross + 1e-9
        assert cross < 0.1 * o[w + 1] ** 2  # the check is not empty
    assert math.isfinite(o[1]) and o[1] > o0[1]
