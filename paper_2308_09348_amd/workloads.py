"""Seeded synthetic workloads shaped like the paper's scenarios.

This module holds parameter sets and seeded parameter draws only -- none of
the method's arithmetic.  Both the HIP path and the CPU oracle consume these
plain dictionaries.  The paper's own runs (Appendix A) are PIC simulations
whose data is not available; these inputs stand in for them.

Units: lengths in micrometres, times in femtoseconds, angles in mrad,
energies in m c^2.
"""
import copy

import numpy as np

BASE = dict(
    # laser
    a0=10.0, lambda_um=0.8, w0_um=0.0, tau_fs=30.0, envelope="gauss",
    x_off_um=0.0, y_off_um=0.0, delay_fs=0.0,
    # beam
    gamma0=2000.0, sigma_gamma=100.0, sigma_r_um=0.0, sigma_z_um=0.0, div_mrad=0.0,
    transverse="gauss", longitudinal="gauss",
    # numerics
    n_samples=10_000, n_steps=512, window_fwhm=2.5, seed=1, shot=0,
    rr_model="classical", amp_mode="a0eff", deposit="point",
    kernel_sigma_bins=1.0, c_theta=1.0,
    # bins
    n_e=200, e_lo=0.0, e_hi=3000.0, n_th=128, th_lo_mrad=-50.0, th_hi_mrad=50.0, n_a=256,
)


def plane_wave_1d():
    """Head-on plane-wave-like collision: a0=10, 0.8 um, Gaussian 30 fs FWHM,
    gamma0 ~ N(2000, 100^2), 10^4 samples, 512 steps, classical LL, 200 energy
    bins over [0, 1.5 gamma0)."""
    return copy.deepcopy(BASE)


def focused_3d():
    """Focused single shot: a0=50, w0=3 um, 30 fs; sigma_r=3 um, sigma_z=5 um,
    gamma0 = 2000 +- 5%, 1 mrad divergence; x offset 2 um, delay 10 fs;
    2^22 samples, 1024 steps, quantum-corrected moments, local amplitude,
    256 energy / 128 angle / 256 a0,eff bins."""
    p = copy.deepcopy(BASE)
    p.update(a0=50.0, w0_um=3.0, tau_fs=30.0, x_off_um=2.0, y_off_um=0.0, delay_fs=10.0,
             gamma0=2000.0, sigma_gamma=100.0, sigma_r_um=3.0, sigma_z_um=5.0, div_mrad=1.0,
             n_samples=1 << 22, n_steps=1024, seed=2, rr_model="quantum", amp_mode="local",
             deposit="cic", n_e=256, e_lo=0.0, e_hi=3000.0, n_th=128, n_a=256)
    return p


def differentiation():
    """Focused-shot physics with the Gaussian-kernel deposit (1 bin), 2^20
    samples, 1024 steps."""
    p = focused_3d()
    p.update(n_samples=1 << 20, deposit="gauss", kernel_sigma_bins=1.0, seed=4)
    return p


GRAD_PARAMS = ("a0", "w0_um", "x_off_um", "y_off_um", "delay_fs", "gamma0", "sigma_gamma",
               "div_mrad")


def differentiation_eval(seed=40):
    """The point where the differentiation workload's loss is evaluated: each
    of the eight differentiable parameters of differentiation() scaled by
    (1 + 0.05 eps), eps ~ N(0, 1) drawn by PCG64(seed)."""
    p = differentiation()
    eps = np.random.Generator(np.random.PCG64(seed)).normal(size=len(GRAD_PARAMS))
    for name, e in zip(GRAD_PARAMS, eps):
        p[name] = float(p[name] * (1.0 + 0.05 * e))
    return p


def batched_shots(n_shots=4096, seed=3):
    """Per-shot parameter draws for the batched workload: samples log-uniform
    in [2^12, 2^18], a0 ~ U[5, 100], w0 ~ U[2, 6] um, offsets ~ N(0, 2^2) um,
    delay ~ N(0, 15^2) fs, gamma0 ~ U[1e3, 1e4], sigma_gamma/gamma0 ~
    U[1%, 10%]; 512 steps, quantum, local amplitude."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(size=n_shots)
    n_samples = np.round(2.0 ** (12 + 6 * u)).astype(np.int64)
    a0 = rng.uniform(5.0, 100.0, n_shots)
    w0 = rng.uniform(2.0, 6.0, n_shots)
    xo = rng.normal(0.0, 2.0, n_shots)
    yo = rng.normal(0.0, 2.0, n_shots)
    dl = rng.normal(0.0, 15.0, n_shots)
    g0 = rng.uniform(1e3, 1e4, n_shots)
    sg = rng.uniform(0.01, 0.10, n_shots) * g0
    shots = []
    for s in range(n_shots):
        p = copy.deepcopy(BASE)
        p.update(a0=float(a0[s]), w0_um=float(w0[s]), tau_fs=30.0, x_off_um=float(xo[s]),
                 y_off_um=float(yo[s]), delay_fs=float(dl[s]), gamma0=float(g0[s]),
                 sigma_gamma=float(sg[s]), sigma_r_um=3.0, sigma_z_um=5.0, div_mrad=1.0,
                 n_samples=int(n_samples[s]), n_steps=512, seed=seed, shot=s,
                 rr_model="quantum", amp_mode="local", deposit="cic", n_e=256,
                 e_lo=0.0, e_hi=1.5 * float(g0[s]), n_th=128, n_a=256)
        shots.append(p)
    return shots


def quantum_batch(n_shots=256, seed=5, n_samples=1 << 18):
    """Quantum batch with gradients and photon spectra: gamma0 ~ N(2e4, 600^2),
    a0 ~ U[50, 150] drawn per shot by PCG64(seed); W0 = 2 um, no offsets or
    delay, 30 fs, beam 3 um x 5 um, 1 mrad, 5 % energy spread; 2^18 samples,
    2048 steps, quantum moments with FP64 steps where chi > 0.1, local
    amplitude, Gaussian-kernel deposit; 256 energy bins over [0, 1.5 gamma0)
    and 256 photon bins over [0, 1.2 gamma0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g0 = rng.normal(2e4, 600.0, n_shots)
    a0 = rng.uniform(50.0, 150.0, n_shots)
    shots = []
    for s in range(n_shots):
        p = copy.deepcopy(BASE)
        p.update(a0=float(a0[s]), w0_um=2.0, tau_fs=30.0, x_off_um=0.0, y_off_um=0.0,
                 delay_fs=0.0, gamma0=float(g0[s]), sigma_gamma=0.05 * float(g0[s]),
                 sigma_r_um=3.0, sigma_z_um=5.0, div_mrad=1.0, n_samples=int(n_samples),
                 n_steps=2048, seed=seed, shot=s, rr_model="quantum", amp_mode="local",
                 deposit="gauss", kernel_sigma_bins=1.0, chi_fp64=0.1, n_e=256, e_lo=0.0,
                 e_hi=1.5 * float(g0[s]), n_th=128, n_a=256, n_ph=256, ph_lo=0.0,
                 ph_hi=1.2 * float(g0[s]))
        shots.append(p)
    return shots


def scaled(params, n_samples=None, n_steps=None, **kw):
    """A copy with fewer samples / steps (parity-test sizes)."""
    p = copy.deepcopy(params)
    if n_samples is not None:
        p["n_samples"] = int(n_samples)
    if n_steps is not None:
        p["n_steps"] = int(n_steps)
    p.update(kw)
    return p
