"""ctypes loader for the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  The oracle takes
the same plain parameter dictionary as the product binding (see
``paper_2308_09348_amd.workloads``) but converts it into its own struct.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QSO_LIB selects another build of the same source (the sanitized one)
LIB_PATH = os.environ.get("QSO_LIB") or os.path.join(HERE, "libqso.so")

ENVELOPE = {"gauss": 0, "sin2": 1}
RR_MODEL = {"classical": 0, "quantum": 1}
AMP_MODE = {"a0eff": 0, "local": 1}
DEPOSIT = {"point": 0, "cic": 1, "gauss": 2}
PROFILE = {"gauss": 0, "flat": 1}
MODE = {"gauss": 0, "hg": 1, "lg": 2}

# per-sample record layout (qso.h)
S_MU, S_SIG2, S_THX, S_THY, S_SIGTH, S_AEFF, S_CHIMAX, S_GAMMA0, S_X, S_Y, S_Z, S_N = range(12)
# moments layout
M_WEIGHT, M_MEAN_G, M_STD_G, M_MEAN_THX, M_RMS_THX, M_MEAN_THY, M_RMS_THY, \
    M_MEAN_AEFF, M_MAX_CHI, M_RAD_FRAC, M_MEAN_SIGF = range(11)
M_N = 16
# node record of the plane-wave reconstruction
N_A, N_GAMMA0, N_MU, N_SIG2, N_CHIMAX, N_N = range(6)


class Problem(ctypes.Structure):
    _fields_ = [
        ("a0", ctypes.c_double), ("lambda_um", ctypes.c_double), ("w0_um", ctypes.c_double),
        ("tau_fs", ctypes.c_double), ("x_off_um", ctypes.c_double),
        ("y_off_um", ctypes.c_double), ("delay_fs", ctypes.c_double),
        ("gamma0", ctypes.c_double), ("sigma_gamma", ctypes.c_double),
        ("sigma_r_um", ctypes.c_double), ("sigma_z_um", ctypes.c_double),
        ("div_mrad", ctypes.c_double), ("window_fwhm", ctypes.c_double),
        ("kernel_sigma_bins", ctypes.c_double), ("c_theta", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("n_samples", ctypes.c_int64),
        ("n_steps", ctypes.c_int32), ("shot", ctypes.c_int32),
        ("envelope", ctypes.c_int32), ("rr_model", ctypes.c_int32),
        ("amp_mode", ctypes.c_int32), ("deposit", ctypes.c_int32),
        ("n_e", ctypes.c_int32), ("n_th", ctypes.c_int32), ("n_a", ctypes.c_int32),
        ("transverse", ctypes.c_int32), ("longitudinal", ctypes.c_int32),
        ("mode", ctypes.c_int32), ("mode_m", ctypes.c_int32), ("mode_n", ctypes.c_int32),
        ("e_lo", ctypes.c_double), ("e_hi", ctypes.c_double),
        ("th_lo_mrad", ctypes.c_double), ("th_hi_mrad", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _b  # noqa: F401  (local build script)
            _b.build()
        _lib = load(LIB_PATH)
    return _lib


def load(path):
    """A ctypes handle on an oracle library built from qso.cpp at `path`
    (the tests also load copies built with a planted mistake)."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(Problem)
    L.qso_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
    L.qso_philox4x32_10.restype = None
    L.qso_normals.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, dp]
    L.qso_normals.restype = None
    L.qso_gh_quadrature.argtypes = [ctypes.c_double, dp, dp]
    L.qso_gh_quadrature.restype = None
    L.qso_radiation.argtypes = [ctypes.c_double, dp]
    L.qso_radiation.restype = None
    L.qso_rhs.argtypes = [pp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    L.qso_rhs.restype = ctypes.c_int
    L.qso_envelope_carrier.argtypes = [pp, ctypes.c_double]
    L.qso_envelope_carrier.restype = ctypes.c_double
    L.qso_derived.argtypes = [pp, dp]
    L.qso_derived.restype = ctypes.c_int
    L.qso_sample.argtypes = [pp, ctypes.c_int64, dp]
    L.qso_sample.restype = ctypes.c_int
    L.qso_forward.argtypes = [pp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                              dp, dp, dp, dp]
    L.qso_forward.restype = ctypes.c_int
    L.qso_flop_tally.argtypes = [pp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, dp]
    L.qso_flop_tally.restype = ctypes.c_int
    L.qso_sample_grad.argtypes = [pp, ctypes.c_int64, dp]
    L.qso_sample_grad.restype = ctypes.c_int
    L.qso_grad.argtypes = [pp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, dp, dp]
    L.qso_grad.restype = ctypes.c_int
    L.qso_grad_outputs.argtypes = [pp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, dp, dp,
                                   dp, dp]
    L.qso_grad_outputs.restype = ctypes.c_int
    L.qso_photons.argtypes = [pp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int32,
                              ctypes.c_double, ctypes.c_double, dp, dp]
    L.qso_photons.restype = ctypes.c_int
    L.qso_photon_cdf.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
    L.qso_photon_cdf.restype = ctypes.c_int
    L.qso_deposit.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                              ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int32, dp]
    L.qso_deposit.restype = ctypes.c_int
    L.qso_factorised.argtypes = [pp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_int, dp, dp, dp, dp, dp, dp]
    L.qso_factorised.restype = ctypes.c_int
    L.qso_factorised_samples.argtypes = [pp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_int, dp]
    L.qso_factorised_samples.restype = ctypes.c_int
    L.qso_photon_angles.argtypes = [pp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, dp]
    L.qso_photon_angles.restype = ctypes.c_int
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def problem(params):
    """Convert a plain parameter dictionary into the oracle's struct."""
    p = Problem()
    for name, _ in Problem._fields_:
        if name == "pad_":
            continue
        if name in ("transverse", "longitudinal"):
            v = params.get(name, "gauss")
            setattr(p, name, PROFILE[v] if isinstance(v, str) else v)
            continue
        if name == "mode":
            v = params.get("mode", "gauss")
            setattr(p, name, MODE[v] if isinstance(v, str) else v)
            continue
        if name in ("mode_m", "mode_n"):
            setattr(p, name, int(params.get(name, 0)))
            continue
        v = params[name]
        if name == "envelope":
            v = ENVELOPE[v] if isinstance(v, str) else v
        elif name == "rr_model":
            v = RR_MODEL[v] if isinstance(v, str) else v
        elif name == "amp_mode":
            v = AMP_MODE[v] if isinstance(v, str) else v
        elif name == "deposit":
            v = DEPOSIT[v] if isinstance(v, str) else v
        setattr(p, name, v)
    return p


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().qso_philox4x32_10(c, k, o)
    return list(o)


def normals(seed, shot, i):
    out = np.zeros(6)
    lib().qso_normals(seed, shot, i, _dp(out))
    return out


def gh_quadrature(chi):
    g, h = ctypes.c_double(), ctypes.c_double()
    lib().qso_gh_quadrature(chi, ctypes.byref(g), ctypes.byref(h))
    return g.value, h.value


def radiation(chi):
    out = np.zeros(4)
    lib().qso_radiation(chi, _dp(out))
    return out


def rhs(params, mu, sig2, a):
    out = np.zeros(6)
    p = problem(params)
    if lib().qso_rhs(ctypes.byref(p), mu, sig2, a, _dp(out)) != 0:
        raise ValueError("invalid problem")
    return out


def envelope_carrier(params, psi):
    p = problem(params)
    return lib().qso_envelope_carrier(ctypes.byref(p), psi)


def derived(params):
    out = np.zeros(7)
    p = problem(params)
    if lib().qso_derived(ctypes.byref(p), _dp(out)) != 0:
        raise ValueError("invalid problem")
    return dict(zip(["omega0", "aS", "K", "CD", "zR", "psi_max", "h"], out))


def sample(params, i):
    rec = np.zeros(S_N)
    p = problem(params)
    rc = lib().qso_sample(ctypes.byref(p), i, _dp(rec))
    if rc == -1:
        raise ValueError("invalid problem")
    return rec


def samples(params, indices):
    return np.stack([sample(params, int(i)) for i in indices])


def forward(params, i_begin=0, i_end=None, nthreads=0):
    """Histograms (raw weights) and moments over samples [i_begin, i_end)."""
    if i_end is None:
        i_end = params["n_samples"]
    p = problem(params)
    he = np.zeros(params["n_e"] + 2)
    ht = np.zeros(params["n_th"] + 2)
    ha = np.zeros(params["n_a"])
    mo = np.zeros(M_N)
    rc = lib().qso_forward(ctypes.byref(p), i_begin, i_end, nthreads,
                           _dp(he), _dp(ht), _dp(ha), _dp(mo))
    if rc == -1:
        raise ValueError("invalid problem")
    if rc == -2:
        raise FloatingPointError("non-finite state")
    return {"energy_hist": he, "angle_hist": ht, "a0eff_hist": ha, "moments": mo}


def factorised(params, n_anodes, n_gnodes, i_begin=0, i_end=None, nthreads=0):
    """Plane-wave reconstruction of the A0EFF forward pass on an n_anodes x
    n_gnodes node grid: histograms, moments, node records [nodes, N_N] and
    node weights [nodes] (node = k n_gnodes + m)."""
    if i_end is None:
        i_end = params["n_samples"]
    p = problem(params)
    he = np.zeros(params["n_e"] + 2)
    ht = np.zeros(params["n_th"] + 2)
    ha = np.zeros(params["n_a"])
    mo = np.zeros(M_N)
    ns = np.zeros((n_anodes * n_gnodes, N_N))
    nw = np.zeros(n_anodes * n_gnodes)
    rc = lib().qso_factorised(ctypes.byref(p), n_anodes, n_gnodes, i_begin, i_end, nthreads,
                              _dp(he), _dp(ht), _dp(ha), _dp(mo), _dp(ns), _dp(nw))
    if rc == -1:
        raise ValueError("invalid problem")
    if rc == -2:
        raise FloatingPointError("non-finite state")
    return {"energy_hist": he, "angle_hist": ht, "a0eff_hist": ha, "moments": mo,
            "node_states": ns, "node_weights": nw}


def factorised_samples(params, n_anodes, n_gnodes, indices, nthreads=0):
    """Records [len(indices), S_N] of the given samples as the reconstruction
    deposits them (interpolated final state, own observables)."""
    idx = np.ascontiguousarray(np.asarray(list(indices), dtype=np.int64))
    recs = np.zeros((len(idx), S_N))
    p = problem(params)
    rc = lib().qso_factorised_samples(ctypes.byref(p), n_anodes, n_gnodes, len(idx),
                                      idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      nthreads, _dp(recs))
    if rc == -1:
        raise ValueError("invalid problem")
    if rc == -2:
        raise FloatingPointError("non-finite state")
    return recs


PARAM_NAMES = ["a0", "w0_um", "x_off_um", "y_off_um", "delay_fs", "gamma0", "sigma_gamma",
               "div_mrad"]


def flop_tally(params, n_tally=16, steps_b=None):
    """The oracle's operation count per sample-step of the phase loop on the
    first n_tally samples of a workload: dict of adds, muls, divs,
    transcendentals and total (the per-sample path run with an
    operation-counting value type at n_steps and steps_b steps), and
    "amplitude": the operations of one amplitude evaluation."""
    out = np.zeros(6)
    p = problem(params)
    steps_b = steps_b or 2 * params["n_steps"]
    if lib().qso_flop_tally(ctypes.byref(p), 0, n_tally, steps_b, _dp(out)) != 0:
        raise ValueError("invalid problem")
    return dict(zip(["add", "mul", "div", "trans", "total", "amplitude"], out.tolist()))


def sample_grad(params, i):
    """(mu_f, d mu_f/dp[8]), (sig2_f, d sig2_f/dp[8]) for sample i."""
    out = np.zeros(18)
    p = problem(params)
    rc = lib().qso_sample_grad(ctypes.byref(p), i, _dp(out))
    if rc == -1:
        raise ValueError("invalid problem")
    return out[:9], out[9:]


def grad(params, i_begin=0, i_end=None, nthreads=0):
    """Energy histogram [n_e + 2] and its Jacobian [n_e + 2, 8] with respect to
    PARAM_NAMES."""
    if i_end is None:
        i_end = params["n_samples"]
    p = problem(params)
    h = np.zeros(params["n_e"] + 2)
    j = np.zeros((params["n_e"] + 2, 8))
    rc = lib().qso_grad(ctypes.byref(p), i_begin, i_end, nthreads, _dp(h), _dp(j))
    if rc == -1:
        raise ValueError("invalid problem")
    if rc == -2:
        raise FloatingPointError("non-finite state")
    return h, j


def grad_outputs(params, i_begin=0, i_end=None, nthreads=0):
    """Angle histogram [n_th + 2] with its Jacobian [n_th + 2, 8] and the
    moments [16] with their Jacobian [16, 8], with respect to PARAM_NAMES."""
    if i_end is None:
        i_end = params["n_samples"]
    p = problem(params)
    ht = np.zeros(params["n_th"] + 2)
    jt = np.zeros((params["n_th"] + 2, 8))
    m = np.zeros(M_N)
    jm = np.zeros((M_N, 8))
    rc = lib().qso_grad_outputs(ctypes.byref(p), i_begin, i_end, nthreads, _dp(ht), _dp(jt),
                                _dp(m), _dp(jm))
    if rc == -1:
        raise ValueError("invalid problem")
    if rc == -2:
        raise FloatingPointError("non-finite state")
    return ht, jt, m, jm


def photons(params, n_ph, ph_lo, ph_hi, i_begin=0, i_end=None, nthreads=0):
    """Expected photon number per photon-energy bin (n_ph + 2 with underflow,
    overflow) over samples [i_begin, i_end), and (emitted photon energy,
    electron energy loss), both in m c^2."""
    if i_end is None:
        i_end = params["n_samples"]
    p = problem(params)
    h = np.zeros(n_ph + 2)
    e = np.zeros(2)
    rc = lib().qso_photons(ctypes.byref(p), i_begin, i_end, nthreads, n_ph, ph_lo, ph_hi,
                           _dp(h), _dp(e))
    if rc == -1:
        raise ValueError("invalid problem")
    if rc == -2:
        raise FloatingPointError("non-finite state")
    return h, e


def photon_angles(params, i_begin=0, i_end=None, nthreads=0):
    """[photon number, rms theta_x, rms theta_y (number-weighted, mrad),
    emitted energy, rms theta_x, rms theta_y (energy-weighted, mrad)]."""
    if i_end is None:
        i_end = params["n_samples"]
    out = np.zeros(6)
    p = problem(params)
    rc = lib().qso_photon_angles(ctypes.byref(p), i_begin, i_end, nthreads, _dp(out))
    if rc == -1:
        raise ValueError("invalid problem")
    if rc == -2:
        raise FloatingPointError("non-finite state")
    return out


def photon_cdf(xi, chi):
    """(Phi(xi; chi), Phi(1; chi)) of the LCFA photon number spectrum."""
    phi, tot = ctypes.c_double(), ctypes.c_double()
    if lib().qso_photon_cdf(xi, chi, ctypes.byref(phi), ctypes.byref(tot)) != 0:
        raise ValueError("chi out of range")
    return phi.value, tot.value


def deposit(v, s, dep, ksig, lo, hi, n):
    hist = np.zeros(n + 2)
    d = DEPOSIT[dep] if isinstance(dep, str) else dep
    if lib().qso_deposit(v, s, d, ksig, lo, hi, n, _dp(hist)) != 0:
        raise ValueError("invalid deposit")
    return hist
