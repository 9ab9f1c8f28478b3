"""ctypes binding of libqscatter.so (the C ABI of include/qscatter.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  The library must be built (``build()`` of
``__graft_entry__`` or ``python -m paper_2308_09348_amd.build``); there is no
fallback when it is missing.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libqscatter.so")

QS_OK, QS_EINVAL, QS_ENOMEM, QS_EDEVICE, QS_ENONFINITE, QS_EUNSUPPORTED, QS_ERANGE = range(7)
ENVELOPE = {"gauss": 0, "sin2": 1}
RR_MODEL = {"classical": 0, "quantum": 1}
AMP_MODE = {"a0eff": 0, "local": 1}
DEPOSIT = {"point": 0, "cic": 1, "gauss": 2}
PRECISION = {"fp32": 0, "fp64": 1}
PROFILE = {"gauss": 0, "flat": 1}
MODE = {"gauss": 0, "hg": 1, "lg": 2}

M_N = 21
# share of the pass's wavefront phase steps taken in FP64 (-1: not counted)
M_FP64_STEPS = 20
# FP64 shadow of an FP32 pass (qs_numerics.flags) and its moment fields
VALIDATE_FP64 = 1
(M_SHADOW_N, M_ERR_MU_MAX, M_ERR_MU_MEAN, M_ERR_SIG_MAX, M_ERR_MEAN_G) = range(11, 16)
(M_ERR_E_L1, M_ERR_E_MAX, M_ERR_T_L1, M_ERR_T_MAX) = range(16, 20)
S_N = 11
# FP64-shadow reports of the photon and adjoint passes (QS_PE_*, QS_GE_*)
(PE_SHADOW_N, PE_HIST_L1, PE_HIST_MAX, PE_ENERGY, PE_LOSS, PE_ANGLES) = range(6)
PE_REF_PHOTONS, PE_REF_ENERGY, PE_REF_LOSS = PE_ANGLES + 6, PE_ANGLES + 7, PE_ANGLES + 8
PE_N = PE_ANGLES + 9
GE_SHADOW_N, GE_DIFF, GE_REF, GE_N = 0, 1, 9, 17
NOALLOC_MAX_SAMPLES = 1 << 20  # QS_NOALLOC_MAX_SAMPLES
(M_WEIGHT, M_MEAN_G, M_STD_G, M_MEAN_THX, M_RMS_THX, M_MEAN_THY, M_RMS_THY, M_MEAN_AEFF,
 M_MAX_CHI, M_RAD_FRAC, M_MEAN_SIGF) = range(11)
(S_MU, S_SIG2, S_THX, S_THY, S_SIGTH, S_AEFF, S_CHIMAX, S_GAMMA0, S_X, S_Y, S_Z) = range(11)


class Laser(ctypes.Structure):
    _fields_ = [("a0", ctypes.c_double), ("lambda_um", ctypes.c_double),
                ("w0_um", ctypes.c_double), ("tau_fs", ctypes.c_double),
                ("envelope", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("x_off_um", ctypes.c_double), ("y_off_um", ctypes.c_double),
                ("delay_fs", ctypes.c_double), ("mode_m", ctypes.c_int32),
                ("mode_n", ctypes.c_int32)]


class Beam(ctypes.Structure):
    _fields_ = [("gamma0", ctypes.c_double), ("sigma_gamma", ctypes.c_double),
                ("sigma_r_um", ctypes.c_double), ("sigma_z_um", ctypes.c_double),
                ("div_mrad", ctypes.c_double), ("transverse", ctypes.c_int32),
                ("longitudinal", ctypes.c_int32)]


class Numerics(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int64), ("n_steps", ctypes.c_int32),
                ("shot", ctypes.c_int32), ("window_fwhm", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("rr_model", ctypes.c_int32),
                ("amp_mode", ctypes.c_int32), ("deposit", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("kernel_sigma_bins", ctypes.c_double),
                ("chi_fp64", ctypes.c_double), ("c_theta", ctypes.c_double),
                ("flags", ctypes.c_int32), ("shadow_stride", ctypes.c_int32)]


class Bins(ctypes.Structure):
    _fields_ = [("n_e", ctypes.c_int32), ("n_th", ctypes.c_int32), ("n_a", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("e_lo", ctypes.c_double),
                ("e_hi", ctypes.c_double), ("th_lo_mrad", ctypes.c_double),
                ("th_hi_mrad", ctypes.c_double)]


class Outputs(ctypes.Structure):
    _fields_ = [("energy_hist", ctypes.c_void_p), ("angle_hist", ctypes.c_void_p),
                ("a0eff_hist", ctypes.c_void_p), ("moments", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("samples", ctypes.c_void_p),
                ("sample_stride", ctypes.c_int64), ("n_sample_records", ctypes.c_int64)]


class NodeGrid(ctypes.Structure):
    _fields_ = [("n_a", ctypes.c_int32), ("n_g", ctypes.c_int32),
                ("node_states", ctypes.c_void_p), ("node_weights", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("dep_tile", ctypes.c_int32), ("phase_cap", ctypes.c_int32),
                ("dep_cap", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("phase_ms", ctypes.c_double), ("deposit_ms", ctypes.c_double)]


NODE_FIELDS = 5  # a0,eff, gamma0, mu_f, sig2_f, chi max
N_A, N_GAMMA0, N_MU, N_SIG2, N_CHIMAX = range(NODE_FIELDS)


class PhotonBins(ctypes.Structure):
    _fields_ = [("n_ph", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("ph_lo", ctypes.c_double), ("ph_hi", ctypes.c_double)]


class PhotonOutputs(ctypes.Structure):
    _fields_ = [("photon_hist", ctypes.c_void_p), ("energy", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("angles", ctypes.c_void_p),
                ("errors", ctypes.c_void_p)]


class GradOutputs(ctypes.Structure):
    _fields_ = [("d_energy_hist", ctypes.c_void_p), ("grad", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("d_angle_hist", ctypes.c_void_p),
                ("d_moments", ctypes.c_void_p), ("moments", ctypes.c_void_p),
                ("errors", ctypes.c_void_p)]


# parameters of the adjoint, in the order of the QS_P_* enum
PARAM_NAMES = ("a0", "w0_um", "x_off_um", "y_off_um", "delay_fs", "gamma0", "sigma_gamma",
               "div_mrad")

TAPE_FIELDS = 2 + 2 * len(PARAM_NAMES)  # mu, sig2, d mu / dp, d sig2 / dp
T_MU, T_SIG2, T_DMU, T_DSIG2 = 0, 1, 2, 2 + len(PARAM_NAMES)

EXPORTS = ["qs_create", "qs_destroy", "qs_forward", "qs_forward_noalloc", "qs_forward_batched",
           "qs_forward_factorised", "qs_forward_factorised_batched", "qs_backward",
           "qs_backward_batched", "qs_forward_tape", "qs_forward_tape_batched",
           "qs_backward_tape", "qs_backward_tape_batched", "qs_photons", "qs_photons_batched",
           "qs_photon_cdf", "qs_radiation_eval",
           "qs_radiation_derivs", "qs_sync_status",
           "qs_set_profiling", "qs_last_timings", "qs_timings_sum", "qs_tune", "qs_set_graphs", "qs_strerror",
           "qs_last_error", "qs_abi_version", "qs_build_id"]

_lib = None


class QScatterError(RuntimeError):
    def __init__(self, status, detail=""):
        self.status = status
        msg = lib().qs_strerror(status).decode()
        super().__init__(f"{msg} ({status})" + (f": {detail}" if detail else ""))


def lib():
    """Load libqscatter.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2308_09348_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.qs_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        L.qs_create.restype = ctypes.c_int
        L.qs_destroy.argtypes = [vp]
        L.qs_destroy.restype = None
        L.qs_forward.argtypes = [vp, ctypes.POINTER(Laser), ctypes.POINTER(Beam),
                                 ctypes.POINTER(Numerics), ctypes.POINTER(Bins),
                                 ctypes.POINTER(Outputs), vp]
        L.qs_forward.restype = ctypes.c_int
        L.qs_forward_noalloc.argtypes = L.qs_forward.argtypes
        L.qs_forward_noalloc.restype = ctypes.c_int
        L.qs_forward_batched.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Laser),
                                         ctypes.POINTER(Beam), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(Numerics), ctypes.POINTER(Bins),
                                         ctypes.POINTER(Outputs), vp]
        L.qs_forward_batched.restype = ctypes.c_int
        L.qs_forward_factorised.argtypes = [vp, ctypes.POINTER(Laser), ctypes.POINTER(Beam),
                                            ctypes.POINTER(Numerics), ctypes.POINTER(Bins),
                                            ctypes.POINTER(NodeGrid), ctypes.POINTER(Outputs), vp]
        L.qs_forward_factorised.restype = ctypes.c_int
        L.qs_forward_factorised_batched.argtypes = [
            vp, ctypes.c_int32, ctypes.POINTER(Laser), ctypes.POINTER(Beam),
            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(Numerics), ctypes.POINTER(Bins),
            ctypes.POINTER(NodeGrid), ctypes.POINTER(Outputs), vp]
        L.qs_forward_factorised_batched.restype = ctypes.c_int
        L.qs_backward.argtypes = [vp, ctypes.POINTER(Laser), ctypes.POINTER(Beam),
                                  ctypes.POINTER(Numerics), ctypes.POINTER(Bins),
                                  ctypes.POINTER(GradOutputs), vp]
        L.qs_backward.restype = ctypes.c_int
        L.qs_backward_batched.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Laser),
                                          ctypes.POINTER(Beam), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(Numerics), ctypes.POINTER(Bins),
                                          ctypes.POINTER(GradOutputs), vp]
        L.qs_backward_batched.restype = ctypes.c_int
        L.qs_forward_tape.argtypes = L.qs_forward.argtypes[:6] + [vp, vp]
        L.qs_forward_tape.restype = ctypes.c_int
        L.qs_forward_tape_batched.argtypes = L.qs_forward_batched.argtypes[:8] + [vp, vp]
        L.qs_forward_tape_batched.restype = ctypes.c_int
        L.qs_backward_tape.argtypes = L.qs_backward.argtypes[:6] + [vp, vp]
        L.qs_backward_tape.restype = ctypes.c_int
        L.qs_backward_tape_batched.argtypes = L.qs_backward_batched.argtypes[:8] + [vp, vp]
        L.qs_backward_tape_batched.restype = ctypes.c_int
        L.qs_photons.argtypes = [vp, ctypes.POINTER(Laser), ctypes.POINTER(Beam),
                                 ctypes.POINTER(Numerics), ctypes.POINTER(PhotonBins),
                                 ctypes.POINTER(PhotonOutputs), vp]
        L.qs_photons.restype = ctypes.c_int
        L.qs_photons_batched.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Laser),
                                         ctypes.POINTER(Beam), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(Numerics), ctypes.POINTER(PhotonBins),
                                         ctypes.POINTER(PhotonOutputs), vp]
        L.qs_photons_batched.restype = ctypes.c_int
        L.qs_photon_cdf.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp]
        L.qs_photon_cdf.restype = ctypes.c_int
        L.qs_radiation_eval.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, vp, vp, vp]
        L.qs_radiation_eval.restype = ctypes.c_int
        L.qs_radiation_derivs.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, vp, vp, vp]
        L.qs_radiation_derivs.restype = ctypes.c_int
        L.qs_sync_status.argtypes = [vp, vp, vp]
        L.qs_sync_status.restype = ctypes.c_int
        L.qs_set_profiling.argtypes = [vp, ctypes.c_int]
        L.qs_set_profiling.restype = ctypes.c_int
        L.qs_last_timings.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.qs_last_timings.restype = ctypes.c_int
        L.qs_timings_sum.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_double)]
        L.qs_timings_sum.restype = ctypes.c_int
        L.qs_tune.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Laser), ctypes.POINTER(Beam),
                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(Numerics),
                              ctypes.POINTER(Bins), ctypes.c_char_p, ctypes.POINTER(Tuning), vp]
        L.qs_tune.restype = ctypes.c_int
        L.qs_set_graphs.argtypes = [vp, ctypes.c_int]
        L.qs_set_graphs.restype = ctypes.c_int
        L.qs_strerror.argtypes = [ctypes.c_int]
        L.qs_strerror.restype = ctypes.c_char_p
        L.qs_last_error.argtypes = [vp]
        L.qs_last_error.restype = ctypes.c_char_p
        L.qs_abi_version.argtypes = []
        L.qs_abi_version.restype = ctypes.c_int
        L.qs_build_id.argtypes = []
        L.qs_build_id.restype = ctypes.c_char_p
        _lib = L
    return _lib


def build_id():
    """The source hash stamped into the loaded library (qs_build_id)."""
    return lib().qs_build_id().decode()


def check_build():
    """Raise unless the loaded library was built from the sources now checked
    out (its stamped hash against build.source_id()); returns the hash."""
    from . import build as _build
    want, have = _build.source_id(), build_id()
    if have != want:
        raise RuntimeError(f"{LIB_PATH} was built from other sources (build id {have[:16]}, "
                           f"sources {want[:16]}): rebuild it")
    return have


def _enum(table, v):
    return table[v] if isinstance(v, str) else int(v)


def photon_bins(params):
    """Photon-energy bins of a parameter dictionary (m c^2 units): n_ph
    (default 256) over [ph_lo, ph_hi) (default [0, e_hi))."""
    return PhotonBins(n_ph=int(params.get("n_ph", 256)), reserved0=0,
                      ph_lo=float(params.get("ph_lo", 0.0)),
                      ph_hi=float(params.get("ph_hi", params["e_hi"])))


def structs(params):
    """Plain parameter dictionary -> (Laser, Beam, Numerics, Bins)."""
    la = Laser(a0=params["a0"], lambda_um=params["lambda_um"], w0_um=params["w0_um"],
               tau_fs=params["tau_fs"], envelope=_enum(ENVELOPE, params["envelope"]),
               mode=_enum(MODE, params.get("mode", "gauss")), x_off_um=params["x_off_um"],
               y_off_um=params["y_off_um"], delay_fs=params["delay_fs"],
               mode_m=int(params.get("mode_m", 0)), mode_n=int(params.get("mode_n", 0)))
    be = Beam(gamma0=params["gamma0"], sigma_gamma=params["sigma_gamma"],
              sigma_r_um=params["sigma_r_um"], sigma_z_um=params["sigma_z_um"],
              div_mrad=params["div_mrad"],
              transverse=_enum(PROFILE, params.get("transverse", "gauss")),
              longitudinal=_enum(PROFILE, params.get("longitudinal", "gauss")))
    nu = Numerics(n_samples=params["n_samples"], n_steps=params["n_steps"],
                  shot=params.get("shot", 0), window_fwhm=params["window_fwhm"],
                  seed=params["seed"], rr_model=_enum(RR_MODEL, params["rr_model"]),
                  amp_mode=_enum(AMP_MODE, params["amp_mode"]),
                  deposit=_enum(DEPOSIT, params["deposit"]),
                  precision=_enum(PRECISION, params.get("precision", "fp32")),
                  kernel_sigma_bins=params["kernel_sigma_bins"],
                  chi_fp64=params.get("chi_fp64", 0.0), c_theta=params["c_theta"],
                  flags=VALIDATE_FP64 if params.get("validate_fp64") else 0,
                  shadow_stride=int(params.get("shadow_stride", 0)))
    bi = Bins(n_e=params["n_e"], n_th=params["n_th"], n_a=params["n_a"], reserved0=0,
              e_lo=params["e_lo"], e_hi=params["e_hi"], th_lo_mrad=params["th_lo_mrad"],
              th_hi_mrad=params["th_hi_mrad"])
    return la, be, nu, bi
