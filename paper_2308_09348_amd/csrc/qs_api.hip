// qs_api.hip -- host side of the C ABI declared in include/qscatter.h.
//
// The host validates arguments, derives the scalar constants of the problem
// (Sec. 2 eq. a0eff; Sec. 4 eq. dpdtRR; Sec. 3 eq. PWCRR) and enqueues
// kernels; all per-sample arithmetic runs on the device.
#include "qscatter.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "qs_internal.h"

struct qs_ctx {
    int device = -1;
    float *rad32 = nullptr;
    double *rad64 = nullptr;
    // per-call device scratch (grow-only)
    float *env32 = nullptr;
    double *env64 = nullptr;
    size_t env32_cap = 0, env64_cap = 0;
    unsigned long long *accum = nullptr;  // [2 + histogram words]: chimax, flags, hist
    size_t accum_cap = 0;
    double *partials = nullptr;
    size_t part_cap = 0;
    unsigned char *states = nullptr;  // per-sample final states (SampleState arrays)
    size_t states_cap = 0;
    int *eval_flags = nullptr;
    // kernel timing
    bool profiling = false;
    bool profiled_call = false;
    hipEvent_t ev[6] = {};
    char last_error[512] = {0};
};

namespace {

// CODATA 2018
constexpr double kPi = 3.14159265358979323846;
constexpr double kAlpha = 7.2973525693e-3;
constexpr double kLambdaBarC_um = 3.8615926796e-7;
constexpr double kC_um_per_fs = 0.299792458;

void set_err(qs_ctx *c, const char *msg) {
    if (c) std::snprintf(c->last_error, sizeof(c->last_error), "%s", msg);
}

qs_status hip_fail(qs_ctx *c, hipError_t e, const char *where) {
    if (c)
        std::snprintf(c->last_error, sizeof(c->last_error), "%s: %s", where, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? QS_ENOMEM : QS_EDEVICE;
}

class DeviceGuard {
   public:
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) (void)hipSetDevice(dev);
        dev_ = dev;
    }
    ~DeviceGuard() {
        if (prev_ >= 0 && prev_ != dev_) (void)hipSetDevice(prev_);
    }

   private:
    int prev_ = -1, dev_ = -1;
};

bool fin(double v) { return std::isfinite(v); }

qs_status validate(qs_ctx *c, const qs_laser *L, const qs_beam *B, const qs_numerics *N,
                   const qs_bins *H, const qs_outputs *O) {
    if (!L || !B || !N || !H || !O) return set_err(c, "null argument"), QS_EINVAL;
    const double vals[] = {L->a0, L->lambda_um, L->w0_um, L->tau_fs, L->x_off_um, L->y_off_um,
                           L->delay_fs, B->gamma0, B->sigma_gamma, B->sigma_r_um, B->sigma_z_um,
                           B->div_mrad, N->window_fwhm, N->kernel_sigma_bins, N->chi_fp64,
                           N->c_theta, H->e_lo, H->e_hi, H->th_lo_mrad, H->th_hi_mrad};
    for (double v : vals)
        if (!fin(v)) return set_err(c, "non-finite parameter"), QS_EINVAL;
    if (!(L->a0 >= 0) || !(L->lambda_um > 0) || !(L->w0_um >= 0) || !(L->tau_fs > 0))
        return set_err(c, "laser parameter out of range"), QS_EINVAL;
    if (L->envelope != QS_ENV_GAUSS && L->envelope != QS_ENV_SIN2)
        return set_err(c, "unknown envelope"), QS_EINVAL;
    if (!(B->gamma0 > 1) || !(B->sigma_gamma >= 0) || !(B->sigma_r_um >= 0) ||
        !(B->sigma_z_um >= 0) || !(B->div_mrad >= 0))
        return set_err(c, "beam parameter out of range"), QS_EINVAL;
    if (N->n_samples < 1 || N->n_samples > (int64_t)1 << 32)
        return set_err(c, "n_samples must be in [1, 2^32]"), QS_EINVAL;
    if (N->n_steps < 1 || N->n_steps > 65536)
        return set_err(c, "n_steps must be in [1, 65536]"), QS_EINVAL;
    if (N->shot < 0) return set_err(c, "shot must be >= 0"), QS_EINVAL;
    if (!(N->window_fwhm > 0) || !(N->kernel_sigma_bins >= 0) || !(N->c_theta >= 0))
        return set_err(c, "numerics parameter out of range"), QS_EINVAL;
    if (N->rr_model != QS_RR_CLASSICAL && N->rr_model != QS_RR_QUANTUM)
        return set_err(c, "unknown rr_model"), QS_EINVAL;
    if (N->amp_mode != QS_AMP_A0EFF && N->amp_mode != QS_AMP_LOCAL)
        return set_err(c, "unknown amp_mode"), QS_EINVAL;
    if (N->deposit < QS_DEP_POINT || N->deposit > QS_DEP_GAUSS)
        return set_err(c, "unknown deposit"), QS_EINVAL;
    if (N->precision != QS_PREC_FP32 && N->precision != QS_PREC_FP64)
        return set_err(c, "unknown precision"), QS_EINVAL;
    if (H->n_e < 1 || H->n_e > 4096 || H->n_th < 1 || H->n_th > 4096 || H->n_a < 1 ||
        H->n_a > 4096)
        return set_err(c, "bin counts must be in [1, 4096]"), QS_EINVAL;
    if (!(H->e_hi > H->e_lo) || !(H->th_hi_mrad > H->th_lo_mrad))
        return set_err(c, "histogram window must have hi > lo"), QS_EINVAL;
    if (!O->energy_hist || !O->angle_hist || !O->a0eff_hist || !O->moments || !O->status)
        return set_err(c, "null output pointer"), QS_EINVAL;
    if (O->samples && (O->sample_stride < 1 || O->n_sample_records < 0))
        return set_err(c, "sample records need stride >= 1"), QS_EINVAL;
    return QS_OK;
}

template <class T>
qs_status grow(qs_ctx *c, T **p, size_t *cap, size_t n, const char *what) {
    if (*cap >= n) return QS_OK;
    if (*p) {
        // earlier work queued on any stream may still read the old buffer
        (void)hipDeviceSynchronize();
        (void)hipFree(*p);
    }
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T));
    if (e != hipSuccess) return hip_fail(c, e, what);
    *cap = n;
    return QS_OK;
}

}  // namespace

extern "C" {

int qs_abi_version(void) { return QS_ABI_VERSION; }

const char *qs_strerror(qs_status s) {
    switch (s) {
        case QS_OK: return "ok";
        case QS_EINVAL: return "invalid argument";
        case QS_ENOMEM: return "out of device memory";
        case QS_EDEVICE: return "HIP runtime error";
        case QS_ENONFINITE: return "non-finite sample state";
        case QS_EUNSUPPORTED: return "unsupported";
        case QS_ERANGE: return "chi beyond the tabulated range";
    }
    return "unknown status";
}

const char *qs_last_error(qs_ctx *ctx) { return ctx ? ctx->last_error : ""; }

qs_status qs_create(qs_ctx **out, int device) {
    if (!out) return QS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return QS_EINVAL;
    qs_ctx *c = new (std::nothrow) qs_ctx;
    if (!c) return QS_ENOMEM;
    c->device = device;
    DeviceGuard g(device);
    hipError_t e;
    double *work = nullptr;
    const size_t wd = qs::radiation_work_doubles();
    if ((e = hipMalloc(&c->rad32, sizeof(float) * qs::kCells32 * qs::kCellVals)) != hipSuccess ||
        (e = hipMalloc(&c->rad64, sizeof(double) * qs::kCells64 * qs::kCellVals)) != hipSuccess ||
        (e = hipMalloc(&c->eval_flags, sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&work, sizeof(double) * wd)) != hipSuccess ||
        (e = hipMemset(c->eval_flags, 0, sizeof(int))) != hipSuccess) {
        qs_status st = hip_fail(c, e, "qs_create allocation");
        if (work) (void)hipFree(work);
        qs_destroy(c);
        return st;
    }
    e = qs::build_radiation_tables(c->rad32, c->rad64, work, wd, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipFree(work);
    if (e != hipSuccess) {
        qs_status st = hip_fail(c, e, "radiation tables");
        qs_destroy(c);
        return st;
    }
    *out = c;
    return QS_OK;
}

void qs_destroy(qs_ctx *c) {
    if (!c) return;
    {
        DeviceGuard g(c->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(c->rad32);
        (void)hipFree(c->rad64);
        (void)hipFree(c->env32);
        (void)hipFree(c->env64);
        (void)hipFree(c->accum);
        (void)hipFree(c->partials);
        (void)hipFree(c->states);
        (void)hipFree(c->eval_flags);
        for (hipEvent_t &e : c->ev)
            if (e) (void)hipEventDestroy(e);
    }
    delete c;
}

qs_status qs_forward(qs_ctx *c, const qs_laser *L, const qs_beam *B, const qs_numerics *N,
                     const qs_bins *H, const qs_outputs *O, void *stream) {
    if (!c) return QS_EINVAL;
    qs_status st = validate(c, L, B, N, H, O);
    if (st != QS_OK) return st;
    DeviceGuard guard(c->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    // ---- derived constants ----
    const double omega0 = 2.0 * kPi * kC_um_per_fs / L->lambda_um;  // rad / fs
    const double aS = L->lambda_um / (2.0 * kPi * kLambdaBarC_um);
    const double omega_tau = omega0 * L->tau_fs;
    const double psi_max = L->envelope == QS_ENV_GAUSS ? N->window_fwhm * omega_tau : omega_tau;

    int prec = qs::PREC_F32;
    if (N->precision == QS_PREC_FP64)
        prec = qs::PREC_F64;
    else if (N->rr_model == QS_RR_QUANTUM && N->chi_fp64 > 0)
        prec = qs::PREC_F32MIX;
    const double h = 2.0 * psi_max / (double)N->n_steps;
    const int64_t n = N->n_samples;

    // ---- scratch ----
    const size_t nh = (size_t)(H->n_e + 2) + (H->n_th + 2) + H->n_a;
    const size_t lds = qs::deposit_lds_bytes(H->n_e, H->n_th, H->n_a);
    int dgrid = 0;
    hipError_t e = qs::deposit_grid(lds, c->device, n, &dgrid);
    if (e != hipSuccess) return hip_fail(c, e, "deposit occupancy query");
    const size_t nenv = (size_t)2 * N->n_steps + 1;
    // 6 doubles + 1 float per sample, each array 256-byte aligned
    const size_t arr = ((size_t)n * 8 + 255) / 256 * 256;
    const size_t arrf = ((size_t)n * 4 + 255) / 256 * 256;
    if ((st = grow(c, &c->env32, &c->env32_cap, nenv, "envelope table")) != QS_OK) return st;
    if ((st = grow(c, &c->env64, &c->env64_cap, nenv, "envelope table")) != QS_OK) return st;
    if ((st = grow(c, &c->accum, &c->accum_cap, 2 + nh, "histogram accumulators")) != QS_OK)
        return st;
    if ((st = grow(c, &c->partials, &c->part_cap, (size_t)dgrid * qs::P_N, "moment partials")) !=
        QS_OK)
        return st;
    if ((st = grow(c, &c->states, &c->states_cap, 6 * arr + arrf, "sample states")) != QS_OK)
        return st;
    qs::SampleState ss;
    ss.mu = reinterpret_cast<double *>(c->states);
    ss.s2 = reinterpret_cast<double *>(c->states + arr);
    ss.S0 = reinterpret_cast<double *>(c->states + 2 * arr);
    ss.g0 = reinterpret_cast<double *>(c->states + 3 * arr);
    ss.thx = reinterpret_cast<double *>(c->states + 4 * arr);
    ss.thy = reinterpret_cast<double *>(c->states + 5 * arr);
    ss.cmx = reinterpret_cast<float *>(c->states + 6 * arr);
    unsigned int *chimax_bits = reinterpret_cast<unsigned int *>(c->accum);
    int *flags = reinterpret_cast<int *>(c->accum + 1);
    unsigned long long *hist = c->accum + 2;

    qs::PhaseParams p{};
    const bool plane_wave = L->w0_um == 0.0;
    p.a0 = L->a0;
    p.inv_w0sq = plane_wave ? 0.0 : 1.0 / (L->w0_um * L->w0_um);
    p.inv_zR = plane_wave ? 0.0 : L->lambda_um / (kPi * L->w0_um * L->w0_um);
    p.x_off = L->x_off_um;
    p.y_off = L->y_off_um;
    p.z_delay = 0.5 * kC_um_per_fs * L->delay_fs;
    p.ell_per_psi = L->lambda_um / (4.0 * kPi);
    p.gamma0 = B->gamma0;
    p.sigma_gamma = B->sigma_gamma;
    p.sigma_r = B->sigma_r_um;
    p.sigma_z = B->sigma_z_um;
    p.div_rad = 1e-3 * B->div_mrad;
    p.two_over_aS = 2.0 / aS;
    p.K = 4.0 * kAlpha / (3.0 * aS);
    p.CD = 55.0 / (6.0 * std::sqrt(3.0)) * kAlpha / (aS * aS);
    p.psi_max = psi_max;
    p.h = h;
    p.a0f = (float)p.a0;
    p.inv_w0sqf = (float)p.inv_w0sq;
    p.inv_zRf = (float)p.inv_zR;
    p.ellf = (float)p.ell_per_psi;
    p.two_over_aSf = (float)p.two_over_aS;
    p.Kf = (float)p.K;
    p.CDf = (float)p.CD;
    p.psi0f = (float)(-psi_max);
    p.hf = (float)h;
    p.chi_fp64 = (float)N->chi_fp64;
    p.n_steps = N->n_steps;
    p.shot = N->shot;
    p.plane_wave = plane_wave ? 1 : 0;
    {
        // the quadratic midpoint of the spatial factor is used only when one
        // phase step moves a sample much less than the focal scales
        const double step_um = h * p.ell_per_psi;
        const double scale = plane_wave ? 0.0
                                        : std::fmax(p.inv_zR, 6.0 * p.div_rad / L->w0_um);
        p.mid_interp = step_um * scale < 1e-3 ? 1 : 0;
    }
    p.key0 = (uint32_t)N->seed;
    p.key1 = (uint32_t)(N->seed >> 32);
    p.n_samples = n;
    p.env32 = c->env32;
    p.env64 = c->env64;
    p.rad32 = c->rad32;
    p.rad64 = c->rad64;
    p.st = ss;
    p.flags = flags;

    qs::DepParams d{};
    d.n_samples = n;
    d.a0 = L->a0;
    d.gamma0 = B->gamma0;
    d.c_theta = N->c_theta;
    d.deposit = N->deposit;
    d.n_e = H->n_e;
    d.n_th = H->n_th;
    d.n_a = H->n_a;
    d.ksig_bins = N->kernel_sigma_bins;
    d.e_lo = H->e_lo;
    d.e_w = (H->e_hi - H->e_lo) / H->n_e;
    d.th_lo = H->th_lo_mrad;
    d.th_w = (H->th_hi_mrad - H->th_lo_mrad) / H->n_th;
    d.st = ss;
    d.hist = hist;
    d.partials = c->partials;
    d.chimax_bits = chimax_bits;
    d.flags = flags;
    d.rec = O->samples;
    d.rec_stride = O->samples ? O->sample_stride : 1;
    d.rec_n = O->samples ? O->n_sample_records : 0;

    qs::FinParams f{};
    f.n_samples = n;
    f.nblocks = dgrid;
    f.n_e = H->n_e;
    f.n_th = H->n_th;
    f.n_a = H->n_a;
    f.gamma0 = B->gamma0;
    f.hist = hist;
    f.partials = c->partials;
    f.chimax_bits = chimax_bits;
    f.flags = flags;
    f.energy_hist = O->energy_hist;
    f.angle_hist = O->angle_hist;
    f.a0eff_hist = O->a0eff_hist;
    f.moments = O->moments;
    f.status = O->status;

    // ---- enqueue ----
    const bool prof = c->profiling;
    auto mark = [&](int k) { return prof ? hipEventRecord(c->ev[k], s) : hipSuccess; };
    if ((e = mark(0)) != hipSuccess) return hip_fail(c, e, "event record");
    if ((e = qs::launch_envelope(psi_max, h, N->n_steps, L->envelope, omega_tau, c->env32,
                                 c->env64, s)) != hipSuccess)
        return hip_fail(c, e, "envelope kernel");
    if ((e = mark(1)) != hipSuccess) return hip_fail(c, e, "event record");
    if ((e = qs::launch_zero(c->accum, 2 + nh, s)) != hipSuccess)
        return hip_fail(c, e, "zero kernel");
    if ((e = mark(2)) != hipSuccess) return hip_fail(c, e, "event record");
    if ((e = qs::launch_phase(p, prec, N->rr_model, N->amp_mode, s)) != hipSuccess)
        return hip_fail(c, e, "phase kernel");
    if ((e = mark(3)) != hipSuccess) return hip_fail(c, e, "event record");
    if ((e = qs::launch_deposit(d, dgrid, s)) != hipSuccess)
        return hip_fail(c, e, "deposit kernel");
    if ((e = mark(4)) != hipSuccess) return hip_fail(c, e, "event record");
    if ((e = qs::launch_finalize(f, s)) != hipSuccess) return hip_fail(c, e, "finalize kernel");
    if ((e = mark(5)) != hipSuccess) return hip_fail(c, e, "event record");
    c->profiled_call = prof;
    c->last_error[0] = 0;
    return QS_OK;
}

qs_status qs_radiation_eval(qs_ctx *c, int32_t precision, int64_t n, const double *chi,
                            double *out, void *stream) {
    if (!c) return QS_EINVAL;
    if (n < 0 || (n > 0 && (!chi || !out)) ||
        (precision != QS_PREC_FP32 && precision != QS_PREC_FP64))
        return set_err(c, "invalid radiation_eval arguments"), QS_EINVAL;
    DeviceGuard guard(c->device);
    hipError_t e = qs::launch_radiation_eval(c->rad32, c->rad64, precision, n, chi, out,
                                             c->eval_flags, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(c, e, "radiation_eval kernel");
    return QS_OK;
}

qs_status qs_set_profiling(qs_ctx *c, int on) {
    if (!c) return QS_EINVAL;
    DeviceGuard guard(c->device);
    if (on && !c->ev[0]) {
        for (hipEvent_t &ev : c->ev) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_fail(c, e, "event create");
        }
    }
    c->profiling = on != 0;
    c->profiled_call = false;
    return QS_OK;
}

qs_status qs_last_timings(qs_ctx *c, double *ms) {
    if (!c || !ms) return QS_EINVAL;
    if (!c->profiling || !c->profiled_call)
        return set_err(c, "no profiled call"), QS_EINVAL;
    DeviceGuard guard(c->device);
    hipError_t e = hipEventSynchronize(c->ev[5]);
    if (e != hipSuccess) return hip_fail(c, e, "event synchronize");
    for (int k = 0; k < 5; ++k) {
        float t = 0.0f;
        e = hipEventElapsedTime(&t, c->ev[k], c->ev[k + 1]);
        if (e != hipSuccess) return hip_fail(c, e, "event elapsed");
        ms[k] = t;
    }
    return QS_OK;
}

qs_status qs_sync_status(qs_ctx *c, const int32_t *status, void *stream) {
    if (!c || !status) return QS_EINVAL;
    DeviceGuard guard(c->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
    int32_t v = 0;
    e = hipMemcpy(&v, status, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "status copy");
    return (qs_status)v;
}

}  // extern "C"
