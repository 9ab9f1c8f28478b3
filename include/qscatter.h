/*
 * qscatter.h -- C ABI of the MI355X (gfx950) beam-phase-space integrator.
 *
 * The library predicts the asymptotic electron energy and angle distributions,
 * the a0,eff distribution and moments after a relativistic electron beam meets
 * a focused, possibly misaligned, laser pulse head-on (Amaro & Vranic,
 * "QScatter", arXiv 2308.09348: abstract; Sec. 2 eq. dNda0eff and eq. a0eff;
 * Sec. 3 eq. PWCRR and eq. dNda2dNdgf; Sec. 4 eq. dpdtRR; Sec. 5.2).
 *
 * Every step of the computation runs in HIP kernels on the device: sample
 * generation, the per-sample laser amplitude, the phase integration of the
 * radiation-reaction moment system, the deposit into spectra, the reductions
 * and the normalisation.  The host only validates arguments and enqueues work.
 *
 * Conventions
 *   - Plain C types only.  Pointers marked "device" must be device memory of
 *     the context's GPU; pointers marked "host" are read during the call only.
 *   - Calls are asynchronous on the given stream (0 = the null stream).  The
 *     library retains no caller pointer after a call returns.
 *   - Return values are qs_status codes; nothing is enqueued when a call
 *     returns an error (no partial writes).  Errors raised inside kernels
 *     (non-finite states, chi beyond the tabulated range) are written to the
 *     caller's device status word and reported by qs_sync_status().
 *   - One context may be used from one host thread at a time.  Calls that
 *     share a context must be ordered on one stream (they share the
 *     context's device scratch).
 */
#ifndef QSCATTER_H
#define QSCATTER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QS_ABI_VERSION 3

typedef enum qs_status {
    QS_OK = 0,
    QS_EINVAL = 1,        /* an argument failed validation                     */
    QS_ENOMEM = 2,        /* device allocation failed                          */
    QS_EDEVICE = 3,       /* a HIP runtime call failed                         */
    QS_ENONFINITE = 4,    /* a sample reached a non-finite state (device-side) */
    QS_EUNSUPPORTED = 5,  /* valid but not supported by this library           */
    QS_ERANGE = 6         /* chi left the tabulated range [0, 256) (device)    */
} qs_status;

enum { QS_ENV_GAUSS = 0, QS_ENV_SIN2 = 1 };
enum { QS_RR_CLASSICAL = 0, QS_RR_QUANTUM = 1 };
enum { QS_AMP_A0EFF = 0, QS_AMP_LOCAL = 1 };
enum { QS_DEP_POINT = 0, QS_DEP_CIC = 1, QS_DEP_GAUSS = 2 };
enum { QS_PREC_FP32 = 0, QS_PREC_FP64 = 1 };
/* qs_numerics.flags: QS_VALIDATE_FP64 shadows every shadow_stride-th sample
 * of an FP32 pass with the FP64 integration and reports the differences: in
 * the moments QS_M_SHADOW_N .. QS_M_ERR_T_MAX (qs_forward), in
 * qs_photon_outputs.errors (qs_photons) and in qs_grad_outputs.errors
 * (qs_backward). */
enum { QS_VALIDATE_FP64 = 1 };
enum { QS_PROFILE_GAUSS = 0, QS_PROFILE_FLAT = 1 };
/* Transverse laser modes, amplitude only (the wave's phase, Gouy phase and
 * curvature neglected as for eq. a0eff), scaled to a peak of 1 in the focal
 * plane so that a0 stays the peak amplitude; with u = x/W, v = y/W,
 * W = W0 sqrt(1 + z^2/zR^2):
 *   GAUSS: (W0/W) exp(-(u^2 + v^2));
 *   HG:    (W0/W) |H_m(sqrt2 u) H_n(sqrt2 v)| exp(-(u^2 + v^2)) / C_mn;
 *   LG:    (W0/W) (2(u^2 + v^2))^(|l|/2) |L_p^|l|(2(u^2 + v^2))|
 *          exp(-(u^2 + v^2)) / C_pl,
 * H the physicists' Hermite and L the generalised Laguerre polynomials. */
enum { QS_MODE_GAUSS = 0, QS_MODE_HG = 1, QS_MODE_LG = 2 };

/* Laser (Sec. 2 eq. a0eff; misalignment of Table 1).  Lengths in um,
 * times in fs.  The laser propagates along +z with its peak at z = c t and
 * focus at z = 0; linear polarisation along x, carrier resolved, CEP 0. */
typedef struct qs_laser {
    double a0;         /* peak normalised vector potential, >= 0               */
    double lambda_um;  /* central wavelength, > 0                              */
    double w0_um;      /* spot size W0 at focus, >= 0; 0 selects a plane wave  */
    double tau_fs;     /* GAUSS: intensity FWHM; SIN2: rise time; > 0          */
    int32_t envelope;  /* QS_ENV_*                                             */
    int32_t mode;      /* transverse mode, QS_MODE_* (conclusions: Laguerre- or
                          Hermite-Gauss in place of the Gaussian focus)        */
    double x_off_um;   /* beam centroid offset from the laser axis (x)         */
    double y_off_um;   /* beam centroid offset from the laser axis (y)         */
    double delay_fs;   /* collision delay: the centroid meets the peak at
                          z = c delay / 2                                      */
    int32_t mode_m;    /* HG: order in x, 0..8; LG: radial index p, 0..8       */
    int32_t mode_n;    /* HG: order in y, 0..8; LG: azimuthal index l, -8..8   */
} qs_laser;

/* Electron beam (abstract: broadband beams, divergence).  The beam moves
 * along -z; positions are taken when the centroid meets the laser peak.  The
 * density profiles are Gaussian, or flat-top as the Wide and Thin beams of
 * Sec. 2 (Table 1): a uniform disk of radius sigma_r_um and a uniform length
 * sigma_z_um. */
typedef struct qs_beam {
    double gamma0;       /* mean initial Lorentz factor, > 1                   */
    double sigma_gamma;  /* rms of the initial Lorentz factor, >= 0           */
    double sigma_r_um;   /* GAUSS: per-axis rms transverse size; FLAT: radius  */
    double sigma_z_um;   /* GAUSS: rms length; FLAT: full length, >= 0        */
    double div_mrad;     /* per-plane rms divergence, >= 0                    */
    int32_t transverse;  /* QS_PROFILE_*                                      */
    int32_t longitudinal; /* QS_PROFILE_*                                     */
} qs_beam;

/* Numerics of the phase-space quadrature. */
typedef struct qs_numerics {
    int64_t n_samples;        /* Monte-Carlo samples (beam volume elements), 1..2^32 */
    int32_t n_steps;          /* RK4 phase steps across the window, 1..65536 */
    int32_t shot;             /* shot index: second word of the RNG counter  */
    double window_fwhm;       /* GAUSS: window is +-window_fwhm FWHM; > 0     */
    uint64_t seed;            /* Philox4x32-10 key                           */
    int32_t rr_model;         /* QS_RR_CLASSICAL (Landau-Lifshitz, g = 1) or
                                 QS_RR_QUANTUM (Gaunt factor g(chi) and the
                                 diffusion of the energy spread)             */
    int32_t amp_mode;         /* QS_AMP_A0EFF: each sample sees a0,eff at its
                                 collision point (Sec. 2); QS_AMP_LOCAL: the
                                 local amplitude along its ballistic path    */
    int32_t deposit;          /* QS_DEP_POINT, QS_DEP_CIC, QS_DEP_GAUSS       */
    int32_t precision;        /* QS_PREC_FP32 (compensated) or QS_PREC_FP64   */
    double kernel_sigma_bins; /* QS_DEP_GAUSS kernel rms, in bins, >= 0       */
    double chi_fp64;          /* FP32 only: a wavefront runs a phase step in
                                 FP64 when any of its samples has chi above
                                 this at the step start; <= 0 disables        */
    double c_theta;           /* pre-factor of the Sec. 5.2 divergence law    */
    int32_t flags;            /* QS_VALIDATE_FP64 or 0                        */
    int32_t shadow_stride;    /* with QS_VALIDATE_FP64: samples i with
                                 i % shadow_stride == 0 are shadowed; 0 means
                                 64; 1 .. 2^20                               */
} qs_numerics;

/* Histogram windows.  Energy and angle histograms have n bins plus
 * underflow at [n] and overflow at [n+1]; the a0,eff histogram has n_a bins
 * over a0,eff / a0 in [0, 1] (top edge closed). */
typedef struct qs_bins {
    int32_t n_e;         /* energy bins, 1..4096                                */
    int32_t n_th;        /* angle bins (x plane), 1..4096                       */
    int32_t n_a;         /* a0,eff bins, 1..4096                                */
    int32_t reserved0;
    double e_lo, e_hi;   /* energy window in m c^2 (Lorentz factor), hi > lo    */
    double th_lo_mrad, th_hi_mrad; /* angle window, hi > lo                     */
} qs_bins;

/* Moments written to qs_outputs.moments (QS_M_N doubles). */
enum {
    QS_M_WEIGHT = 0,    /* number of samples                                    */
    QS_M_MEAN_G,        /* mean final Lorentz factor                            */
    QS_M_STD_G,         /* std of the final energy law (incl. beamlet spread)   */
    QS_M_MEAN_THX,      /* mean angle, polarisation plane [mrad]                */
    QS_M_RMS_THX,       /* rms angle incl. the Sec. 5.2 broadening [mrad]       */
    QS_M_MEAN_THY,      /* mean angle, other plane [mrad]                       */
    QS_M_RMS_THY,       /* rms angle, other plane [mrad]                        */
    QS_M_MEAN_AEFF,     /* mean a0,eff                                          */
    QS_M_MAX_CHI,       /* largest chi met at a step start                      */
    QS_M_RAD_FRAC,      /* mean radiated energy fraction                        */
    QS_M_MEAN_SIGF,     /* mean beamlet energy spread sigma_f                   */
    /* FP64 shadow of an FP32 pass (QS_VALIDATE_FP64; zero otherwise and for
     * FP64 passes): over the shadowed samples, the final state of this pass
     * (mu32, sig32) against the FP64 integration of the same samples
     * (mu64, sig64), sig = sqrt(max(sig2, 0)). */
    QS_M_SHADOW_N,      /* shadowed samples                                     */
    QS_M_ERR_MU_MAX,    /* max |mu32 - mu64| / mu64                             */
    QS_M_ERR_MU_MEAN,   /* mean (mu32 - mu64) / mu64 (signed)                   */
    QS_M_ERR_SIG_MAX,   /* max |sig32 - sig64| / mu64                           */
    QS_M_ERR_MEAN_G,    /* mean (mu32 - mu64): the FP32 bias of QS_M_MEAN_G     */
    /* ... and the spectra: D_k = sum over the shadowed samples of the bin-k
     * mass of the law deposited from (mu32, sig32) minus that from (mu64,
     * sig64) (both CDFs exact in FP64, so D is the trajectories' part of the
     * FP32 error); per shadowed sample, i.e. as a fraction of the weight: */
    QS_M_ERR_E_L1,      /* sum_k |D_k| / n over the energy bins (+ under/over)  */
    QS_M_ERR_E_MAX,     /* max_k |D_k| / n, energy                              */
    QS_M_ERR_T_L1,      /* the same for the angle histogram                     */
    QS_M_ERR_T_MAX,
    /* Precision of the phase steps (R21 of the FP64 promotion rule): the share
     * of the pass's wavefront phase steps taken in FP64 -- 1 for QS_PREC_FP64,
     * 0 for FP32 without chi_fp64, the promoted share otherwise (promoted
     * wave-steps over ceil(n_samples / 64) x n_steps).  qs_forward and
     * qs_forward_batched count it; the derivative-tape and plane-wave
     * reconstruction passes report -1 (not counted). */
    QS_M_FP64_STEPS,
    QS_M_N = 21
};

/* Per-sample record (QS_S_N doubles) for diagnostics and parity checks. */
enum {
    QS_S_MU = 0, QS_S_SIG2, QS_S_THX, QS_S_THY, QS_S_SIGTH, QS_S_AEFF, QS_S_CHIMAX,
    QS_S_GAMMA0, QS_S_X, QS_S_Y, QS_S_Z, QS_S_N
};

/* Outputs: all device pointers, caller-allocated, fully overwritten. */
typedef struct qs_outputs {
    double *energy_hist;  /* [n_e + 2] weight per bin (one unit per sample)      */
    double *angle_hist;   /* [n_th + 2]                                          */
    double *a0eff_hist;   /* [n_a]                                               */
    double *moments;      /* [QS_M_N]                                            */
    int32_t *status;      /* [1] qs_status of the device-side checks             */
    double *samples;      /* optional [n_sample_records][QS_S_N]: records of
                             samples i = r * sample_stride; NULL for none       */
    int64_t sample_stride;     /* >= 1 when samples != NULL                      */
    int64_t n_sample_records;  /* records written (those with i < n_samples)     */
} qs_outputs;

typedef struct qs_ctx qs_ctx;

/* Create a context on HIP device `device`: builds the radiation-function
 * tables (g, chi g', chi^2 g'', h of the LCFA spectrum, Sec. 4 eq. dpdtRR) on
 * the device.  *ctx receives the handle; on error it is set to NULL.
 * Errors: QS_EINVAL (ctx NULL or no such device), QS_ENOMEM, QS_EDEVICE. */
qs_status qs_create(qs_ctx **ctx, int device);

/* Release the context and its device memory.  Waits for the device.  NULL
 * is accepted. */
void qs_destroy(qs_ctx *ctx);

/* One forward pass (abstract; Sec. 2-3 and 5.2): draw n_samples beam samples,
 * integrate each sample's mean energy and energy variance along the laser
 * phase under classical (eq. PWCRR) or quantum-corrected (eq. dpdtRR)
 * radiation reaction, and deposit the final laws into the histograms
 * (eq. dNda2dNdgf as a push-forward) and moments.  `stream` is a hipStream_t
 * (void* here so the header needs no HIP include).  Results are deterministic
 * for a given device and arguments.
 * Errors: QS_EINVAL (any NULL struct or output pointer, a value outside its
 * documented range, a non-finite input), QS_ENOMEM, QS_EDEVICE. */
qs_status qs_forward(qs_ctx *ctx, const qs_laser *laser, const qs_beam *beam,
                     const qs_numerics *num, const qs_bins *bins,
                     const qs_outputs *out, void *stream);

/* Largest n_samples of qs_forward_noalloc. */
#define QS_NOALLOC_MAX_SAMPLES (1 << 20)

/* qs_forward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same pass, kernels and results (bit for bit) as qs_forward, with every
 * piece of device scratch -- the per-sample final states, the envelope
 * tables, the accumulators, the moment partials and the device shot table --
 * taken from one static device array of about 55 MiB that each GPU the library
 * runs on holds until the process ends (its address is looked up by
 * qs_create, which also makes the call's pinned staging block and event).
 * The call itself allocates nothing: no hipMalloc, hipFree or allocating
 * library routine, and it never captures a HIP graph.  Limits: one shot of at
 * most QS_NOALLOC_MAX_SAMPLES samples; every other size as qs_forward (steps
 * up to 65536, bins up to 4096 each).  The caller still owns and passes the
 * outputs.  Every call on a GPU shares that GPU's array and leaves its
 * contents behind (the accumulators are cleared by a kernel at the start of
 * each call): calls that overlap on one GPU -- on different streams, or from
 * different contexts on the same device -- race and give wrong results;
 * order them on one stream.
 * Errors: as qs_forward; QS_EINVAL for n_samples above
 * QS_NOALLOC_MAX_SAMPLES; QS_EUNSUPPORTED for QS_VALIDATE_FP64 (the FP64
 * shadow needs scratch of its own). */
qs_status qs_forward_noalloc(qs_ctx *ctx, const qs_laser *laser, const qs_beam *beam,
                             const qs_numerics *num, const qs_bins *bins,
                             const qs_outputs *out, void *stream);

/* Many shots in one launch (the high-repetition-rate use of the abstract and
 * the conclusions): shot k uses lasers[k], beams[k], bins[k], outs[k] and
 * n_samples[k] samples, and the shared numerics (num->n_samples is ignored;
 * shot k draws its samples with RNG counter word num->shot + k).  All host
 * arrays have n_shots entries; the outputs are device pointers as in
 * qs_forward.  Shot k gives bit-for-bit the result of qs_forward with
 * num->shot + k and n_samples[k].  The shots must share lambda_um, tau_fs and
 * envelope (one phase grid serves them all): otherwise QS_EUNSUPPORTED.
 * At most 2^20 shots and 2^36 samples in total.
 * Errors: QS_EINVAL (as qs_forward, per shot), QS_EUNSUPPORTED, QS_ENOMEM,
 * QS_EDEVICE. */
qs_status qs_forward_batched(qs_ctx *ctx, int32_t n_shots, const qs_laser *lasers,
                             const qs_beam *beams, const int64_t *n_samples,
                             const qs_numerics *num, const qs_bins *bins,
                             const qs_outputs *outs, void *stream);

/* Evaluate the device radiation-function approximation at n values of chi
 * (device arrays): out[4*k + {0,1,2,3}] = {g, chi g', chi^2 g'', h} at
 * chi[k], in FP32 (precision QS_PREC_FP32) or FP64.  Diagnostic entry point
 * for parity checks of the tables against their definition (Sec. 4).
 * Errors: QS_EINVAL, QS_EDEVICE. */
qs_status qs_radiation_eval(qs_ctx *ctx, int32_t precision, int64_t n, const double *chi,
                            double *out, void *stream);

/* Parameters the adjoint differentiates with respect to: index into
 * qs_grad_outputs.grad.  Units as in qs_laser / qs_beam (um, fs, mrad). */
enum {
    QS_P_A0 = 0,       /* qs_laser.a0          */
    QS_P_W0,           /* qs_laser.w0_um       */
    QS_P_X_OFF,        /* qs_laser.x_off_um    */
    QS_P_Y_OFF,        /* qs_laser.y_off_um    */
    QS_P_DELAY,        /* qs_laser.delay_fs    */
    QS_P_GAMMA0,       /* qs_beam.gamma0       */
    QS_P_SIGMA_GAMMA,  /* qs_beam.sigma_gamma  */
    QS_P_DIV,          /* qs_beam.div_mrad     */
    QS_P_N
};

/* Adjoint inputs and outputs of one shot: device pointers, caller-allocated. */
typedef struct qs_grad_outputs {
    const double *d_energy_hist; /* in: [n_e + 2] dL/dH for the energy histogram of
                                    qs_forward (bins, underflow, overflow), or NULL */
    double *grad;                /* out: [QS_P_N] dL/dp                           */
    int32_t *status;             /* out: [1] qs_status of the device-side checks,
                                    or NULL                                       */
    const double *d_angle_hist;  /* in: [n_th + 2] dL/dH for the angle histogram,
                                    or NULL                                       */
    const double *d_moments;     /* in: [QS_M_N] dL/dM for the moments, or NULL;
                                    the weight, QS_M_MAX_CHI and the FP64-shadow
                                    fields carry no derivative (their entries are
                                    not read)                                     */
    const double *moments;       /* in: [QS_M_N] the moments qs_forward returned for
                                    the same arguments (needed with d_moments: the
                                    derivatives of the std and rms moments depend
                                    on their values)                              */
    double *errors;              /* out: optional [QS_GE_N] FP64-shadow report, or
                                    NULL; zero-filled unless an FP32 pass runs with
                                    QS_VALIDATE_FP64                              */
} qs_grad_outputs;

/* FP64 shadow of an FP32 adjoint (QS_VALIDATE_FP64): the gradient of the
 * view that holds every shadow_stride-th sample (the same upstream weights
 * and forward moments; the view's weight is its own sample count) is taken
 * twice, at the pass's precision (FP32, with its chi_fp64 rule) and in FP64,
 * both by integrating the trajectories with their tangents, and
 * qs_grad_outputs.errors receives: */
enum {
    QS_GE_SHADOW_N = 0,            /* samples in the view                          */
    QS_GE_DIFF = 1,                /* + p: dL/dp of the view, FP32 minus FP64     */
    QS_GE_REF = 1 + QS_P_N,        /* + p: dL/dp of the view in FP64 (the scale)   */
    QS_GE_N = 1 + 2 * QS_P_N
};

/* Adjoint of the forward outputs (the parameter-reconstruction use the
 * abstract and the conclusions give for the method's speed): for
 * L = sum_k w_k H_k + sum_k u_k T_k + sum_m v_m M_m with w = d_energy_hist,
 * u = d_angle_hist, v = d_moments (each optional, at least one given) and H,
 * T, M the energy histogram, angle histogram and moments that qs_forward
 * returns for the same arguments, write dL/dp for the QS_P_* parameters.
 * The angle law's centre is the initial angle (a function of the divergence)
 * and its width the Sec. 5.2 broadening, which depends on a0,eff and on the
 * final energy state.  Each sample's trajectory (Sec. 2-4, as in qs_forward) is
 * integrated again together with its forward-mode tangents, i.e. the exact
 * derivatives of the discrete RK4 map, and contracted with the derivative of
 * the sample's deposited law at the bin edges (the smooth law, without the
 * forward pass's 2^-32 quantisation and 6-sigma cut).  The quantum model
 * needs chi^3 g''' and chi h', tabulated on the device like g and h.
 * precision QS_PREC_FP64 integrates in FP64; QS_PREC_FP32 in compensated
 * FP32 with FP32 tangents, and with chi_fp64 > 0 (quantum model) takes FP64
 * steps where qs_forward does: the state advances by the forward pass's FP64
 * step, the FP32 tangents by the step's linearisation at the state rounded to
 * FP32.  num->deposit may be any of the
 * three kernels; n_samples and the RNG stream as in qs_forward, so the
 * derivative is that of the same Monte-Carlo estimate.
 * Errors: QS_EINVAL (as qs_forward; NULL grad; no upstream weights;
 * d_moments without moments),
 * QS_ENOMEM, QS_EDEVICE. */
qs_status qs_backward(qs_ctx *ctx, const qs_laser *laser, const qs_beam *beam,
                      const qs_numerics *num, const qs_bins *bins, const qs_grad_outputs *out,
                      void *stream);

/* The adjoint of qs_forward_batched: shot k as qs_backward with outs[k], RNG
 * counter word num->shot + k and n_samples[k] samples; same batch rules
 * (shared lambda_um, tau_fs and envelope, else QS_EUNSUPPORTED).  Shot k gives
 * bit-for-bit the result of qs_backward with num->shot + k.
 * Errors: QS_EINVAL, QS_EUNSUPPORTED, QS_ENOMEM, QS_EDEVICE. */
qs_status qs_backward_batched(qs_ctx *ctx, int32_t n_shots, const qs_laser *lasers,
                              const qs_beam *beams, const int64_t *n_samples,
                              const qs_numerics *num, const qs_bins *bins,
                              const qs_grad_outputs *outs, void *stream);

/* Fields of a derivative tape (doubles, structure of arrays): field f of
 * sample i of shot k is at tape[f * n_total + off_k + i], with n_total the
 * samples of the whole call and off_k those of the shots before k.
 * Fields: QS_T_MU final mean energy mu_f, QS_T_SIG2 final variance sig2_f,
 * QS_T_DMU + p = d mu_f / d p, QS_T_DSIG2 + p = d sig2_f / d p (p a QS_P_*). */
enum { QS_T_MU = 0, QS_T_SIG2 = 1, QS_T_DMU = 2, QS_T_DSIG2 = 2 + QS_P_N,
       QS_TAPE_FIELDS = 2 + 2 * QS_P_N };

/* qs_forward that also records the derivative tape (device, caller-allocated,
 * QS_TAPE_FIELDS * n_samples doubles, overwritten): each sample's trajectory
 * is integrated together with its tangents (as qs_backward does), its final
 * state goes to the deposit as in qs_forward, and mu_f, sig2_f and their
 * derivatives go to the tape.  The histograms and moments agree with
 * qs_forward's to the parity tolerances (not bit for bit: the FP32 step
 * arithmetic differs), and qs_backward_tape on the tape then costs one read
 * of it instead of a second integration.  Errors: as qs_forward; QS_EINVAL
 * for a NULL tape. */
qs_status qs_forward_tape(qs_ctx *ctx, const qs_laser *laser, const qs_beam *beam,
                          const qs_numerics *num, const qs_bins *bins, const qs_outputs *out,
                          double *tape, void *stream);

/* qs_forward_batched with a tape over all shots (n_total = sum of n_samples). */
qs_status qs_forward_tape_batched(qs_ctx *ctx, int32_t n_shots, const qs_laser *lasers,
                                  const qs_beam *beams, const int64_t *n_samples,
                                  const qs_numerics *num, const qs_bins *bins,
                                  const qs_outputs *outs, double *tape, void *stream);

/* qs_backward from a tape recorded by qs_forward_tape with the same
 * arguments: dL/dp = sum_i (dL/dmu_i d mu_i/dp + dL/dsig2_i d sig2_i/dp) with
 * the law sensitivities of qs_backward (read-only tape).  Errors: as
 * qs_backward; QS_EINVAL for a NULL tape. */
qs_status qs_backward_tape(qs_ctx *ctx, const qs_laser *laser, const qs_beam *beam,
                           const qs_numerics *num, const qs_bins *bins,
                           const qs_grad_outputs *out, const double *tape, void *stream);

/* qs_backward_batched from a batched tape. */
qs_status qs_backward_tape_batched(qs_ctx *ctx, int32_t n_shots, const qs_laser *lasers,
                                   const qs_beam *beams, const int64_t *n_samples,
                                   const qs_numerics *num, const qs_bins *bins,
                                   const qs_grad_outputs *outs, const double *tape,
                                   void *stream);

/* Photon-energy bins: n_ph bins over [ph_lo, ph_hi) in m c^2 units, plus
 * underflow [n_ph] and overflow [n_ph + 1]. */
typedef struct qs_photon_bins {
    int32_t n_ph;        /* 1..4096                                            */
    int32_t reserved0;
    double ph_lo, ph_hi; /* 0 <= ph_lo < ph_hi                                 */
} qs_photon_bins;

/* Photon outputs of one shot: device pointers, caller-allocated. */
typedef struct qs_photon_outputs {
    double *photon_hist; /* [n_ph + 2] expected photon number per bin, summed
                            over the samples (one electron each)              */
    double *energy;      /* [2]: emitted photon energy, and the electrons'
                            energy loss sum(gamma0_i - mu_f), m c^2 units      */
    int32_t *status;     /* [1] qs_status of the device-side checks, or NULL   */
    double *angles;      /* optional [6] (NULL: not computed), Sec. 5.1: the
                            emitted photon number (all energies), its rms
                            angles theta_x, theta_y [mrad]; the emitted photon
                            energy, its rms theta_x, theta_y [mrad].  A stage
                            emits along (theta_x + a/mu, theta_y), the sample's
                            direction plus the quiver angle in the polarisation
                            plane, within a 1/mu cone per plane; each stage's
                            photons weigh by their number (the paper's
                            N_gamma/N_e weighting) or by their energy        */
    double *errors;      /* optional [QS_PE_N] FP64-shadow report, or NULL;
                            zero-filled unless an FP32 pass runs with
                            QS_VALIDATE_FP64                                  */
} qs_photon_outputs;

/* FP64 shadow of an FP32 photon pass (QS_VALIDATE_FP64): the view that holds
 * every shadow_stride-th sample is integrated twice, at the pass's precision
 * (FP32, with its chi_fp64 rule) and in FP64, on the same emission grid, and
 * qs_photon_outputs.errors receives (X32, X64: the view's outputs): */
enum {
    QS_PE_SHADOW_N = 0,  /* samples in the view                                 */
    QS_PE_HIST_L1,       /* sum_k |H32_k - H64_k| / sum_k H64_k, over the n_ph + 2
                            bins of photon_hist                                 */
    QS_PE_HIST_MAX,      /* max_k |H32_k - H64_k| / sum_k H64_k                  */
    QS_PE_ENERGY,        /* (E32 - E64) / E64 of the emitted energy (energy[0])  */
    QS_PE_LOSS,          /* the same for the electrons' energy loss (energy[1])  */
    QS_PE_ANGLES,        /* + j, j < 6: (A32_j - A64_j) / A64_j of angles[j] (0
                            without angles or where A64_j is 0)                */
    QS_PE_REF_PHOTONS = QS_PE_ANGLES + 6, /* the scales: sum_k H64_k,          */
    QS_PE_REF_ENERGY,    /* E64,                                                */
    QS_PE_REF_LOSS,      /* and the FP64 energy loss of the view                */
    QS_PE_N
};

/* The approximate photon spectrum of Sec. 4: along each sample's trajectory
 * (integrated as in qs_forward) every phase pairs the mean energy with the
 * instantaneous amplitude and emits the LCFA quantum-synchrotron spectrum of
 * chi = 2 gamma |a| / a_S; the spectra are integrated over the phase with the
 * RK4 stage weights.  On the device each stage deposits its emission weight
 * into an emission grid over (ln chi, ln mu) (bilinear, 0.2 in ln chi, at
 * most 64 columns over the shot's energy range), which is contracted with
 * the tabulated LCFA number spectrum: about 1e-3 of the spectrum in L1.  The
 * emitted photon energy (energy[0]) is summed exactly per stage; in the
 * classical model it equals the electrons' energy loss (energy[1]).  With
 * QS_PREC_FP32 and chi_fp64 > 0 (quantum model) the steps that qs_forward
 * takes in FP64 are taken in FP64 here too, emission included.
 * Errors: QS_EINVAL (as qs_forward; photon bins out of range; NULL outputs),
 * QS_ENOMEM, QS_EDEVICE.  Device status QS_ERANGE: a stage left the grid. */
qs_status qs_photons(qs_ctx *ctx, const qs_laser *laser, const qs_beam *beam,
                     const qs_numerics *num, const qs_photon_bins *bins,
                     const qs_photon_outputs *out, void *stream);

/* qs_photons over many shots in one launch (rules of qs_forward_batched;
 * shot k uses RNG counter word num->shot + k). */
qs_status qs_photons_batched(qs_ctx *ctx, int32_t n_shots, const qs_laser *lasers,
                             const qs_beam *beams, const int64_t *n_samples,
                             const qs_numerics *num, const qs_photon_bins *bins,
                             const qs_photon_outputs *outs, void *stream);

/* The device's LCFA number CDF Phi(xi; chi) = Int_0^xi F(xi', chi) dxi' at n
 * points (device arrays; diagnostic entry point for parity checks).
 * Errors: QS_EINVAL, QS_EDEVICE. */
qs_status qs_photon_cdf(qs_ctx *ctx, int64_t n, const double *chi, const double *xi,
                        double *out, void *stream);

/* Evaluate the derivative tables that the adjoint uses at n values of chi
 * (device arrays): out[6*k + {0..5}] = {g, chi g', chi^2 g'', h, chi^3 g''',
 * chi h'} at chi[k], FP32 or FP64 (Sec. 4 eq. dpdtRR; diagnostic entry point).
 * Errors: QS_EINVAL, QS_EDEVICE. */
qs_status qs_radiation_derivs(qs_ctx *ctx, int32_t precision, int64_t n, const double *chi,
                              double *out, void *stream);

/* Node grid of the plane-wave reconstruction of one shot.  a0,eff nodes
 * a_k = a0 k / (n_a - 1), k = 0 .. n_a - 1; gamma0 nodes gamma_m = gamma0 +
 * 6 sigma_gamma (2 m / (n_g - 1) - 1), m = 0 .. n_g - 1 (six standard
 * deviations hold every drawn sample); node index k n_g + m. */
typedef struct qs_node_grid {
    int32_t n_a;          /* >= 2                                                */
    int32_t n_g;          /* >= 2 when sigma_gamma > 0, exactly 1 when it is 0   */
    double *node_states;  /* optional device [n_a n_g][5]: a0,eff, gamma0, mu_f,
                             sig2_f, largest chi at a step start; NULL for none */
    double *node_weights; /* optional device [n_a n_g]: the samples' bilinear
                             weights summed per node (they add up to
                             n_samples); NULL for none                         */
} qs_node_grid;

/* The A0EFF forward pass by the paper's plane-wave reconstruction (Sec. 3.2:
 * the 3D spectrum from plane-wave runs over a uniform a0,eff set weighted by
 * dN_b/da0,eff; Sec. 3.3 for the quantum case).  The moment system runs once
 * per node of `grid` (the plane-wave runs); each sample, drawn as in
 * qs_forward, takes the bilinear interpolant of the nodes' final mean,
 * variance and largest chi at its (a0,eff, gamma0_i) and is deposited as in
 * qs_forward (histograms, moments, Sec. 5.2 width from its interpolated state
 * and its own a0,eff).  The result converges to qs_forward's at second order
 * in the node spacing.  num->amp_mode must be QS_AMP_A0EFF; num->precision
 * and chi_fp64 apply to the node runs; sample records (out->samples) hold the
 * interpolated state, with QS_S_X .. QS_S_Z zero as in qs_forward.  When
 * grid->node_weights is requested, n_a n_g 8-byte words must fit the 160 KiB
 * LDS of a CU (20480 nodes); at most 2^20 nodes otherwise.
 * Errors: QS_EINVAL (as qs_forward; grid NULL or out of range; amp_mode not
 * A0EFF), QS_ENOMEM, QS_EDEVICE. */
qs_status qs_forward_factorised(qs_ctx *ctx, const qs_laser *laser, const qs_beam *beam,
                                const qs_numerics *num, const qs_bins *bins,
                                const qs_node_grid *grid, const qs_outputs *out, void *stream);

/* qs_forward_factorised over many shots in one launch (rules of
 * qs_forward_batched; shot k uses grids[k] and RNG counter word num->shot + k,
 * and gives bit-for-bit the single-shot result with num->shot + k). */
qs_status qs_forward_factorised_batched(qs_ctx *ctx, int32_t n_shots, const qs_laser *lasers,
                                        const qs_beam *beams, const int64_t *n_samples,
                                        const qs_numerics *num, const qs_bins *bins,
                                        const qs_node_grid *grids, const qs_outputs *outs,
                                        void *stream);

/* Synchronise `stream` and return the device status word of the last call
 * that wrote `status` (device pointer) -- QS_OK, QS_ENONFINITE or QS_ERANGE. */
qs_status qs_sync_status(qs_ctx *ctx, const int32_t *status, void *stream);

/* Enable (on != 0) or disable event timing of the kernels that qs_forward
 * enqueues on this context.  Events are recorded on the caller's stream
 * between the launches, so they bracket each kernel.  Every call (also one
 * that leaves profiling on) starts a new count for qs_timings_sum.  Errors:
 * QS_EINVAL, QS_EDEVICE. */
qs_status qs_set_profiling(qs_ctx *ctx, int on);

/* Durations in milliseconds of the kernels of the last qs_forward enqueued
 * with profiling on: ms[0] envelope table, ms[1] accumulator clear, ms[2]
 * phase integration, ms[3] deposit, ms[4] finalize (host array of 5).  After
 * qs_forward_factorised: ms[2] node runs, ms[3] interpolation pass, ms[4]
 * deposit and finalize.
 * Waits for that call's last event.  Errors: QS_EINVAL (profiling off or no
 * profiled call yet), QS_EDEVICE. */
qs_status qs_last_timings(qs_ctx *ctx, double *ms);

/* Sums of the kernel durations that qs_last_timings reports, over the last
 * min(n, 64) calls enqueued with profiling on since it was switched on (n of
 * them): ms[0..4] as there (host array of 5), *n_calls the number of calls
 * summed.  The events of up to 64 calls are kept, so calls can be enqueued
 * back to back and read once at the end.  Waits for each summed call's last
 * event.  Errors: QS_EINVAL (profiling off or no profiled call yet),
 * QS_EDEVICE. */
qs_status qs_timings_sum(qs_ctx *ctx, int32_t *n_calls, double *ms);

/* Launch choices for a class of forward launches (qs_tune).  None of them
 * changes a result bit: moment partial sums are kept per tile of 1024
 * samples whatever the deposit tile. */
typedef struct qs_tuning {
    int32_t dep_tile;    /* samples of one deposit work item: 1024 .. 8192      */
    int32_t phase_cap;   /* resident phase blocks per compute unit at most; 0 =
                            as many as fit                                    */
    int32_t dep_cap;     /* the same for the deposit kernel                     */
    int32_t from_cache;  /* 1: read from the cache file, nothing was timed      */
    double phase_ms;     /* phase kernel time of the choice (from the cache if
                            from_cache)                                       */
    double deposit_ms;   /* deposit kernel time of the choice                   */
} qs_tuning;

/* Tune the forward launches of one class (batching of the high-repetition-
 * rate use in the abstract and the conclusions: many shots, each launch
 * sized to the machine).  The class is (n_steps, rr_model, amp_mode,
 * deposit, precision with its FP64 steps, the largest histogram word count
 * n_e + n_th + n_a + 4 of a shot, floor(log2 total samples), floor(log2
 * n_shots)); it is taken from a batch given as to qs_forward_batched
 * (n_shots >= 1 entries in lasers, beams, n_samples and bins; num->n_samples
 * is ignored).  The call times forward launches of that batch on `stream`
 * under each candidate (phase blocks per CU in {all, 3, 2}, then deposit
 * tile in {1024, 2048, 4096, 8192} x deposit blocks per CU in {all, 4, 2}),
 * keeps the fastest for later launches of the class on this context and,
 * when cache_path is not NULL, appends it to that text file as one line
 * keyed by the device (architecture and compute-unit count) and the class.
 * A cache line for this device and class is used instead of timing.  `out`
 * (host, optional) receives the choice.  Blocks until the trial launches
 * end; allocates its own trial outputs.  Launches of other classes keep the
 * defaults (deposit tile 4096, all resident blocks).
 * Errors: QS_EINVAL (as qs_forward_batched; a cache file that cannot be
 * appended to), QS_EUNSUPPORTED, QS_ENOMEM, QS_EDEVICE. */
qs_status qs_tune(qs_ctx *ctx, int32_t n_shots, const qs_laser *lasers, const qs_beam *beams,
                  const int64_t *n_samples, const qs_numerics *num, const qs_bins *bins,
                  const char *cache_path, qs_tuning *out, void *stream);

/* Enable (on != 0) or disable HIP graphs for qs_forward and
 * qs_forward_batched on this context: the device work of a launch after the
 * shot-table copy (envelope table, accumulator clear, phase, deposit,
 * finalize kernels) is captured once into a graph and replayed by later
 * launches whose kernel arguments are byte-identical (same shapes, sample
 * counts, numerics and scratch buffers; the per-shot parameters and output
 * pointers travel in the shot table, which is copied before every replay).
 * Up to 8 graphs are kept.  Results are the same bits as without graphs.
 * Profiled launches and derivative-tape launches are not captured.
 * Errors: QS_EINVAL (ctx NULL). */
qs_status qs_set_graphs(qs_ctx *ctx, int on);

/* Static description of a status code. */
const char *qs_strerror(qs_status s);

/* Detail of the last error raised on this context (empty if none). */
const char *qs_last_error(qs_ctx *ctx);

/* QS_ABI_VERSION of the built library. */
int qs_abi_version(void);

/* Build provenance: the SHA-256 (64 hex digits) of the sources, headers and
 * compiler flags the library was built from, or "unknown" for a build that
 * did not stamp it.  Static string; never NULL. */
const char *qs_build_id(void);

#ifdef __cplusplus
}
#endif
#endif /* QSCATTER_H */
