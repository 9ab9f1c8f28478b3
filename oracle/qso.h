/*
 * qso.h -- FP64 CPU oracle for the QScatter beam-phase-space integration.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the HIP library, and the HIP library never calls it.
 *
 * What it computes (Amaro & Vranic, "QScatter", arXiv 2308.09348):
 *   - each Monte-Carlo sample of the electron beam (a "volume element" in the
 *     sense of Sec. 2, eq. dNda0eff) meets the focused Gaussian pulse of
 *     eq. a0eff with spatial and temporal misalignment (Table 1 geometry);
 *   - it evolves its mean energy mu and energy variance sig2 along the laser
 *     phase under the radiation-reaction drift of eq. dpdtRR (classical
 *     Landau-Lifshitz when g = 1, which integrates to eq. PWCRR) closed at
 *     second order (Fokker-Planck regime named in Sec. 1);
 *   - it is deposited into energy / angle / a0,eff histograms and moments
 *     (eq. dNda2dNdgf as a push-forward; electron divergence of Sec. 5.2).
 *
 * Every floating-point step is FP64.  Parity unpinned: the sigma_f moment
 * closure physics, h(chi) as a physical model, the Sec. 5.2 angular broadening
 * and its pre-factor (see the test suite for what each pin covers).
 */
#ifndef QSO_H
#define QSO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { QSO_ENV_GAUSS = 0, QSO_ENV_SIN2 = 1 };
enum { QSO_RR_CLASSICAL = 0, QSO_RR_QUANTUM = 1 };
enum { QSO_AMP_A0EFF = 0, QSO_AMP_LOCAL = 1 };
enum { QSO_DEP_POINT = 0, QSO_DEP_CIC = 1, QSO_DEP_GAUSS = 2 };
enum { QSO_PROFILE_GAUSS = 0, QSO_PROFILE_FLAT = 1 };
enum { QSO_MODE_GAUSS = 0, QSO_MODE_HG = 1, QSO_MODE_LG = 2 };

/* One scattering problem.  Lengths in micrometres, times in femtoseconds,
 * angles in milliradians, energies in units of m c^2. */
typedef struct qso_problem {
    /* laser */
    double a0;          /* peak normalised vector potential                    */
    double lambda_um;   /* central wavelength                                  */
    double w0_um;       /* focal spot size W0; 0 means plane wave (S = 1)      */
    double tau_fs;      /* GAUSS: intensity FWHM; SIN2: rise time (0 -> peak)  */
    double x_off_um;    /* beam centroid offset from the laser axis, x         */
    double y_off_um;    /* beam centroid offset from the laser axis, y         */
    double delay_fs;    /* collision delay; centroid meets the peak at z=c*d/2 */
    /* beam */
    double gamma0;      /* mean initial Lorentz factor                         */
    double sigma_gamma; /* rms of the initial Lorentz factor (absolute)        */
    double sigma_r_um;  /* per-axis rms transverse size                        */
    double sigma_z_um;  /* rms length                                          */
    double div_mrad;    /* per-plane rms divergence                            */
    /* numerics */
    double window_fwhm; /* GAUSS: phase window is +-window_fwhm * FWHM         */
    double kernel_sigma_bins; /* GAUSS deposit: kernel rms in bins             */
    double c_theta;     /* pre-factor of the Sec. 5.2 divergence scaling       */
    uint64_t seed;
    int64_t n_samples;
    int32_t n_steps;
    int32_t shot;
    int32_t envelope;
    int32_t rr_model;
    int32_t amp_mode;
    int32_t deposit;
    /* bins */
    int32_t n_e, n_th, n_a;
    int32_t transverse;   /* QSO_PROFILE_GAUSS: rms sigma_r_um per axis;
                             QSO_PROFILE_FLAT: uniform disk of radius sigma_r_um */
    int32_t longitudinal; /* QSO_PROFILE_GAUSS: rms sigma_z_um;
                             QSO_PROFILE_FLAT: uniform over a length sigma_z_um */
    int32_t mode;         /* QSO_MODE_GAUSS, QSO_MODE_HG (orders mode_m in x,
                             mode_n in y), QSO_MODE_LG (p = mode_m, l = mode_n) */
    int32_t mode_m, mode_n;
    double e_lo, e_hi;          /* energy window, units of m c^2          */
    double th_lo_mrad, th_hi_mrad;
} qso_problem;

/* Per-sample record (index order of the doubles). */
enum {
    QSO_S_MU = 0,     /* final mean Lorentz factor mu_f                     */
    QSO_S_SIG2,       /* final energy variance sig2_f                       */
    QSO_S_THX,        /* final angle in the polarisation plane [mrad]       */
    QSO_S_THY,        /* final angle out of that plane [mrad]               */
    QSO_S_SIGTH,      /* Sec. 5.2 broadening rms in x [mrad]                */
    QSO_S_AEFF,       /* a0,eff at the collision point                      */
    QSO_S_CHIMAX,     /* max chi at the step starts                         */
    QSO_S_GAMMA0,     /* the sample's initial Lorentz factor                */
    QSO_S_X, QSO_S_Y, QSO_S_Z, /* sample position [um]                      */
    QSO_S_N           /* record length                                      */
};

/* Moments output (16 doubles). */
enum {
    QSO_M_WEIGHT = 0, QSO_M_MEAN_G, QSO_M_STD_G, QSO_M_MEAN_THX, QSO_M_RMS_THX,
    QSO_M_MEAN_THY, QSO_M_RMS_THY, QSO_M_MEAN_AEFF, QSO_M_MAX_CHI,
    QSO_M_RAD_FRAC, QSO_M_MEAN_SIGF, QSO_M_N = 16
};

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void qso_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* The six standard normals of sample i of a shot (Box-Muller). */
void qso_normals(uint64_t seed, int32_t shot, int64_t i, double out[6]);

/* Radiation functions by direct quadrature (slow): g and h. */
void qso_gh_quadrature(double chi, double *g, double *h);
/* Same from the interpolation table used by the ODE: g, G1=chi g', G2=chi^2 g'', h. */
void qso_radiation(double chi, double out[4]);
/* Right-hand side of the moment system at amplitude a:
 * out = {A, A', A'', D, dmu/dpsi, dsig2/dpsi}. */
int qso_rhs(const qso_problem *p, double mu, double sig2, double a, double out[6]);
/* Laser amplitude along the phase axis: envelope * carrier at psi. */
double qso_envelope_carrier(const qso_problem *p, double psi);
/* Derived scalars: {omega0 [rad/fs], a_S, K, C_D, zR [um], psi_max, h}. */
int qso_derived(const qso_problem *p, double out[7]);

/* One sample's full trajectory and observables; rec has QSO_S_N doubles. */
int qso_sample(const qso_problem *p, int64_t i, double *rec);

/* Forward pass over samples [i_begin, i_end).  Histograms hold raw weight
 * (one per sample) with bins [0,n), underflow at [n], overflow at [n+1]; the
 * a0,eff histogram covers [0, a0].  Returns 0, or nonzero on invalid input
 * (-1) or a non-finite state (-2). */
int qso_forward(const qso_problem *p, int64_t i_begin, int64_t i_end, int nthreads,
                double *energy_hist, double *angle_hist, double *a0eff_hist,
                double *moments);

/* Node record of the plane-wave reconstruction (index order of the doubles). */
enum {
    QSO_N_A = 0,      /* the node's a0,eff                                   */
    QSO_N_GAMMA0,     /* its initial Lorentz factor                          */
    QSO_N_MU,         /* final mean Lorentz factor                           */
    QSO_N_SIG2,       /* final energy variance                               */
    QSO_N_CHIMAX,     /* max chi at the step starts                          */
    QSO_N_N
};

/* Plane-wave reconstruction of the A0EFF forward pass (Sec. 3.2, 3.3): the
 * moment system runs on n_anodes x n_gnodes nodes (a0,eff uniform over
 * [0, a0]; gamma0 uniform over gamma0 +- 6 sigma_gamma, one node when
 * sigma_gamma = 0); each of the samples [i_begin, i_end) takes the bilinear
 * interpolant of the node states at its (a0,eff, gamma0) and is deposited as
 * in qso_forward.  node_states ([nodes][QSO_N_N]) and node_weights ([nodes],
 * the samples' bilinear weights summed; node = k n_gnodes + m) are optional.
 * Returns 0, -1 on invalid input (also when amp_mode is not A0EFF), -2 on a
 * non-finite node state. */
int qso_factorised(const qso_problem *p, int32_t n_anodes, int32_t n_gnodes, int64_t i_begin,
                   int64_t i_end, int nthreads, double *energy_hist, double *angle_hist,
                   double *a0eff_hist, double *moments, double *node_states,
                   double *node_weights);
/* Photon angular moments (Sec. 5.1) over samples [i_begin, i_end): out[6] =
 * {photon number, number-weighted rms theta_x, theta_y [mrad], emitted
 * energy, energy-weighted rms theta_x, theta_y [mrad]}; per RK4 stage the
 * emission angle is (theta_x + a/mu, theta_y) with a 1/mu cone per plane. */
int qso_photon_angles(const qso_problem *p, int64_t i_begin, int64_t i_end, int nthreads,
                      double *out);

/* Records (QSO_S_N doubles) of samples idx[0 .. n_idx) as the reconstruction
 * deposits them: the interpolated final state and the sample's observables. */
int qso_factorised_samples(const qso_problem *p, int32_t n_anodes, int32_t n_gnodes,
                           int64_t n_idx, const int64_t *idx, int nthreads, double *recs);

/* The method's operation tally: the per-sample path instantiated with a
 * value type that counts its operations, each sample of [i_begin, i_end) run
 * at p->n_steps and at n_steps_b > p->n_steps steps; the difference per
 * sample-step: out[0] adds and subtracts, out[1] multiplies, out[2] divides,
 * out[3] transcendentals (exp, log, sqrt, erfc), out[4] their total; out[5]
 * the operations of one amplitude evaluation (spatial factor at a phase,
 * times a0 and the envelope).  Only per-sample arithmetic counts (the
 * envelope at each phase is shared by all samples). */
int qso_flop_tally(const qso_problem *p, int64_t i_begin, int64_t i_end, int32_t n_steps_b,
                   double *out);

/* Derivatives with respect to the eight parameters, in this order:
 * (a0, w0_um, x_off_um, y_off_um, delay_fs, gamma0, sigma_gamma, div_mrad).
 * qso_sample_grad: out[0] = mu_f, out[1..8] = d mu_f / d p, out[9] = sig2_f,
 * out[10..17] = d sig2_f / d p for sample i.
 * qso_grad: energy histogram hist[n_e + 2] (as qso_forward) and its Jacobian
 * jac[(n_e + 2) * 8] (row = bin) over samples [i_begin, i_end).  Forward-mode
 * derivatives (dual numbers) of exactly the arithmetic qso_forward does. */
int qso_sample_grad(const qso_problem *p, int64_t i, double *out);
int qso_grad(const qso_problem *p, int64_t i_begin, int64_t i_end, int nthreads,
             double *hist, double *jac);
/* The other differentiable outputs over samples [i_begin, i_end): the angle
 * histogram angle_hist[n_th + 2] and its Jacobian jac_angle[(n_th + 2) * 8],
 * the moments moments[QSO_M_N] and their Jacobian jac_moments[QSO_M_N * 8]
 * (rows of the weight, the largest chi and the unused fields are zero: the
 * chi maximum has no derivative almost anywhere).  Dual numbers through the
 * definitions of qso_forward (its values up to summation order). */
int qso_grad_outputs(const qso_problem *p, int64_t i_begin, int64_t i_end, int nthreads,
                     double *angle_hist, double *jac_angle, double *moments, double *jac_moments);

/* Photon emission (Sec. 4): at every RK4 stage the electron's mean energy
 * and the instantaneous amplitude give the LCFA photon spectrum of
 * chi = 2 gamma |a| / a_S, integrated over the phase with the stage weights.
 * hist[n_ph + 2]: expected photon number per bin of photon energy over
 * [ph_lo, ph_hi) in m c^2 units (underflow [n_ph], overflow [n_ph + 1]),
 * summed over samples [i_begin, i_end); energy[0] = emitted photon energy,
 * energy[1] = sum of the electrons' energy loss gamma0_i - mu_f (m c^2). */
int qso_photons(const qso_problem *p, int64_t i_begin, int64_t i_end, int nthreads, int32_t n_ph,
                double ph_lo, double ph_hi, double *hist, double *energy);
/* Number CDF Phi(xi; chi) = Int_0^xi F(xi', chi) dxi' of the LCFA spectrum
 * (F as in qso_photons' notes) and its total Phi(1; chi). */
int qso_photon_cdf(double xi, double chi, double *phi, double *total);

/* Deposit one law into a histogram (exposed for the pins). */
int qso_deposit(double v, double s, int32_t deposit, double kernel_sigma_bins,
                double lo, double hi, int32_t n, double *hist);

#ifdef __cplusplus
}
#endif
#endif
