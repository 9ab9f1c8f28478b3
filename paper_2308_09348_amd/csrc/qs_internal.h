// qs_internal.h -- kernel parameter block and launchers shared by the host
// side of the library (qs_api.hip) and the kernels (qs_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qs {

// ---- radiation-function tables -------------------------------------------
// g, chi g', chi^2 g'', h are stored as one cubic per cell in the local
// coordinate t in [0, 1).  Cell 0 covers chi in [0, 2^kEMin); cell
// 1 + (e - kEMin) * 2^SB + s covers the s-th of 2^SB equal sub-intervals of
// the octave [2^e, 2^(e+1)), e = kEMin .. kEMax.  Each cell holds 16 values:
// four functions x four monomial coefficients (t^0 .. t^3).  The FP32 table is
// function-major ([function][cell][power]), the FP64 table cell-major
// ([cell][function][power]).
constexpr int kEMin = -20;
constexpr int kEMax = 7;
constexpr int kSB32 = 4;  // FP32 table: 16 sub-cells per octave (LDS resident)
constexpr int kSB64 = 6;  // FP64 table: 64 sub-cells per octave (global)
constexpr int kCells32 = 1 + (kEMax - kEMin + 1) * (1 << kSB32);
constexpr int kCells64 = 1 + (kEMax - kEMin + 1) * (1 << kSB64);
constexpr int kCellVals = 16;
// Derivative tables (adjoint): six functions per cell, in the order g,
// chi g', chi^2 g'', h, chi^3 g''', chi h'; FP32 function-major
// ([function][cell][power]), FP64 cell-major ([cell][function][power]).
constexpr int kDerivFuncs = 6;

// ---- device status bits ---------------------------------------------------
constexpr int kFlagNonFinite = 1;
constexpr int kFlagRange = 2;

// ---- per-block moment partial sums ---------------------------------------
enum {
    P_S1E = 0,  // sum (mu_f - gamma0)
    P_S2E,      // sum (mu_f - gamma0)^2 + sig2_f
    P_S1X,      // sum theta_x
    P_S2X,      // sum theta_x^2 + sigma_theta^2
    P_S1Y,
    P_S2Y,
    P_SAEFF,    // sum a0,eff
    P_SRAD,     // sum 1 - mu_f / gamma0_i
    P_SSIGF,    // sum sigma_f
    P_SHN,      // FP64 shadow: samples compared
    P_SHMU,     //   sum (mu32 - mu64) / mu64
    P_SHG,      //   sum (mu32 - mu64)
    P_N
};
// after the sums, the maxima of a moment tile: chi, the shadow's relative
// energy and spread differences
constexpr int kPMaxChi = P_N, kPMaxEmu = P_N + 1, kPMaxEsig = P_N + 2;

constexpr int kPhaseBlock = 256;  // one phase work item = kPhaseBlock samples of one shot
constexpr int kDepBlock = 256;
constexpr int kDepTile = 4096;    // default deposit work item: kDepTile samples of one shot
// Moment partial sums are kept per tile of kMomTile samples whatever the
// deposit work item (a multiple of it), so the moments do not depend on it.
constexpr int kMomTile = 1024;
constexpr int kPartials = P_N + 3;  // moment sums and maxima of a moment tile
// Passes with FP64 steps (forward, tape forward, adjoint, and the
// contraction of their tapes): a work item is a group of up to kChiGroup
// samples of one shot, which the block takes in rounds of kPhaseBlock in
// order of their chi scale, so that wavefronts hold samples of similar chi
// over a wider pool than one phase item; gradient partials are per group.
constexpr int kChiGroup = 2048;
constexpr int kMoments = 21;        // moments a shot returns (QS_M_N)

enum Prec { PREC_F32 = 0, PREC_F32MIX = 1, PREC_F64 = 2 };

// Final state of every sample (structure of arrays in device scratch,
// indexed by the shot's state offset + sample index).
struct SampleState {
    double *mu;    // final mean Lorentz factor
    double *s2;    // final energy variance
    double *S0;    // spatial factor at the collision point (a0,eff / a0)
    double *g0;    // initial Lorentz factor
    double *thx;   // angle in the polarisation plane [rad]
    double *thy;   // angle in the other plane [rad]
    float *cmx;    // largest chi at a step start
};

// Per-shot parameters (device table, read with scalar loads: every lane of a
// block works on the same shot).
struct ShotParams {
    double a0, inv_w0sq, inv_zR, x_off, y_off, z_delay;
    double gamma0, sigma_gamma, sigma_r, sigma_z, div_rad;
    float a0f, inv_w0sqf, inv_zRf, pad0;
    int32_t plane_wave, mid_interp, shot_word;
    int32_t profile;     // kFlatR | kFlatZ: flat-top beam profiles
    int32_t mode, mode_m, mode_n;  // transverse laser mode (QS_MODE_*), its indices
    float mode_inv_normf;          // 1 / the mode's peak in the focal plane
    double mode_inv_norm;
    int64_t n_samples;   // samples of this shot
    int64_t state_off;   // index of its first sample state
    int64_t item0;       // its first phase work item
    int64_t ditem0;      // its first deposit work item
    int64_t mtile0;      // its first moment tile (kMomTile samples each)
    int64_t gitem0;      // its first group (kChiGroup samples) of the passes with FP64 steps
    int64_t hist_off;    // its first histogram word in the accumulators
    // FP64 shadow: samples i with i % shadow_stride == 0 have the FP64 state
    // shadow_off + i / shadow_stride (shadow_stride 0: none); a shot view
    // with draw_stride > 1 integrates samples draw_stride i of the shot
    int64_t shadow_off;
    int64_t shd_off;     // its per-bin FP32 - FP64 law differences [n_e + 2 | n_th + 2]
    int64_t src_off;     // shadow view: the FP32 state of the shot's sample 0
    int32_t shadow_stride, draw_stride;
    // bins
    int32_t n_e, n_th, n_a, pad2;
    double e_lo, e_w, th_lo, th_w;
    // plane-wave reconstruction: the shot's node grid (node = k n_gnode + m)
    int32_t n_anode, n_gnode;
    int64_t node_off;             // index of its first node state
    double g_node_lo, g_node_step;  // gamma0 of node m: g_node_lo + m g_node_step
};

// Beam profile bits of ShotParams::profile: a uniform disk of radius sigma_r
// (else Gaussian of rms sigma_r per axis), a uniform length sigma_z (else
// Gaussian of rms sigma_z).
constexpr int kFlatR = 1;
constexpr int kFlatZ = 2;

// Output pointers of one shot (device table).
struct ShotOut {
    double *energy_hist, *angle_hist, *a0eff_hist, *moments;
    int32_t *status;
    double *samples;
    int64_t rec_stride, rec_n;
    double *node_states;   // plane-wave reconstruction (optional): [nodes][kNodeFields]
    double *node_weights;  // [nodes]
};

// Node record of the plane-wave reconstruction: a0,eff, gamma0, mu_f, sig2_f,
// chi max.
constexpr int kNodeFields = 5;

// ---- photon spectrum (Sec. 4) ---------------------------------------------
// Number CDF of the LCFA photon spectrum, stored as Phi(xi; chi) / (chi z) on
// global rows u_r = kPhU0 + r kPhDu (u = ln chi) and nodes z_j = j kPhDz
// (z = y^(1/3), y = 2 xi / (3 chi (1 - xi))), FP64, [kPhRows][kPhNZ + 1].
constexpr double kPhDu = 0.2;
constexpr double kPhU0 = kEMin * 0.69314718055994530942;
constexpr int kPhRows = 100;  // u up to kPhU0 + 99 kPhDu: chi beyond 2^(kEMax+1)
constexpr int kPhNZ = 1024;
constexpr double kPhYMax = 80.0;
// After the rows (in the same allocation): the photon number per unit of
// the forward FP32 table's cells, a float cubic in the cell coordinate per
// cell ([kCells32][4]), for the FP32 photon angular moments.
constexpr size_t kPhCellOff = (size_t)kPhRows * (kPhNZ + 1);  // in doubles
constexpr size_t kPhTabBytes = sizeof(double) * kPhCellOff + sizeof(float) * 4 * kCells32;
// Emission grid of one shot: at most kPhNU rows (ln chi, global rows
// r_lo .. r_lo + nu - 1) x kPhNV columns (t = sqrt(mu), uniform), weights
// in fixed point.
constexpr int kPhNU = 64, kPhNV = 64, kPhNodes = kPhNU * kPhNV;
constexpr int kPhotTile = 2048;          // one photon work item = kPhotTile samples
// photon energy, electron loss, soft weight; then the Sec. 5.1 angular sums:
// number, number x theta_x^2, number x theta_y^2, energy, energy x theta_x^2,
// energy x theta_y^2
constexpr int kPhotPartials = 9;
constexpr double kPhScale = 16777216.0;  // 2^24: unit of the grid weights

struct ShotPhot {
    int32_t r_lo, nu, nv, n_ph;  // first global row, rows, columns, photon bins
    double t_lo, dt;             // sqrt(mu) at column 0, column width
    float t_lof, inv_dt;         // the same for the FP32 deposit: t_lo, 1 / dt
    double ph_lo, ph_w;          // photon-energy bins [m c^2]
    double *hist;                // [n_ph + 2]
    double *energy;              // [2]: photon energy, electron energy loss
    int32_t *status;             // optional
    double *angles;              // optional [6]: Sec. 5.1 photon angular moments
    int64_t pitem0;              // first photon work item
    int64_t grid_off;            // its grid in the accumulators (kPhNodes words)
    double *errors;              // optional [14]: FP64-shadow report of the shot
};

// Adjoint in/out pointers of one shot (device table).
struct ShotGrad {
    const double *d_energy;  // upstream weights dL/dH over the n_e + 2 energy bins, or null
    double *grad;            // 8 derivatives (order of the qs_grad_param enum)
    int32_t *status;         // optional
    const double *d_angle;   // upstream weights over the n_th + 2 angle bins, or null
    const double *d_moments; // upstream weights over the kMoments moments, or null
    const double *moments;   // the forward pass's moments (with d_moments)
    double *errors;          // optional [17]: FP64-shadow report of the shot
};

constexpr int kGradParams = 8;
constexpr int kTapeFields = 2 + 2 * kGradParams;  // mu, sig2, d mu / dp, d sig2 / dp

// Parameters shared by every shot of a launch.
struct BatchParams {
    // FP64 and FP32 copies of the shared physics constants
    double ell_per_psi, two_over_aS, K, CD, psi_max, h;
    float ellf, two_over_aSf, Kf, CDf, psi0f, hf, chi_fp64, pad0;
    int32_t n_steps, n_shots, deposit;
    int32_t any_mode;  // some shot uses a higher transverse mode
    int32_t dep_tile;   // samples of one deposit work item (a tuning choice)
    int32_t phase_cap;  // resident phase blocks per CU at most (0: all that fit)
    int32_t dep_cap;    // resident deposit blocks per CU at most (0: all that fit)
    int32_t prec;       // the pass's precision (Prec)
    uint32_t key0, key1;
    double ksig_bins, c_theta;
    int64_t n_items, n_ditems, n_mtiles;
    int64_t n_gitems;   // groups of the passes with FP64 steps
    const ShotParams *shots;
    const ShotOut *outs;
    const float *rad32;   // [kCells32 * 16]
    const double *rad64;  // [kCells64 * 16]
    const float *rad32d;  // [kCells32 * 4 * kDerivFuncs]
    const double *rad64d; // [kCells64 * 4 * kDerivFuncs]
    const ShotGrad *gouts;  // adjoint launches only
    const ShotPhot *phot;   // photon launches only
    const double *phtab;    // photon CDF table
    unsigned long long *pgrid;  // per-shot emission grids
    int64_t n_pitems;
    double *tape;           // derivative tape: [2 + 2 kGradParams][tape_n]
    int64_t tape_n;         // samples over the batch (tape field stride)
    SampleState st;
    SampleState nst;        // plane-wave reconstruction: final states of the nodes
    SampleState sst;        // FP64 shadow states of an FP32 pass
    // accumulators (device scratch, cleared before each launch)
    unsigned long long *hist;      // per shot: [n_e + 2 | n_th + 2 | n_a] in 32.32 fixed point
    unsigned long long *shdiff;    // FP64 shadow, per shot: sum over the shadowed samples of
                                   // (FP32-state law - FP64-state law) bin masses, signed, 2^-40
    unsigned int *chimax_bits;     // [n_shots]
    int *flags;                    // [n_shots]
    unsigned int *queue;           // [2]: phase and deposit work counters
    unsigned long long *fp64_steps;  // [n_shots]: wavefront phase steps taken in FP64 by
                                     // the forward pass's FP32 loop (null: not counted)
    double *partials;              // [n_mtiles][kPartials]; adjoint: [n_items][kGradParams]
                                   // ([n_gitems][kGradParams] with FP64 steps)
};

// ---- launchers (qs_kernels.hip) -------------------------------------------
hipError_t build_radiation_tables(float *rad32, double *rad64, float *rad32d, double *rad64d,
                                  double *work, size_t work_doubles, hipStream_t s);
size_t radiation_work_doubles();
hipError_t launch_envelope(double psi_max, double h, int n_steps, int envelope, double omega_tau,
                           float *env32, double *env64, hipStream_t s);
hipError_t launch_zero(unsigned long long *p, size_t n64, hipStream_t s);
hipError_t launch_phase(const BatchParams &p, const float *env32, const double *env64, int prec,
                        int rr, int amp, hipStream_t s);
size_t deposit_lds_bytes(int max_hist_words);
hipError_t launch_deposit(const BatchParams &p, int max_hist_words, hipStream_t s);
hipError_t launch_finalize(const BatchParams &p, hipStream_t s);
hipError_t launch_shadow_diff(const BatchParams &p, int64_t n_items, int max_hist_words,
                              hipStream_t s);
hipError_t launch_radiation_eval(const float *rad32, const double *rad64, int prec, int64_t n,
                                 const double *chi, double *out, int *flags, hipStream_t s);
hipError_t launch_radiation_derivs(const float *rad32d, const double *rad64d, int prec, int64_t n,
                                   const double *chi, double *out, int *flags, hipStream_t s);
hipError_t launch_tangent(const BatchParams &p, const float *env32, const double *env64, int prec,
                          int rr, int amp, bool tape, hipStream_t s);
hipError_t launch_contract(const BatchParams &p, bool obs, int max_ne, hipStream_t s);
size_t photon_work_doubles();
hipError_t build_photon_table(double *phtab, double *work, size_t work_doubles, hipStream_t s);
hipError_t launch_photon(const BatchParams &p, const float *env32, const double *env64, int prec,
                         int rr, int amp, hipStream_t s);
hipError_t launch_photon_finalize(const BatchParams &p, double c_ph, hipStream_t s);
// FP64-shadow report of a photon pass: the batch is the FP64 view pass, whose
// outputs sit `span` doubles after those of the FP32 view pass; span 0 writes
// zeros (no shadow).  One block per shot with errors.
hipError_t launch_photon_shadow(const BatchParams &p, int64_t span, hipStream_t s);
hipError_t launch_photon_cdf(const double *phtab, int64_t n, const double *chi, const double *xi,
                             double *out, hipStream_t s);
hipError_t launch_grad_finalize(const BatchParams &p, hipStream_t s);
// The same for an adjoint pass (gradients `span` doubles apart).
hipError_t launch_grad_shadow(const BatchParams &p, int64_t span, hipStream_t s);
// plane-wave reconstruction (qs_factor.hip): the node pass is the phase
// kernel in node mode on the node view of the shot table; the interpolation
// pass writes sample states for the deposit and finalize kernels
hipError_t launch_phase_nodes(const BatchParams &p, const float *env32, const double *env64,
                              int prec, int rr, hipStream_t s);
hipError_t launch_interp(const BatchParams &p, int weight_words, hipStream_t s);
hipError_t launch_node_outputs(const BatchParams &p, hipStream_t s);

}  // namespace qs
