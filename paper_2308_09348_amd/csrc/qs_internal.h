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
    P_N
};

constexpr int kPhaseBlock = 256;
constexpr int kDepBlock = 256;

enum Prec { PREC_F32 = 0, PREC_F32MIX = 1, PREC_F64 = 2 };

// Final state of every sample (structure of arrays in device scratch).
struct SampleState {
    double *mu;    // final mean Lorentz factor
    double *s2;    // final energy variance
    double *S0;    // spatial factor at the collision point (a0,eff / a0)
    double *g0;    // initial Lorentz factor
    double *thx;   // angle in the polarisation plane [rad]
    double *thy;   // angle in the other plane [rad]
    float *cmx;    // largest chi at a step start
};

// Phase kernel: sample -> geometry -> RK4 loop -> SampleState.
struct PhaseParams {
    // FP64 copies (per-sample set-up and FP64 steps)
    double a0, inv_w0sq, inv_zR, x_off, y_off, z_delay, ell_per_psi;
    double gamma0, sigma_gamma, sigma_r, sigma_z, div_rad;
    double two_over_aS, K, CD, psi_max, h;
    // FP32 copies (FP32 steps)
    float a0f, inv_w0sqf, inv_zRf, ellf, two_over_aSf, Kf, CDf, psi0f, hf, chi_fp64;
    int32_t n_steps, shot, plane_wave;
    int32_t mid_interp;   // stage-2/3 spatial factor by quadratic interpolation
    uint32_t key0, key1;
    int64_t n_samples;
    const float *env32;   // [2 n_steps + 1] envelope x carrier at psi_k = -psi_max + k h/2
    const double *env64;
    const float *rad32;   // [kCells32 * 16]
    const double *rad64;  // [kCells64 * 16]
    SampleState st;
    int *flags;
};

// Deposit kernel: SampleState -> observables -> histograms and moments.
struct DepParams {
    int64_t n_samples;
    double a0, gamma0, c_theta;
    int32_t deposit, n_e, n_th, n_a;
    double ksig_bins, e_lo, e_w, th_lo, th_w;
    SampleState st;
    unsigned long long *hist;  // [n_e + 2 | n_th + 2 | n_a] fixed point 2^-32
    double *partials;          // [gridDim.x * P_N]
    unsigned int *chimax_bits;
    int *flags;
    double *rec;               // optional per-sample records
    int64_t rec_stride, rec_n;
};

struct FinParams {
    int64_t n_samples;
    int nblocks;
    int n_e, n_th, n_a;
    double gamma0;
    const unsigned long long *hist;
    const double *partials;
    const unsigned int *chimax_bits;
    const int *flags;
    double *energy_hist, *angle_hist, *a0eff_hist, *moments;
    int32_t *status;
};

// ---- launchers (qs_kernels.hip) -------------------------------------------
hipError_t build_radiation_tables(float *rad32, double *rad64, double *work, size_t work_doubles,
                                  hipStream_t s);
size_t radiation_work_doubles();
hipError_t launch_envelope(double psi_max, double h, int n_steps, int envelope, double omega_tau,
                           float *env32, double *env64, hipStream_t s);
hipError_t launch_zero(unsigned long long *p, size_t n64, hipStream_t s);
hipError_t launch_phase(const PhaseParams &p, int prec, int rr, int amp, hipStream_t s);
size_t deposit_lds_bytes(int n_e, int n_th, int n_a);
hipError_t deposit_grid(size_t lds_bytes, int device, int64_t n_samples, int *grid);
hipError_t launch_deposit(const DepParams &p, int grid, hipStream_t s);
hipError_t launch_finalize(const FinParams &p, hipStream_t s);
hipError_t launch_radiation_eval(const float *rad32, const double *rad64, int prec, int64_t n,
                                 const double *chi, double *out, int *flags, hipStream_t s);

}  // namespace qs
