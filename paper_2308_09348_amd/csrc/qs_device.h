// qs_device.h -- device helpers shared by the kernels of the library: the
// sample generator, the radiation-function table lookups, the moment system,
// the spatial factor and ballistic path, RK4 steps, compensated sums, work
// items and wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <climits>
#include <math.h>

#include <type_traits>

#include "qs_internal.h"

namespace qs {

// ===========================================================================
// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller normals
// ===========================================================================
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// The beam coordinates of sample i of a shot (a volume element of Sec. 2):
// counter (i, shot, k, 0) for k = 0, 1 gives eight words, the first six make
// 24-bit uniforms u = ((r >> 8) + 1/2) 2^-24, and Box-Muller on the pairs
// (u0, u1), (u2, u3), (u4, u5) gives six standard normals n.  Transverse
// position: x_off + sigma_r (n0, n1), or for a flat-top beam the uniform disk
// x_off + sigma_r sqrt(u0) (cos 2 pi u1, sin 2 pi u1); longitudinal offset
// sigma_z n2, or sigma_z (u2 - 1/2) for a flat-top beam of length sigma_z;
// gamma0 + sigma_gamma n3; angles div (n4, n5).
struct SampleCoords {
    double x, y, z, g0, thx, thy;
    double n[6];
};

// Sample i of a shot table entry: sample i draw_stride of the shot (a view
// with draw_stride > 1 holds every draw_stride-th sample).
__device__ __forceinline__ void sample_coords(const ShotParams &sp, uint32_t k0, uint32_t k1,
                                              int64_t i, SampleCoords &sc) {
    uint32_t r[8];
    const uint32_t ctr0 = (uint32_t)(i * (int64_t)sp.draw_stride);
#pragma unroll
    for (uint32_t k = 0; k < 2; ++k) {
        uint32_t c[4] = {ctr0, (uint32_t)sp.shot_word, k, 0u};
        philox4x32_10(c, k0, k1);
        r[4 * k + 0] = c[0];
        r[4 * k + 1] = c[1];
        r[4 * k + 2] = c[2];
        r[4 * k + 3] = c[3];
    }
    double u[6], cs0 = 0.0, sn0 = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) u[m] = ((double)(r[m] >> 8) + 0.5) * 0x1p-24;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double R = sqrt(-2.0 * log(u[2 * m]));
        double s, c;
        sincospi(2.0 * u[2 * m + 1], &s, &c);
        sc.n[2 * m] = R * c;
        sc.n[2 * m + 1] = R * s;
        if (m == 0) {
            cs0 = c;
            sn0 = s;
        }
    }
    // selects rather than branches: the hot loops that follow keep their
    // register budget
    const bool flat_r = (sp.profile & kFlatR) != 0;
    const double rad = sp.sigma_r * sqrt(u[0]);
    sc.x = fma(flat_r ? rad : sp.sigma_r, flat_r ? cs0 : sc.n[0], sp.x_off);
    sc.y = fma(flat_r ? rad : sp.sigma_r, flat_r ? sn0 : sc.n[1], sp.y_off);
    sc.z = sp.sigma_z * ((sp.profile & kFlatZ) ? u[2] - 0.5 : sc.n[2]);
    sc.g0 = fma(sp.sigma_gamma, sc.n[3], sp.gamma0);
    sc.thx = sp.div_rad * sc.n[4];
    sc.thy = sp.div_rad * sc.n[5];
}

// ===========================================================================
// Radiation functions: g, chi g', chi^2 g'', h from per-cell cubics
// ===========================================================================
__device__ __forceinline__ void rad_eval32(const float *__restrict__ tab, float chi, float &g,
                                           float &G1, float &G2, float &hq) {
    // exponent and the top kSB32 mantissa bits give the cell directly
    const uint32_t b = __float_as_uint(chi);
    int c = (int)(b >> (23 - kSB32)) - ((127 + kEMin) << kSB32) + 1;
    float t = __uint_as_float(((b & ((1u << (23 - kSB32)) - 1)) << kSB32) | 0x3f800000u) - 1.0f;
    if (c < 1) {  // chi < 2^kEMin: the first cell, linear in chi
        c = 0;
        t = chi * 0x1p20f;
    }
    c = min(c, kCells32 - 1);  // chi >= 2^(kEMax+1) is reported by the caller
    // function-major layout: four arrays of 16-byte cubics, so that the cells
    // read by one wavefront start on eight different 4-bank groups of LDS
    const float4 *T = reinterpret_cast<const float4 *>(tab);
    const float4 q0 = T[c], q1 = T[kCells32 + c], q2 = T[2 * kCells32 + c],
                 q3 = T[3 * kCells32 + c];
    g = fmaf(t, fmaf(t, fmaf(t, q0.w, q0.z), q0.y), q0.x);
    G1 = fmaf(t, fmaf(t, fmaf(t, q1.w, q1.z), q1.y), q1.x);
    G2 = fmaf(t, fmaf(t, fmaf(t, q2.w, q2.z), q2.y), q2.x);
    hq = fmaf(t, fmaf(t, fmaf(t, q3.w, q3.z), q3.y), q3.x);
}

// One FP32 table cell held in registers.  Any chi near the cell maps to
// its local coordinate by t = chi * tw + ts; the RK4 stages that share a
// phase with the previous lookup (stage 3 after stage 2, the next step's
// stage 1 after stage 4) evaluate the same cubics a hair outside [0, 1]
// instead of reading LDS again.
struct RadCell32 {
    float4 q0, q1, q2, q3;
    float tw, ts;
};

// The index comes from chi clamped to the octave cells [2^kEMin, 2^(kEMax+1)).
// Below 2^kEMin the first octave cell's cubic is extrapolated down to chi = 0
// (t >= -2^kSB32): there g, chi g', chi^2 g'' and h are linear in chi to
// 1e-12, and so is the cell's cubic.  Above the table the result is not used
// (the caller reports the range error).
// With ncell, *nq also receives that cell's entry of ncell (a per-cell cubic
// of another function on the same cells).
__device__ __forceinline__ void rad_lookup32(const float *__restrict__ tab, float chi,
                                             RadCell32 &cell,
                                             const float4 *__restrict__ ncell = nullptr,
                                             float4 *nq = nullptr) {
    const float xc = fminf(fmaxf(chi, 0x1p-20f), 0x1.fffffep7f);
    const uint32_t b = __float_as_uint(xc);
    // cell 1 + (b - bits(2^kEMin)) >> (23 - SB): non-negative by the clamp
    const uint32_t c = ((b - ((uint32_t)(127 + kEMin) << 23)) >> (23 - kSB32)) + 1u;
    // cell start 2^e (1 + sub/2^SB) and inverse width 2^(SB - e)
    const float tw = __uint_as_float((uint32_t)(254 + kSB32 - (int)(b >> 23)) << 23);
    const float ts = -__uint_as_float(b & ~((1u << (23 - kSB32)) - 1)) * tw;
    const float4 *T = reinterpret_cast<const float4 *>(tab);
    cell.q0 = T[c];
    cell.q1 = T[kCells32 + c];
    cell.q2 = T[2 * kCells32 + c];
    cell.q3 = T[3 * kCells32 + c];
    cell.tw = tw;
    cell.ts = ts;
    if (ncell) *nq = ncell[c];
}

__device__ __forceinline__ void rad_cell_eval(const RadCell32 &cell, float chi, float &g,
                                              float &G1, float &G2, float &hq) {
    // returns the four table functions of the cell (see rhs_q32)
    const float t = fmaf(chi, cell.tw, cell.ts);
    g = fmaf(t, fmaf(t, fmaf(t, cell.q0.w, cell.q0.z), cell.q0.y), cell.q0.x);
    G1 = fmaf(t, fmaf(t, fmaf(t, cell.q1.w, cell.q1.z), cell.q1.y), cell.q1.x);
    G2 = fmaf(t, fmaf(t, fmaf(t, cell.q2.w, cell.q2.z), cell.q2.y), cell.q2.x);
    hq = fmaf(t, fmaf(t, fmaf(t, cell.q3.w, cell.q3.z), cell.q3.y), cell.q3.x);
}

// FP64 cell of chi and the coordinate t in the cell (cell 0 is linear in chi
// below 2^kEMin; chi beyond the table is clamped to the last cell and
// reported by the caller).
__device__ __forceinline__ int rad_index64(double chi, double &t) {
    const uint64_t b = (uint64_t)__double_as_longlong(chi);
    int64_t c = (int64_t)(b >> (52 - kSB64)) - ((int64_t)(1023 + kEMin) << kSB64) + 1;
    t = __longlong_as_double((long long)(((b & ((1ull << (52 - kSB64)) - 1)) << kSB64) |
                                         0x3ff0000000000000ull)) - 1.0;
    if (c < 1) {
        c = 0;
        t = chi * 0x1p20;
    }
    return (int)(c < kCells64 - 1 ? c : kCells64 - 1);
}

__device__ __forceinline__ void rad_cell_eval64(const double *q, double t, double &g, double &G1,
                                                double &G2, double &hq) {
    g = fma(t, fma(t, fma(t, q[3], q[2]), q[1]), q[0]);
    G1 = fma(t, fma(t, fma(t, q[7], q[6]), q[5]), q[4]);
    G2 = fma(t, fma(t, fma(t, q[11], q[10]), q[9]), q[8]);
    hq = fma(t, fma(t, fma(t, q[15], q[14]), q[13]), q[12]);
}

__device__ __forceinline__ void rad_eval64(const double *__restrict__ tab, double chi, double &g,
                                           double &G1, double &G2, double &hq) {
    double t;
    const int c = rad_index64(chi, t);
    rad_cell_eval64(tab + (size_t)c * kCellVals, t, g, G1, G2, hq);
}

// The FP64 cells of all 64 lanes of a wavefront, fetched together.  A cell
// is 128 bytes, one cache line; read lane by lane, every load instruction
// would touch 64 lines.  Here four lanes read 64 bytes of one cell, so every
// load instruction touches 16 lines and uses each fully for its half, and
// the cells reach their lanes through a per-wavefront LDS staging area: one
// row a lane holding half a cell (first the lower, then the upper 64 bytes),
// rows padded to 80 bytes so that the row reads of eight lanes fall on
// distinct banks.  Every lane of the wavefront must be active; the values
// are those rad_eval64 reads.
constexpr int kStageStride = 5;                  // 16-byte chunks a row
constexpr int kStageChunks = 64 * kStageStride;  // per wavefront

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same for cells of 64 PASSES bytes (8 PASSES doubles, row after row):
// PASSES rounds of the staged read above, one 64-byte part of every cell each.
template <int PASSES>
__device__ __forceinline__ void coop_rows64(const double *__restrict__ tab, int c,
                                            double2 *__restrict__ stage, double *q) {
    const int lane = (int)(threadIdx.x & 63u);
    const int k = lane & 3;
    const double2 *cell[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int cr = __shfl(c, 16 * r + (lane >> 2), 64);
        cell[r] = reinterpret_cast<const double2 *>(tab + (size_t)cr * (8 * PASSES)) + k;
    }
    const double2 *row = stage + lane * kStageStride;
#pragma unroll
    for (int part = 0; part < PASSES; ++part) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            stage[(16 * r + (lane >> 2)) * kStageStride + k] = cell[r][4 * part];
        wave_sync_lds();
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const double2 v = row[m];
            q[8 * part + 2 * m] = v.x;
            q[8 * part + 2 * m + 1] = v.y;
        }
        wave_sync_lds();  // the next part overwrites the rows
    }
}

__device__ __forceinline__ void coop_cell64(const double *__restrict__ tab, int c,
                                            double2 *__restrict__ stage, double q[16]) {
    static_assert(kCellVals == 16, "a forward-table cell is two 64-byte parts");
    coop_rows64<2>(tab, c, stage, q);
}

// Chi at coordinate t in [0, 1) of a table cell (SB: sub-cells per octave;
// cell 0 is linear in chi below 2^kEMin), the four Chebyshev nodes of a cell
// and the monomial coefficients l[0..3] of the Lagrange polynomial of node m
// (a cubic through the node values v_m is sum_m v_m l_m(t)).
__device__ __forceinline__ double cell_chi(int cell, double t, int sb) {
    if (cell == 0) return t * 0x1p-20;
    const int c = cell - 1;
    const int e = kEMin + (c >> sb);
    const int sub = c & ((1 << sb) - 1);
    return ldexp(1.0 + ((double)sub + t) / (double)(1 << sb), e);
}

__device__ __forceinline__ double cheb_node(int m) {
    return 0.5 * (1.0 - cospi((2.0 * m + 1.0) / 8.0));
}

__device__ __forceinline__ void cheb_basis(int m, double l[4]) {
    double r[3];
    int k = 0;
    double den = 1.0;
    for (int n = 0; n < 4; ++n)
        if (n != m) {
            r[k++] = cheb_node(n);
            den *= cheb_node(m) - cheb_node(n);
        }
    // (t - r0)(t - r1)(t - r2) / den
    l[3] = 1.0 / den;
    l[2] = -(r[0] + r[1] + r[2]) / den;
    l[1] = (r[0] * r[1] + r[0] * r[2] + r[1] * r[2]) / den;
    l[0] = -(r[0] * r[1] * r[2]) / den;
}

template <class T>
struct RadTab;
template <>
struct RadTab<float> {
    const float *p;
    __device__ __forceinline__ void eval(float chi, float &g, float &G1, float &G2, float &h) const {
        rad_eval32(p, chi, g, G1, G2, h);
    }
};
template <>
struct RadTab<double> {
    const double *p;
    __device__ __forceinline__ void eval(double chi, double &g, double &G1, double &G2,
                                         double &h) const {
        rad_eval64(p, chi, g, G1, G2, h);
    }
};
// FP64 table read cooperatively by the whole wavefront (see coop_cell64).
// The last cells read stay in registers: a stage whose lanes all fall in the
// cells they already hold (the third RK4 stage mostly, and the first stage
// after the fourth at the same amplitude) reads nothing.
struct RadTabWave {
    const double *p;
    double2 *stage;
    mutable double q[16];
    mutable int c = -1;
    __device__ __forceinline__ RadTabWave(const double *tab, double2 *st) : p(tab), stage(st) {}
    __device__ __forceinline__ void eval(double chi, double &g, double &G1, double &G2,
                                         double &h) const {
        double t;
        const int cn = rad_index64(chi, t);
        if (__any(cn != c)) {
            coop_cell64(p, cn, stage, q);
            c = cn;
        }
        rad_cell_eval64(q, t, g, G1, G2, h);
    }
};

// ===========================================================================
// The moment system (second-order closure of the drift-diffusion process
// whose drift is eq. dpdtRR in phase units):
//   dmu/dpsi   = A + A'' sig2 / 2,   dsig2/dpsi = 2 A' sig2 + D,
//   A = -K a^2 mu^2 g,  A' = -K a^2 mu (2g + G1),  A'' = -K a^2 (2g + 4G1 + G2),
//   D = C_D |a|^3 mu^4 h,  chi = 2 mu |a| / a_S.
// ===========================================================================
template <class T>
struct Phys {
    T K, CD, two_over_aS;
};

template <class T, bool QUANTUM, class Tab = RadTab<T>>
__device__ __forceinline__ void rhs(T mu, T s2, T a, const Phys<T> &ph, const Tab &tab,
                                    T &dmu, T &ds2, T &chi_hi) {
    const T a2 = a * a;
    const T Ka2 = ph.K * a2;
    if (!QUANTUM) {
        dmu = -Ka2 * mu * mu;
        ds2 = T(0);
        return;
    }
    const T aa = fabs(a);
    const T chi = ph.two_over_aS * mu * aa;
    chi_hi = fmax(chi_hi, chi);
    T g, G1, G2, hq;
    tab.eval(chi, g, G1, G2, hq);
    const T two_g = T(2) * g;
    const T A = -Ka2 * mu * mu * g;
    const T A1 = -Ka2 * mu * (two_g + G1);
    const T A2 = -Ka2 * (two_g + T(4) * G1 + G2);
    const T mu2 = mu * mu;
    const T D = ph.CD * a2 * aa * mu2 * mu2 * hq;
    dmu = fma(T(0.5) * A2, s2, A);
    ds2 = fma(T(2) * A1, s2, D);
}

// Spatial factor a/a0 of eq. a0eff at (x, y, z) [um].  The FP32 version uses
// the hardware reciprocal, reciprocal square root and base-2 exponential
// (about one ulp each; the exponent's argument rounding adds |r2/q| ulps,
// which matters only where the factor itself is small).
__device__ __forceinline__ float spatial(float x, float y, float z, float inv_w0sq, float inv_zR) {
    const float zz = z * inv_zR;
    const float q = fmaf(zz, zz, 1.0f);
    const float rq = __builtin_amdgcn_rsqf(q);  // 1/sqrt(q); 1/q = rq^2
    const float r2 = fmaf(x, x, y * y) * inv_w0sq;
    return __builtin_amdgcn_exp2f(-1.4426950408889634f * r2 * (rq * rq)) * rq;
}
__device__ __forceinline__ double spatial(double x, double y, double z, double inv_w0sq,
                                          double inv_zR) {
    const double zz = z * inv_zR;
    const double q = fma(zz, zz, 1.0);
    const double iq = 1.0 / q;
    const double r2 = fma(x, x, y * y) * inv_w0sq;
    return exp(-r2 * iq) * sqrt(iq);
}

// Higher transverse modes (amplitude only, peak 1 in the focal plane): with
// u = x/W, v = y/W, W = W0 sqrt(q), q = 1 + z^2/zR^2,
//   Hermite-Gauss m, n:  |H_m(sqrt2 u) H_n(sqrt2 v)| exp(-(u^2 + v^2)) / sqrt(q),
//   Laguerre-Gauss p, l: t^(|l|/2) |L_p^|l|(t)| exp(-t/2) / sqrt(q), t = 2(u^2 + v^2),
// divided by the mode's focal-plane peak; H and L by their three-term
// recurrences (H_(k+1) = 2s H_k - 2k H_(k-1); (k+1) L_(k+1) =
// (2k + 1 + l - t) L_k - (k + l) L_(k-1)).
template <class T>
__device__ __forceinline__ T hermite(int m, T s) {
    T h0 = T(1), h1 = T(2) * s;
    if (m == 0) return h0;
    for (int k = 1; k < m; ++k) {
        const T h2 = fma(T(2) * s, h1, T(-2 * k) * h0);
        h0 = h1;
        h1 = h2;
    }
    return h1;
}
template <class T>
__device__ __forceinline__ T spatial_mode(T x, T y, T z, T inv_w0sq, T inv_zR, int mode, int mm,
                                          int mn, T inv_norm) {
    const T zz = z * inv_zR;
    const T q = fma(zz, zz, T(1));
    const T iq = T(1) / q;
    const T u2 = x * x * inv_w0sq * iq, v2 = y * y * inv_w0sq * iq;
    const T g = exp(-(u2 + v2)) * sqrt(iq) * inv_norm;
    if (mode == 1) {  // Hermite-Gauss
        const T r2 = sqrt(T(2) * inv_w0sq * iq);
        return fabs(hermite<T>(mm, x * r2) * hermite<T>(mn, y * r2)) * g;
    }
    const int l = abs(mn);  // Laguerre-Gauss, p = mm
    const T t = T(2) * (u2 + v2);
    T L0 = T(1), L1 = T(1 + l) - t, Lp = L0;
    if (mm >= 1) Lp = L1;
    for (int k = 1; k < mm; ++k) {
        const T L2 = (fma(T(2 * k + 1 + l) - t, L1, T(-(k + l)) * L0)) / T(k + 1);
        L0 = L1;
        L1 = L2;
        Lp = L2;
    }
    T tp = T(1);
    for (int k = 0; k < l / 2; ++k) tp *= t;
    if (l & 1) tp *= sqrt(t);
    return tp * fabs(Lp) * g;
}

// Geometry of one sample along its ballistic path: at phase psi it has
// travelled l = psi lambda / (4 pi) past its collision point.  mode != 0
// selects a higher transverse mode (QS_MODE_HG 1, QS_MODE_LG 2).
// MODES = false compiles the Gaussian focus alone (the hot loop's register
// budget does not carry the mode recurrences).
template <class T, bool MODES = true>
struct Path {
    T xc, yc, thx, thy, zstar, inv_w0sq, inv_zR;
    int mode, mm, mn;
    T inv_norm;
    __device__ __forceinline__ T S(T ell) const {
        if constexpr (MODES) {
            if (mode != 0)
                return spatial_mode<T>(fma(thx, ell, xc), fma(thy, ell, yc), zstar - ell,
                                       inv_w0sq, inv_zR, mode, mm, mn, inv_norm);
        }
        return spatial(fma(thx, ell, xc), fma(thy, ell, yc), zstar - ell, inv_w0sq, inv_zR);
    }
};

// Sample i of a shot (Sec. 2 volume element): its initial Lorentz factor and
// angles, its ballistic path and the spatial factor at its collision point.
template <bool MODES = true>
__device__ __forceinline__ void draw_sample(const ShotParams &sp, uint32_t key0, uint32_t key1,
                                            int64_t i, double &g0, double &thx, double &thy,
                                            Path<double, MODES> &pd, double &S0) {
    SampleCoords sc;
    sample_coords(sp, key0, key1, i, sc);
    const double x = sc.x, y = sc.y, z = sc.z;
    g0 = sc.g0;
    thx = sc.thx;
    thy = sc.thy;
    pd.xc = fma(thx, 0.5 * z, x);
    pd.yc = fma(thy, 0.5 * z, y);
    pd.thx = thx;
    pd.thy = thy;
    pd.zstar = fma(0.5, z, sp.z_delay);
    pd.inv_w0sq = sp.inv_w0sq;
    pd.inv_zR = sp.inv_zR;
    pd.mode = sp.mode;
    pd.mm = sp.mode_m;
    pd.mn = sp.mode_n;
    pd.inv_norm = sp.mode_inv_norm;
    S0 = sp.plane_wave ? 1.0 : pd.S(0.0);
}

// Order in which the lanes of a block take the G consecutive samples of a
// group (from `base`) in passes with FP64 steps where chi exceeds a
// threshold.  A wavefront steps in FP64 when any of its lanes needs it, so its
// lanes should hold samples of similar chi: they take the samples in
// increasing order of S0 gamma0, the chi scale of a sample at its collision
// point.  The order is stable (ties by index), so every launch of a group
// forms the same wavefronts.  s_idx[r] receives the group offset of rank r;
// offsets at or past `end` (no sample) rank last.  B threads take part.
// An FP32 estimate of that key, for passes whose results do not depend on the
// order (no FP64 steps): the first counter block's normals by Box-Muller in
// FP32, the collision point without the divergence's shift (below 1e-2 um).
__device__ __forceinline__ float chi_key32(const ShotParams &sp, uint32_t k0, uint32_t k1,
                                           int64_t i) {
    uint32_t c[4] = {(uint32_t)(i * (int64_t)sp.draw_stride), (uint32_t)sp.shot_word, 0u, 0u};
    philox4x32_10(c, k0, k1);
    float u[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) u[m] = ((float)(c[m] >> 8) + 0.5f) * 0x1p-24f;
    const float R0 = __builtin_sqrtf(-2.0f * __logf(u[0])), R1 = __builtin_sqrtf(-2.0f * __logf(u[2]));
    float s0, c0, s1, c1;
    __sincosf(6.28318530717958648f * u[1], &s0, &c0);
    __sincosf(6.28318530717958648f * u[3], &s1, &c1);
    const bool flat_r = (sp.profile & kFlatR) != 0;
    const float sr = (float)sp.sigma_r, rad = flat_r ? sr * __builtin_sqrtf(u[0]) : sr * R0;
    const float x = fmaf(rad, c0, (float)sp.x_off), y = fmaf(rad, s0, (float)sp.y_off);
    const float z = (float)sp.sigma_z * ((sp.profile & kFlatZ) ? u[2] - 0.5f : R1 * c1);
    const float g0 = fmaf((float)sp.sigma_gamma, R1 * s1, (float)sp.gamma0);
    if (sp.plane_wave) return g0;
    return g0 * spatial(x, y, fmaf(0.5f, z, (float)sp.z_delay), sp.inv_w0sqf, sp.inv_zRf);
}

// FAST: the FP32 key (passes without FP64 steps, where any order gives the same
// results); else the FP64 one.
template <int G, int B, bool FAST = false>
__device__ __forceinline__ void chi_order(const ShotParams &sp, uint32_t key0, uint32_t key1,
                                          int64_t base, int64_t end, float *s_key,
                                          unsigned short *s_idx) {
    static_assert(G % B == 0 && G <= 65536, "group of whole rounds, 16-bit offsets");
    __syncthreads();  // the previous group's order is no longer read
    for (int q = threadIdx.x; q < G; q += B) {
        float key = __builtin_inff();
        const int64_t i = base + q;
        if (i < end) {
            if constexpr (FAST) {
                key = chi_key32(sp, key0, key1, i);
            } else {
                // (the Gaussian focus's factor also orders samples of a higher
                // mode: any order gives the same results up to the FP64-step
                // choice)
                double g0, thx, thy, S0;
                Path<double, false> pd{};
                draw_sample<false>(sp, key0, key1, i, g0, thx, thy, pd, S0);
                key = (float)(S0 * g0);
            }
        }
        s_key[q] = key;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < G; q += B) {
        const float k = s_key[q];
        int rank = 0;
        for (int j = 0; j < G; ++j) {
            const float kj = s_key[j];
            rank += (kj < k || (kj == k && j < q)) ? 1 : 0;
        }
        s_idx[rank] = (unsigned short)q;
    }
    __syncthreads();
}

// One RK4 step of (mu, sig2) from psi_j with amplitudes a1 = a(psi_j),
// ah = a(psi_j + h/2), a4 = a(psi_j + h); returns the increments.
template <class T, bool QUANTUM, class Tab = RadTab<T>>
__device__ __forceinline__ void rk4_increment(T mu, T s2, T a1, T ah, T a4, T h,
                                              const Phys<T> &ph, const Tab &tab, T &dmu,
                                              T &ds2, T &chi_hi) {
    const T hh = T(0.5) * h;
    T k1m, k1s, k2m, k2s, k3m, k3s, k4m, k4s;
    rhs<T, QUANTUM, Tab>(mu, s2, a1, ph, tab, k1m, k1s, chi_hi);
    rhs<T, QUANTUM, Tab>(fma(hh, k1m, mu), fma(hh, k1s, s2), ah, ph, tab, k2m, k2s, chi_hi);
    rhs<T, QUANTUM, Tab>(fma(hh, k2m, mu), fma(hh, k2s, s2), ah, ph, tab, k3m, k3s, chi_hi);
    rhs<T, QUANTUM, Tab>(fma(h, k3m, mu), fma(h, k3s, s2), a4, ph, tab, k4m, k4s, chi_hi);
    const T h6 = h * T(1.0 / 6.0);
    dmu = h6 * (k1m + T(2) * (k2m + k3m) + k4m);
    ds2 = h6 * (k1s + T(2) * (k2s + k3s) + k4s);
}

// Moment right-hand side (quantum model) from the FP32 table's combined
// functions at chi = two_over_aS mu |a|:  T1 = g,  T2 = 2g + chi g',
// T3 = g + 2 chi g' + chi^2 g''/2,  T4 = h, so that
//   dmu/dpsi   = -K a^2 (mu^2 T1 + sig2 T3),
//   dsig2/dpsi = -2 K a^2 mu sig2 T2 + C_D a^2 |a| mu^4 T4.
// The factors that depend on the amplitude only are formed once per phase
// point (stages 2 and 3 share one, stage 4 hands its to the next stage 1).
struct AmpQ {
    float nu;   // -K a^2
    float nu2;  // -2 K a^2
    float cd;   // C_D a^2 |a|
    float cpm;  // chi per unit mu: 2 |a| / a_S
    __device__ __forceinline__ AmpQ() {}
    __device__ __forceinline__ AmpQ(float a, const Phys<float> &ph) {
        const float aa = fabsf(a), a2 = a * a;
        nu = -ph.K * a2;
        nu2 = 2.0f * nu;
        cd = ph.CD * aa * a2;
        cpm = ph.two_over_aS * aa;
    }
};

__device__ __forceinline__ void rhs_q32(float mu, float s2, const AmpQ &A, float T1, float T2,
                                        float T3, float T4, float &dmu, float &ds2) {
    const float mu2 = mu * mu;
    dmu = A.nu * fmaf(mu2, T1, s2 * T3);
    ds2 = fmaf(A.nu2 * mu * s2, T2, A.cd * (mu2 * mu2) * T4);
}

// One FP32 RK4 step of the quantum moment system with two table reads:
// stage 2 and stage 4 read LDS, stage 3 reuses stage 2's cell, and stage 4's
// cell is handed to the next step's stage 1 (with its amplitude factors).
__device__ __forceinline__ void rk4_q32(float mu, float s2, AmpQ &A1, float ah, float a4, float h,
                                        const Phys<float> &ph, const float *__restrict__ tab,
                                        RadCell32 &carry, float &dmu, float &ds2,
                                        float &chi_hi) {
    const float hh = 0.5f * h;
    float g, G1, G2, hq;
    // stage 1 (cell and amplitude factors carried from the previous stage 4)
    const float c1 = A1.cpm * mu;
    rad_cell_eval(carry, c1, g, G1, G2, hq);
    float k1m, k1s;
    rhs_q32(mu, s2, A1, g, G1, G2, hq, k1m, k1s);
    // stage 2 (table read)
    const AmpQ Ah(ah, ph);
    const float m2 = fmaf(hh, k1m, mu), s22 = fmaf(hh, k1s, s2);
    const float c2 = Ah.cpm * m2;
    RadCell32 mid;
    rad_lookup32(tab, c2, mid);
    rad_cell_eval(mid, c2, g, G1, G2, hq);
    float k2m, k2s;
    rhs_q32(m2, s22, Ah, g, G1, G2, hq, k2m, k2s);
    // stage 3 (same phase as stage 2: reuse its cell)
    const float m3 = fmaf(hh, k2m, mu), s23 = fmaf(hh, k2s, s2);
    const float c3 = Ah.cpm * m3;
    rad_cell_eval(mid, c3, g, G1, G2, hq);
    float k3m, k3s;
    rhs_q32(m3, s23, Ah, g, G1, G2, hq, k3m, k3s);
    // stage 4 (table read; its cell serves the next step's stage 1)
    A1 = AmpQ(a4, ph);
    const float m4 = fmaf(h, k3m, mu), s24 = fmaf(h, k3s, s2);
    const float c4 = A1.cpm * m4;
    rad_lookup32(tab, c4, carry);
    rad_cell_eval(carry, c4, g, G1, G2, hq);
    float k4m, k4s;
    rhs_q32(m4, s24, A1, g, G1, G2, hq, k4m, k4s);
    // the range check takes the chi of the table reads: stages 1 and 3
    // evaluate the cells of stages 4 and 2 at a chi a hair away (the state
    // moved by less than one step's increment)
    chi_hi = fmaxf(chi_hi, fmaxf(c2, c4));
    const float h6 = h * (1.0f / 6.0f);
    dmu = h6 * (k1m + 2.0f * (k2m + k3m) + k4m);
    ds2 = h6 * (k1s + 2.0f * (k2s + k3s) + k4s);
}

// Compensated accumulation: (hi, lo) += d, renormalised (Fast2Sum, |hi| >= |d|).
__device__ __forceinline__ void comp_add(float &hi, float &lo, float d) {
    const float dd = d + lo;
    const float s = hi + dd;
    lo = dd - (s - hi);
    hi = s;
}

// ===========================================================================
// Work items.  A launch covers n_shots shots; phase items are tiles of
// kPhaseBlock consecutive samples of one shot (one sample per lane), deposit
// items tiles of dep_tile samples (a multiple of kMomTile, the tile of the
// moment partial sums).  Blocks take items from a counter; an item's result
// does not depend on which block runs it, nor on dep_tile, so the output is
// deterministic, and a shot gives the same bits alone or in a batch.
// ===========================================================================
__device__ __forceinline__ int find_shot(const ShotParams *shots, int n_shots, int64_t item,
                                         bool deposit) {
    int lo = 0, hi = n_shots - 1;  // largest s whose first item is <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t first = deposit ? shots[mid].ditem0 : shots[mid].item0;
        if (first <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The same from shot s0 on, for a block that took an item of shot s0 before
// (a block takes items in increasing order, so the shot is s0 or a later one,
// mostly within a few): a doubling search forward from s0, then bisection.
__device__ __forceinline__ int find_shot_from(const ShotParams *shots, int n_shots, int64_t item,
                                              bool deposit, int s0) {
    auto first = [&](int s) { return deposit ? shots[s].ditem0 : shots[s].item0; };
    int lo = s0, step = 1;  // first(lo) <= item throughout
    while (lo + step < n_shots && first(lo + step) <= item) {
        lo += step;
        step <<= 1;
    }
    int hi = min(lo + step, n_shots) - 1;  // first(hi + 1) > item, or hi the last shot
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first(mid) <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The shot of a group of the mixed-precision derivative passes.
__device__ __forceinline__ int find_group_shot(const ShotParams *shots, int n_shots, int64_t grp) {
    int lo = 0, hi = n_shots - 1;  // largest s whose first group is <= grp
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (shots[mid].gitem0 <= grp)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t next_item(unsigned int *counter, int64_t *slot) {
    if (threadIdx.x == 0) *slot = (int64_t)atomicAdd(counter, 1u);
    __syncthreads();
    const int64_t item = *slot;
    __syncthreads();
    return item;
}

// ===========================================================================
// Deposit of sample laws into fixed-point histograms
// ===========================================================================
// The deposited law of a sample is its own law (a point at v if s = 0, else
// N(v, s^2)) convolved with the deposit kernel (POINT: none; CIC: a box one
// bin wide; GAUSS: N(0, (ksig bins)^2)).  Bin masses are differences of the
// law's CDF at the bin edges, quantised to 2^-32 so that every sample adds
// exactly 2^32; beyond 6 standard deviations the CDF is taken as 0 or 1 (the
// neglected mass, 2e-9 a sample, goes to the edge bins of the window).  The
// CDF is evaluated in FP32 on whichever side of v keeps it small (the tail),
// so its error is a few ulps of the smaller tail mass.  For the box (x)
// Gaussian law the CDF is a difference of Psi(x) = Int_-inf^x Phi(u/s) du at
// the two box ends, and consecutive edges share one end.  Psi is of order s
// while the difference is of order one bin, so for laws wider than 4 bins
// that difference would lose log2(s / bin) bits in FP32; there the CDF is
// the box average of Phi as a series in beta = bin / s instead,
//   F = Phi(z) + beta^2/24 Phi''(z) + beta^4/1920 Phi''''(z),  z = t / s,
// whose next term is below 2e-9 for beta <= 1/4.
constexpr unsigned long long kOne = 1ull << 32;

// erfc(a) for a >= 0 without branches, given ea2 = exp(-a^2): the
// Chebyshev-fitted form erfc(a) = t exp(-a^2 + P(t)), t = 1 / (1 + a/2), of
// Press, Teukolsky, Vetterling and Flannery, Numerical Recipes (2nd ed.,
// Sec. 6.2), fractional error below 1.2e-7 for every a >= 0.  The library
// erfcf branches on the argument range, which costs a wavefront every branch
// its lanes take.
__device__ __forceinline__ float erfc_pos(float a, float ea2) {
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, a, 1.0f));
    float p = 0.17087277f;
    p = fmaf(p, t, -0.82215223f);
    p = fmaf(p, t, 1.48851587f);
    p = fmaf(p, t, -1.13520398f);
    p = fmaf(p, t, 0.27886807f);
    p = fmaf(p, t, -0.18628806f);
    p = fmaf(p, t, 0.09678418f);
    p = fmaf(p, t, 0.37409196f);
    p = fmaf(p, t, 1.00002368f);
    p = fmaf(p, t, -1.26551223f);
    return t * ea2 * __expf(p);
}

// One law of a lane, ready for the wavefront deposit: kind 1 box, 2 Gaussian,
// 3 box (x) Gaussian, 4 box (x) Gaussian wider than 4 bins (the series), over
// edges ka .. kb (t0 = edge ka - v; sf the width, for kind 4 beta^2 instead);
// kind 0 when the sample deposits as a point (NGP bin in `ngp`: 0 underflow,
// k + 1 for bin k, n + 1 overflow), -1 when the lane has no sample.
struct LawLane {
    int kind, ka, kb, ngp;
    float t0, sf, inv_s;
};

// (inv_w: 1 / w; the window and bin decisions take the product, which
// differs from the quotient by an ulp at most: a value within 1e-16 of an
// edge may fall on either side)
__device__ __forceinline__ LawLane law_setup(double v, double s, int dep, double ksig, double lo,
                                             double w, double inv_w, int n) {
    LawLane L{0, 0, -1, 0, 0.0f, 0.0f, 0.0f};
    const double half = 0.5 * w;
    double se = s;
    if (dep == 2) {  // GAUSS
        const double ks = ksig * w;
        se = sqrt(s * s + ks * ks);
        L.kind = se > 0.0 ? 2 : 0;
    } else if (dep == 1) {  // CIC
        L.kind = s > 0.0 ? 3 : 1;
    } else {
        L.kind = s > 0.0 ? 2 : 0;
    }
    if (L.kind != 0) {
        const double reach =
            L.kind == 1 ? half : (L.kind == 2 ? 6.0 * se : 6.0 * se + half);
        const int ka =
            max((int)fmin(fmax(ceil((v - reach - lo) * inv_w), -1.0), (double)n + 1.0), 0);
        const int kb =
            min((int)fmin(fmax(floor((v + reach - lo) * inv_w), -1.0), (double)n + 1.0), n);
        if (ka > kb) {
            L.kind = 0;  // the whole law lies inside one bin (or outside)
        } else {
            L.ka = ka;
            L.kb = kb;
            L.t0 = (float)(fma((double)ka, w, lo) - v);
            L.sf = (float)se;
            L.inv_s = L.kind >= 2 ? __builtin_amdgcn_rcpf((float)se) : 0.0f;  // about one ulp
            if (L.kind == 3 && se >= 4.0 * w) {
                L.kind = 4;
                const float beta = (float)w * L.inv_s;
                L.sf = beta * beta;
            }
        }
    }
    if (L.kind == 0) {
        const double x = (v - lo) * inv_w;  // bin floor(x); v on an edge goes up
        L.ngp = !(x >= 0.0) ? 0 : (x >= (double)n ? n + 1 : (int)x + 1);
    }
    return L;
}

// Inclusive prefix maximum over the 64 lanes of a wavefront (DPP: shifts
// within rows of 16 lanes, then the row ends broadcast to the rows after).
__device__ __forceinline__ int wave_incl_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

// The laws of the 64 lanes of a wavefront, deposited together.  A law spans
// anywhere from one bin to the whole window, so one lane per law would leave
// most lanes idle behind the widest: instead the work of all 64 laws is laid
// end to end and the lanes take 64 consecutive pieces at a time; a lane finds
// its law from the marked starts of the block through a prefix maximum, and
// reads the law from the wavefront's LDS rows.  Two passes:
//  - positions (the box, the narrow box (x) Gaussian, Gaussians whose edges
//    lie more than a quarter standard deviation apart): one piece per edge,
//    law s taking edges ka - 1 .. kb (the first only to supply the lower box
//    end of edge ka), each edge's CDF evaluated on its own;
//  - runs (the wide box (x) Gaussian series and Gaussians with edges at most a
//    quarter standard deviation apart): one piece per run of up to kRunLen
//    consecutive edges on one side of the law's centre, starting at the run's
//    edge farthest from the centre.  The tail there is evaluated as in the
//    position pass; towards the centre the run adds the integral of the
//    Gaussian density phi over each edge interval by Boole's rule on four
//    subintervals of h = dz / 4 (dz: edge spacing in standard deviations, at
//    most 1/4), or by Simpson's on two of h = dz / 2 when every run of the
//    wavefront has dz <= 1/10, phi following the lattice by
//    phi(a - h) = phi(a) e^(a h - h^2/2) (one exponential a run: the ratio
//    itself shrinks by e^(-h^2) from one subinterval to the next).  Boole's
//    rule errs by 8/945 h^7 phi^(6), below 1e-5 of an interval's mass out to
//    6.4 standard deviations (its sixth derivative is He6(a) phi); Simpson's
//    by h^5/90 phi^(4), below 1e-5 of it out to 4 and below 4e-5 out to 6
//    standard deviations at dz <= 1/10, where the masses are below 1e-9 of a
//    sample; the products' roundings grow with the square of the edges
//    walked.  An FP32 emulation of thirteen-edge runs starting out to 6.2
//    standard deviations finds at most 2.0e-5 relative error in an
//    interval's mass with Boole's rule (dz in [0.02, 0.25]), and 1.2e-5 with
//    Simpson's (dz in [0.02, 0.125]) for runs starting within 4, against the
//    1e-4 a bin may err.
// Q[e] (u64) accumulates the quantised weight at or below edge e of the laws
// that cover e; cnt[c] (u32) counts the samples whose weight is all at or
// below edge c - 1 (a point in bin c - 1, or a law ending at edge c - 1), so
// that edge e carries Q[e] + 2^32 sum_(c <= e) cnt[c] in total.
//
// Per-wavefront LDS rows of wave_deposit: the 64 laws (kind | ka << 3, t0,
// sf, inv_s), their run shape (edges, edges below the centre), the piece
// offsets, and the start marks of a block of 64 pieces (-1 between uses; set
// to -1 once before the first use).
struct WaveLaws {
    int4 *rec;
    int2 *ext;
    int *off;
    int *mark;
};

// Edges a run.  Consecutive lanes of one law walk runs whose edges lie kRunLen
// words of 8 bytes apart: with eight, every second lane's atomic falls on the
// same 4-byte LDS bank (16 banks on); with an odd length they spread over the
// banks (the deposit's bank-conflict cycles drop by three quarters).  Thirteen
// rather than nine spreads a run's set-up over more edges (4% less time); the
// products' roundings grow with the square of the length.
constexpr int kRunLen = 13;

// Owner of piece p of a block (base .. base + 63): the last lane whose first
// piece is <= p.  Lanes with pieces mark their start if it falls in the block
// (starts are distinct); a prefix maximum carries each start to the pieces
// after it, the previous block's last owner (carry) to those before the first.
__device__ __forceinline__ int piece_owner(bool has, int off, int base, int carry,
                                           const WaveLaws &WL) {
    const int lane = threadIdx.x & 63;
    if (has && off >= base && off < base + 64) WL.mark[off - base] = lane;
    wave_sync_lds();
    const int m = WL.mark[lane];
    WL.mark[lane] = -1;
    return max(wave_incl_max(m), carry);
}

// Exclusive scan of n over the wavefront; *total receives the sum.
__device__ __forceinline__ int wave_excl_scan(int n, int *total) {
    const int lane = threadIdx.x & 63;
    int incl = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    *total = __builtin_amdgcn_readlane(incl, 63);
    return incl - n;
}

// Quantised weight of a CDF value at edge e (F: the tail mass on the side of
// the edge away from the law's centre), added to Q[e].
__device__ __forceinline__ void add_edge(unsigned long long *Q, int e, float F, bool upper) {
    F = fminf(fmaxf(F, 0.0f), 1.0f);
    // below 1, 2^32 F rounds to at most 2^32 - 256: 32 bits
    const unsigned long long qf =
        F >= 1.0f ? kOne : (unsigned long long)(uint32_t)rintf(F * 4294967296.0f);
    const unsigned long long q = upper ? kOne - qf : qf;
    if (q) atomicAdd(&Q[e], q);
}

// The same for an edge of a run, whose tail mass F is at most about one half:
// 2^32 F fits 32 bits, and the weight on the upper side, 2^32 - 2^32 F, has
// its high word set only when 2^32 F rounds to zero.  SPLIT: the upper side's
// tails go to an array of their own (Qe points into it) as they are, the
// 2^32 of each upper edge counted once a law at its first upper edge.
template <bool SPLIT>
__device__ __forceinline__ void add_run_edge(unsigned long long *Qe, float F, bool upper) {
    const uint32_t qf =
        (uint32_t)rintf(__builtin_amdgcn_fmed3f(F, 0.0f, 0x1.fffffep-1f) * 4294967296.0f);
    if constexpr (SPLIT) {
        atomicAdd(Qe, (unsigned long long)qf);
    } else {
        const uint32_t lo = upper ? 0u - qf : qf;
        const uint32_t hi = upper && qf == 0u ? 1u : 0u;
        atomicAdd(Qe, ((unsigned long long)hi << 32) | lo);
    }
}

// The edges of one run from the tail inwards (see wave_deposit): a0, ph0 and
// T0 are the distance from the centre, the density and the tail mass at the
// run's first edge; each step adds the density's integral over one edge
// interval, by Simpson's rule on two subintervals (SIMP) or Boole's on four,
// the density following the lattice by phi(a - h) = phi(a) e^(a h - h^2/2): the
// ratio itself shrinks by e^(-h^2) from one subinterval to the next.
template <bool SIMP, bool SPLIT>
__device__ __forceinline__ void walk_run(unsigned long long *qe, int step, int len, int kind,
                                         float sf, float da, float a0, float ph0, float T0,
                                         bool upper) {
    constexpr int kSub = SIMP ? 2 : 4;
    const float hs = da * (1.0f / kSub);
    const float q = __expf(-hs * hs), qn = __expf(-(float)kSub * hs * hs);
    const float cb = hs * (SIMP ? 1.0f / 3.0f : 2.0f / 45.0f);
    float a = a0, ph = ph0, T = T0;
    float rho = __expf(fmaf(a, hs, -0.5f * hs * hs));  // phi(a - hs) / phi(a)
    for (int k = 0; k < kRunLen; ++k) {
        if (k < len) {
            if (k > 0) {
                // from the previous edge (a) one edge towards the centre
                float r = rho;
                const float p1 = ph * r;
                r *= q;
                const float p2 = p1 * r;
                if constexpr (SIMP) {
                    T = fmaf(cb, fmaf(4.0f, p1, ph + p2), T);
                    ph = p2;
                } else {
                    r *= q;
                    const float p3 = p2 * r;
                    r *= q;
                    const float p4 = p3 * r;
                    T = fmaf(cb, fmaf(7.0f, ph + p4, fmaf(32.0f, p1 + p3, 12.0f * p2)), T);
                    ph = p4;
                }
                rho *= qn;
                a -= da;
            }
            // wide box (x) Gaussian: the series' even terms beside the tail
            // (sf holds beta^2), with the sign of the tail on either side
            const float c = sf * fmaf(sf * (1.0f / 1920.0f), fmaf(a, a, -3.0f), 1.0f / 24.0f);
            const float F = kind == 4 ? fmaf(a * ph, c, T) : T;
            add_run_edge<SPLIT>(qe + step * k, F, upper);
        }
    }
}

// SPLIT: the runs' upper-side tails go to QU (see add_run_edge), and a law
// walked in runs counts its sample at its first upper edge instead of past
// its last edge: edge e carries Q[e] - QU[e] + 2^32 sum_(c <= e) cnt[c].
template <bool SPLIT>
__device__ __forceinline__ void wave_deposit(const LawLane &L, double w, float hf,
                                             unsigned long long *Q, unsigned long long *QU,
                                             unsigned int *cnt, const WaveLaws &WL) {
    const int lane = threadIdx.x & 63;
    const float wf = (float)w, inv_w = (float)(1.0 / w);
    // runs: the wide box (x) Gaussian, and Gaussians with dz <= 1/4
    const bool run = L.kind == 4 || (L.kind == 2 && wf * L.inv_s <= 0.25f);
    const int ne = L.kind > 0 ? L.kb - L.ka + 1 : 0;  // edges of the law
    // edges at or below the centre (t <= 0, as the position pass decides it)
    int nl = 0;
    if (run) {
        nl = min(max((int)floorf(-L.t0 * inv_w) + 1, 0), ne);
        if (nl > 0 && fmaf((float)(nl - 1), wf, L.t0) > 0.0f) --nl;
        if (nl < ne && fmaf((float)nl, wf, L.t0) <= 0.0f) ++nl;
    }
    if (L.kind == 0) atomicAdd(&cnt[L.ngp], 1u);
    if (L.kind > 0) atomicAdd(&cnt[SPLIT && run ? L.ka + nl : L.kb + 1], 1u);
    WL.rec[lane] = make_int4(L.kind | (L.ka << 3), __float_as_int(L.t0), __float_as_int(L.sf),
                             __float_as_int(L.inv_s));
    WL.ext[lane] = make_int2(ne, nl);

    // ---- position pass ----
    const int np = L.kind > 0 && !run ? ne + 1 : 0;
    int total;
    int off = wave_excl_scan(np, &total);
    WL.off[lane] = off;
    float cP = 0.0f, cPc = 0.0f;  // box ends of the previous block's last position
    int carry = 0;                // owner of the previous block's last position
    for (int base = 0; base < total; base += 64) {
        const int p = base + lane;
        const int own = piece_owner(np > 0, off, base, carry, WL);
        carry = __builtin_amdgcn_readlane(own, 63);
        const int4 r = WL.rec[own];
        const int kind = r.x & 7, ka = r.x >> 3;
        const int rel = p - WL.off[own] - 1;  // edge - ka
        const float t0 = __int_as_float(r.y), sf = __int_as_float(r.z);
        const float inv_s = __int_as_float(r.w);
        wave_sync_lds();  // the marks and rows are rewritten after this block
        const bool live = p < total && rel >= 0;
        const float t = fmaf((float)rel, wf, t0);
        const bool upper = t > 0.0f;
        // One Gaussian tail a position, without branches (one exponential
        // serves phi and the tail): at the edge for the Gaussian law, at the
        // upper box end x = t + b/2 for the narrow box (x) Gaussian, whose CDF
        // is a difference of Psi(x) = x Phi(x/s) + s phi(x/s) at the two box
        // ends; Psi(x) and Psi(x) - x = -x Phi(-x/s) + s phi(x/s) are formed
        // from the tail on the side of x (no cancellation) and consecutive
        // edges share one end.  All positions of a law are alike, so the box
        // ends passed between lanes are those of narrow laws only.
        const float x = kind == 3 ? t + hf : t;
        const float zz = x * inv_s;
        const float e2 = __expf(-0.5f * zz * zz);  // relative error below 2e-6 out to 6 sigma
        const float phz = 0.39894228040143267794f * e2;
        const float tail = 0.5f * erfc_pos(fabsf(zz) * 0.70710678118654752440f, e2);
        float P = 0.0f, Pc = 0.0f;
        if (__any(kind == 3)) {
            const float ph = sf * phz;
            const float lo = fmaf(x, tail, ph);   // Psi(x) when x <= 0
            const float hi = fmaf(-x, tail, ph);  // Psi(x) - x when x > 0
            P = zz <= 0.0f ? lo : hi + x;
            Pc = zz <= 0.0f ? lo - x : hi;
        }
        float lP = __shfl_up(P, 1, 64), lPc = __shfl_up(Pc, 1, 64);
        if (lane == 0) {
            lP = cP;
            lPc = cPc;
        }
        cP = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(P), 63));
        cPc = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Pc), 63));
        if (live) {
            const float Fbox = upper ? 0.5f - t * inv_w : fmaf(t, inv_w, 0.5f);
            const float Fpsi = upper ? (lPc - Pc) * inv_w : (P - lP) * inv_w;
            const float F = kind == 3 ? Fpsi : (kind == 2 ? tail : Fbox);
            add_edge(Q, ka + rel, F, upper);
        }
    }
    wave_sync_lds();  // the offsets are rewritten below

    // ---- run pass ----
    const int rl = run ? (nl + kRunLen - 1) / kRunLen : 0;
    const int nr = run ? rl + (ne - nl + kRunLen - 1) / kRunLen : 0;
    off = wave_excl_scan(nr, &total);
    WL.off[lane] = off;
    carry = 0;
    for (int base = 0; base < total; base += 64) {
        const int p = base + lane;
        const int own = piece_owner(nr > 0, off, base, carry, WL);
        carry = __builtin_amdgcn_readlane(own, 63);
        const int4 r = WL.rec[own];
        const int2 x2 = WL.ext[own];
        const int j = p - WL.off[own];  // run of the law
        wave_sync_lds();
        const int kind = r.x & 7, ka = r.x >> 3;
        const float t0 = __int_as_float(r.y), sf = __int_as_float(r.z);
        const float inv_s = __int_as_float(r.w);
        const int n_e = x2.x, n_l = x2.y, r_l = (n_l + kRunLen - 1) / kRunLen;
        const bool upper = j >= r_l;
        // first edge (farthest from the centre) and length of the run
        const int rel0 = upper ? n_e - 1 - (j - r_l) * kRunLen : j * kRunLen;
        const int len = p < total ? (upper ? min(kRunLen, n_e - n_l - (j - r_l) * kRunLen)
                                           : min(kRunLen, n_l - j * kRunLen))
                                  : 0;
        const int step = upper ? -1 : 1;
        const float da = wf * inv_s;  // edge spacing in standard deviations
        // the tail at the run's first edge
        const float a0 = fabsf(fmaf((float)rel0, wf, t0) * inv_s);
        const float e2 = __expf(-0.5f * a0 * a0);
        const float ph0 = 0.39894228040143267794f * e2;
        const float T0 = 0.5f * erfc_pos(a0 * 0.70710678118654752440f, e2);
        unsigned long long *qe = (SPLIT && upper ? QU : Q) + (ka + rel0);
        // Simpson's rule on half edges where the laws of all the wavefront's
        // runs have edges at most a tenth of a standard deviation apart (its
        // error then stays within 1e-5 of an interval's mass out to four
        // standard deviations), Boole's on quarter edges otherwise
        if (__all(!(p < total) || da <= 0.1f))
            walk_run<true, SPLIT>(qe, step, len, kind, sf, da, a0, ph0, T0, upper);
        else
            walk_run<false, SPLIT>(qe, step, len, kind, sf, da, a0, ph0, T0, upper);
    }
    wave_sync_lds();  // the next call rewrites the rows
}

// ===========================================================================
// Wavefront reductions
// ===========================================================================
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Grid of resident blocks for a persistent work-queue kernel (never more
// blocks than items; at most cap blocks a CU when cap > 0).
inline hipError_t resident_grid(const void *fn, int block, size_t lds, int64_t items, int *grid,
                                int cap = 0) {
    int device = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds);
    if (e != hipSuccess) return e;
    if (cap > 0 && per_cu > cap) per_cu = cap;
    int64_t g = (int64_t)(per_cu < 1 ? 1 : per_cu) * ncu;
    if (g > items) g = items;
    *grid = (int)(g < 1 ? 1 : g);
    return hipSuccess;
}

}  // namespace qs
