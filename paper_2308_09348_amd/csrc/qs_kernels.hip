// qs_kernels.hip -- gfx950 kernels of the beam-phase-space integrator.
//
// Hot path (Amaro & Vranic, arXiv 2308.09348).  The phase kernel gives one
// lane one beam sample at a time: it draws the sample (Philox4x32-10 +
// Box-Muller), places it on its ballistic path through the focused pulse
// (Sec. 2, eq. a0eff, Table 1 offsets) and integrates its mean energy and
// energy variance along the phase with RK4 under the radiation-reaction drift
// of eq. dpdtRR (classical limit: eq. PWCRR), with the state in registers and
// the radiation-function table in LDS.  It writes the final state (56 bytes a
// sample).  The deposit kernel turns final states into energy and angle laws
// (eq. dNda2dNdgf as a push-forward; Sec. 5.2 divergence) deposited into
// block-private LDS histograms in 32.32 fixed point, merged into global
// integer histograms (order-independent), plus FP64 moment partials that a
// finalize kernel reduces in a fixed order.  The split keeps the FP64
// deposit arithmetic from setting the register budget of the phase loop.
// Nothing here is a dense contraction, so no MFMA: the bound is the vector
// ALU of the phase loop.
#include "qs_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

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

// Six standard normals of sample i: counter (i, shot, k, 0) for k = 0, 1,
// 24-bit uniforms u = ((r >> 8) + 1/2) 2^-24, Box-Muller on pairs.
__device__ __forceinline__ void sample_normals(uint32_t i, uint32_t shot, uint32_t k0, uint32_t k1,
                                               double n[6]) {
    uint32_t r[8];
#pragma unroll
    for (uint32_t k = 0; k < 2; ++k) {
        uint32_t c[4] = {i, shot, k, 0u};
        philox4x32_10(c, k0, k1);
        r[4 * k + 0] = c[0];
        r[4 * k + 1] = c[1];
        r[4 * k + 2] = c[2];
        r[4 * k + 3] = c[3];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double u1 = ((double)(r[2 * m] >> 8) + 0.5) * 0x1p-24;
        const double u2 = ((double)(r[2 * m + 1] >> 8) + 0.5) * 0x1p-24;
        const double R = sqrt(-2.0 * log(u1));
        double s, c;
        sincospi(2.0 * u2, &s, &c);
        n[2 * m] = R * c;
        n[2 * m + 1] = R * s;
    }
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

__device__ __forceinline__ void rad_lookup32(const float *__restrict__ tab, float chi,
                                             RadCell32 &cell) {
    const uint32_t b = __float_as_uint(chi);
    int c = (int)(b >> (23 - kSB32)) - ((127 + kEMin) << kSB32) + 1;
    // cell start 2^e (1 + sub/2^SB) and inverse width 2^(SB - e)
    float tw = __uint_as_float((uint32_t)(254 + kSB32 - (int)(b >> 23)) << 23);
    float ts = -__uint_as_float(b & ~((1u << (23 - kSB32)) - 1)) * tw;
    if (c < 1) {  // chi < 2^kEMin: the first cell, linear in chi
        c = 0;
        tw = 0x1p20f;
        ts = 0.0f;
    }
    if (c > kCells32 - 1) {  // beyond the table (reported by the caller)
        c = kCells32 - 1;
        tw = 0.0f;
        ts = 1.0f;
    }
    const float4 *T = reinterpret_cast<const float4 *>(tab);
    cell.q0 = T[c];
    cell.q1 = T[kCells32 + c];
    cell.q2 = T[2 * kCells32 + c];
    cell.q3 = T[3 * kCells32 + c];
    cell.tw = tw;
    cell.ts = ts;
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

__device__ __forceinline__ void rad_eval64(const double *__restrict__ tab, double chi, double &g,
                                           double &G1, double &G2, double &hq) {
    const uint64_t b = (uint64_t)__double_as_longlong(chi);
    int64_t c = (int64_t)(b >> (52 - kSB64)) - ((int64_t)(1023 + kEMin) << kSB64) + 1;
    double t = __longlong_as_double((long long)(((b & ((1ull << (52 - kSB64)) - 1)) << kSB64) |
                                                0x3ff0000000000000ull)) - 1.0;
    if (c < 1) {
        c = 0;
        t = chi * 0x1p20;
    }
    c = c < kCells64 - 1 ? c : kCells64 - 1;
    const double *q = tab + (size_t)c * kCellVals;
    g = fma(t, fma(t, fma(t, q[3], q[2]), q[1]), q[0]);
    G1 = fma(t, fma(t, fma(t, q[7], q[6]), q[5]), q[4]);
    G2 = fma(t, fma(t, fma(t, q[11], q[10]), q[9]), q[8]);
    hq = fma(t, fma(t, fma(t, q[15], q[14]), q[13]), q[12]);
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

template <class T, bool QUANTUM>
__device__ __forceinline__ void rhs(T mu, T s2, T a, const Phys<T> &ph, const RadTab<T> &tab,
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

// Geometry of one sample along its ballistic path: at phase psi it has
// travelled l = psi lambda / (4 pi) past its collision point.
template <class T>
struct Path {
    T xc, yc, thx, thy, zstar, inv_w0sq, inv_zR;
    __device__ __forceinline__ T S(T ell) const {
        return spatial(fma(thx, ell, xc), fma(thy, ell, yc), zstar - ell, inv_w0sq, inv_zR);
    }
};

// One RK4 step of (mu, sig2) from psi_j with amplitudes a1 = a(psi_j),
// ah = a(psi_j + h/2), a4 = a(psi_j + h); returns the increments.
template <class T, bool QUANTUM>
__device__ __forceinline__ void rk4_increment(T mu, T s2, T a1, T ah, T a4, T h,
                                              const Phys<T> &ph, const RadTab<T> &tab, T &dmu,
                                              T &ds2, T &chi_hi) {
    const T hh = T(0.5) * h;
    T k1m, k1s, k2m, k2s, k3m, k3s, k4m, k4s;
    rhs<T, QUANTUM>(mu, s2, a1, ph, tab, k1m, k1s, chi_hi);
    rhs<T, QUANTUM>(fma(hh, k1m, mu), fma(hh, k1s, s2), ah, ph, tab, k2m, k2s, chi_hi);
    rhs<T, QUANTUM>(fma(hh, k2m, mu), fma(hh, k2s, s2), ah, ph, tab, k3m, k3s, chi_hi);
    rhs<T, QUANTUM>(fma(h, k3m, mu), fma(h, k3s, s2), a4, ph, tab, k4m, k4s, chi_hi);
    const T h6 = h * T(1.0 / 6.0);
    dmu = h6 * (k1m + T(2) * (k2m + k3m) + k4m);
    ds2 = h6 * (k1s + T(2) * (k2s + k3s) + k4s);
}

// Moment right-hand side (quantum model) from the FP32 table's combined
// functions at chi = two_over_aS mu |a|:  T1 = g,  T2 = 2g + chi g',
// T3 = g + 2 chi g' + chi^2 g''/2,  T4 = h, so that
//   dmu/dpsi   = -K a^2 (mu^2 T1 + sig2 T3),
//   dsig2/dpsi = -2 K a^2 mu sig2 T2 + C_D a^2 |a| mu^4 T4.
__device__ __forceinline__ void rhs_q32(float mu, float s2, float a2, float aa, float T1, float T2,
                                        float T3, float T4, const Phys<float> &ph, float &dmu,
                                        float &ds2) {
    const float u = ph.K * a2;
    const float mu2 = mu * mu;
    dmu = -u * fmaf(mu2, T1, s2 * T3);
    const float D = (ph.CD * aa) * a2 * (mu2 * mu2) * T4;
    ds2 = fmaf(-2.0f * u * mu * s2, T2, D);
}

// One FP32 RK4 step of the quantum moment system with two table reads:
// stage 2 and stage 4 read LDS, stage 3 reuses stage 2's cell, and stage 4's
// cell is handed to the next step's stage 1.
__device__ __forceinline__ void rk4_q32(float mu, float s2, float a1, float ah, float a4, float h,
                                        const Phys<float> &ph, const float *__restrict__ tab,
                                        RadCell32 &carry, float &dmu, float &ds2,
                                        float &chi_hi) {
    const float hh = 0.5f * h;
    float g, G1, G2, hq;
    // stage 1 (cell carried from the previous stage 4)
    const float aa1 = fabsf(a1), a21 = a1 * a1;
    const float c1 = ph.two_over_aS * mu * aa1;
    rad_cell_eval(carry, c1, g, G1, G2, hq);
    float k1m, k1s;
    rhs_q32(mu, s2, a21, aa1, g, G1, G2, hq, ph, k1m, k1s);
    // stage 2 (table read)
    const float aah = fabsf(ah), a2h = ah * ah;
    const float m2 = fmaf(hh, k1m, mu), s22 = fmaf(hh, k1s, s2);
    const float c2 = ph.two_over_aS * m2 * aah;
    RadCell32 mid;
    rad_lookup32(tab, c2, mid);
    rad_cell_eval(mid, c2, g, G1, G2, hq);
    float k2m, k2s;
    rhs_q32(m2, s22, a2h, aah, g, G1, G2, hq, ph, k2m, k2s);
    // stage 3 (same phase as stage 2: reuse its cell)
    const float m3 = fmaf(hh, k2m, mu), s23 = fmaf(hh, k2s, s2);
    const float c3 = ph.two_over_aS * m3 * aah;
    rad_cell_eval(mid, c3, g, G1, G2, hq);
    float k3m, k3s;
    rhs_q32(m3, s23, a2h, aah, g, G1, G2, hq, ph, k3m, k3s);
    // stage 4 (table read; its cell serves the next step's stage 1)
    const float aa4 = fabsf(a4), a24 = a4 * a4;
    const float m4 = fmaf(h, k3m, mu), s24 = fmaf(h, k3s, s2);
    const float c4 = ph.two_over_aS * m4 * aa4;
    rad_lookup32(tab, c4, carry);
    rad_cell_eval(carry, c4, g, G1, G2, hq);
    float k4m, k4s;
    rhs_q32(m4, s24, a24, aa4, g, G1, G2, hq, ph, k4m, k4s);
    chi_hi = fmaxf(chi_hi, fmaxf(fmaxf(c1, c2), fmaxf(c3, c4)));
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
// Deposit of one law into block-private fixed-point histograms
// ===========================================================================
constexpr unsigned long long kOne = 1ull << 32;


__device__ __forceinline__ void ngp(double v, double lo, double w, int n,
                                    unsigned long long *h) {
    const double x = (v - lo) / w;
    int k;
    if (!(x >= 0.0))
        k = n;  // underflow
    else if (x >= (double)n)
        k = n + 1;  // overflow
    else
        k = (int)x;
    atomicAdd(&h[k], kOne);
}

// The deposited law is the sample's own law (a point at v if s = 0, else
// N(v, s^2)) convolved with the deposit kernel (POINT: none; CIC: a box one
// bin wide; GAUSS: N(0, (ksig bins)^2)).  Bin masses are differences of the
// law's CDF at the bin edges, quantised to 2^-32 so that every sample adds
// exactly 2^32; beyond 6 standard deviations the CDF is taken as 0 or 1 (the
// neglected mass, 2e-9 a sample, goes to the edge bins of the window).  The
// CDF is evaluated in FP32 on whichever side of v keeps it small (erfc of
// the tail), so its error is a few ulps of the smaller tail mass.  For the
// box (x) Gaussian law the CDF is a difference of Psi(x) = Int_-inf^x
// Phi(u/s) du at the two box ends, and consecutive edges share one end.
struct PsiPair {
    float P, Pc;  // Psi(x) and Psi(x) - x
};
__device__ __forceinline__ PsiPair psi_pair(float x, float s, float inv_s) {
    const float zz = x * inv_s;
    const float ph = s * 0.39894228040143267794f * expf(-0.5f * zz * zz);
    PsiPair r;
    if (zz <= 0.0f) {
        r.P = fmaf(x, 0.5f * erfcf(-zz * 0.70710678118654752440f), ph);
        r.Pc = r.P - x;
    } else {
        r.Pc = fmaf(-x, 0.5f * erfcf(zz * 0.70710678118654752440f), ph);
        r.P = r.Pc + x;
    }
    return r;
}

__device__ void deposit_law(double v, double s, int dep, double ksig, double lo, double w, int n,
                            unsigned long long *h) {
    const double half = 0.5 * w;
    int mode;
    double se = s;
    if (dep == 2) {  // GAUSS
        const double ks = ksig * w;
        se = sqrt(s * s + ks * ks);
        mode = se > 0.0 ? 2 : 0;
    } else if (dep == 1) {  // CIC
        mode = s > 0.0 ? 3 : 1;
    } else {
        mode = s > 0.0 ? 2 : 0;
    }
    if (mode == 0) {
        ngp(v, lo, w, n, h);
        return;
    }
    const double reach = mode == 1 ? half : (mode == 2 ? 6.0 * se : 6.0 * se + half);
    int ka = (int)fmin(fmax(ceil((v - reach - lo) / w), -1.0), (double)n + 1.0);
    int kb = (int)fmin(fmax(floor((v + reach - lo) / w), -1.0), (double)n + 1.0);
    ka = max(ka, 0);
    kb = min(kb, n);
    if (ka > kb) {
        ngp(v, lo, w, n, h);  // the whole law lies inside one bin (or outside)
        return;
    }
    const float sf = (float)se, inv_s = mode >= 2 ? (float)(1.0 / se) : 0.0f;
    const float wf = (float)w, inv_w = (float)(1.0 / w), hf = (float)half;
    PsiPair lower{0.0f, 0.0f};
    if (mode == 3) lower = psi_pair((float)(fma((double)ka, w, lo) - v) - hf, sf, inv_s);
    unsigned long long qprev = 0;
    for (int k = ka; k <= kb; ++k) {
        const float t = (float)(fma((double)k, w, lo) - v);  // edge - v
        const bool upper = t > 0.0f;  // F is taken from the upper tail there
        float F;
        if (mode == 1) {
            F = upper ? 0.5f - t * inv_w : fmaf(t, inv_w, 0.5f);
        } else if (mode == 2) {
            F = 0.5f * erfcf((upper ? t : -t) * inv_s * 0.70710678118654752440f);
        } else {
            const PsiPair up = psi_pair(t + hf, sf, inv_s);
            F = upper ? (lower.Pc - up.Pc) * inv_w : (up.P - lower.P) * inv_w;
            lower = up;
        }
        (void)wf;
        F = fminf(fmaxf(F, 0.0f), 1.0f);
        const unsigned long long qf = (unsigned long long)llrintf(F * 4294967296.0f);
        unsigned long long q = upper ? kOne - qf : qf;
        q = q < qprev ? qprev : q;
        const int bin = k == 0 ? n : k - 1;  // mass between edge k-1 and edge k
        if (q != qprev) atomicAdd(&h[bin], q - qprev);
        qprev = q;
    }
    const int bin = kb == n ? n + 1 : kb;  // mass above the last edge in the window
    if (qprev != kOne) atomicAdd(&h[bin], kOne - qprev);
}

// ===========================================================================
// Work items.  A launch covers n_shots shots; phase items are tiles of
// kPhaseBlock consecutive samples of one shot (one sample per lane), deposit
// items tiles of kDepTile samples.  Blocks take items from a counter; an
// item's result does not depend on which block runs it, so the output is
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

__device__ __forceinline__ int64_t next_item(unsigned int *counter, int64_t *slot) {
    if (threadIdx.x == 0) *slot = (int64_t)atomicAdd(counter, 1u);
    __syncthreads();
    const int64_t item = *slot;
    __syncthreads();
    return item;
}

// ===========================================================================
// Phase kernel: sample -> ballistic path -> RK4 phase loop -> final state
// ===========================================================================
// The envelope tables come as separate restrict-qualified arguments: the
// kernel never writes them, so the compiler reads them with scalar loads
// (every lane of a wavefront is at the same phase step).
template <int PREC, bool QUANTUM, bool LOCAL>
__device__ __forceinline__ void phase_sample(const BatchParams &P, const ShotParams &sp, int64_t i,
                                             const float *__restrict__ env32,
                                             const double *__restrict__ env64,
                                             const float *tab32, int &flags) {
    const RadTab<double> tabd{P.rad64};
    const RadTab<float> tabf{tab32};
    const Phys<float> phf{P.Kf, P.CDf, P.two_over_aSf};
    const Phys<double> phd{P.K, P.CD, P.two_over_aS};
    const int N = P.n_steps;
    const bool local = LOCAL && !sp.plane_wave;
    const float chi_top = (float)(1 << (kEMax + 1));  // end of the tabulated range

    // ---- sample and geometry (FP64, once per sample) ----
    double nrm[6];
    sample_normals((uint32_t)i, (uint32_t)sp.shot_word, P.key0, P.key1, nrm);
    const double x = fma(sp.sigma_r, nrm[0], sp.x_off);
    const double y = fma(sp.sigma_r, nrm[1], sp.y_off);
    const double z = sp.sigma_z * nrm[2];
    const double g0 = fma(sp.sigma_gamma, nrm[3], sp.gamma0);
    const double thx = sp.div_rad * nrm[4];
    const double thy = sp.div_rad * nrm[5];
    Path<double> pd;
    pd.xc = fma(thx, 0.5 * z, x);
    pd.yc = fma(thy, 0.5 * z, y);
    pd.thx = thx;
    pd.thy = thy;
    pd.zstar = fma(0.5, z, sp.z_delay);
    pd.inv_w0sq = sp.inv_w0sq;
    pd.inv_zR = sp.inv_zR;
    const double S0 = sp.plane_wave ? 1.0 : pd.S(0.0);
    const double a0S0 = sp.a0 * S0;

    double mu_f, s2_f;
    float cmx = 0.0f;     // largest chi at a step start for this sample
    float chi_hi = 0.0f;  // largest chi at any stage (range check)
    if (PREC == PREC_F64) {
        double mu = g0, s2 = 0.0, chd = 0.0;
        double aS_prev = local ? sp.a0 * pd.S(-P.psi_max * P.ell_per_psi) : a0S0;
        for (int j = 0; j < N; ++j) {
            const double psi = fma((double)j, P.h, -P.psi_max);
            double aSh = a0S0, aS4 = a0S0;
            if (local) {
                aSh = sp.a0 * pd.S(fma(0.5, P.h, psi) * P.ell_per_psi);
                aS4 = sp.a0 * pd.S((psi + P.h) * P.ell_per_psi);
            }
            const double a1 = aS_prev * env64[2 * j];
            const double ah = aSh * env64[2 * j + 1];
            const double a4 = aS4 * env64[2 * j + 2];
            cmx = fmaxf(cmx, (float)(P.two_over_aS * mu * fabs(a1)));
            double dm, ds;
            rk4_increment<double, QUANTUM>(mu, s2, a1, ah, a4, P.h, phd, tabd, dm, ds, chd);
            mu += dm;
            s2 += ds;
            aS_prev = aS4;
        }
        mu_f = mu;
        s2_f = s2;
        chi_hi = (float)chd;
    } else {
        Path<float> pf;
        pf.xc = (float)pd.xc;
        pf.yc = (float)pd.yc;
        pf.thx = (float)thx;
        pf.thy = (float)thy;
        pf.zstar = (float)pd.zstar;
        pf.inv_w0sq = sp.inv_w0sqf;
        pf.inv_zR = sp.inv_zRf;
        const float a0f = sp.a0f;
        const float a0S0f = (float)a0S0;
        float mu = (float)g0, mu_lo = (float)(g0 - (double)mu), s2 = 0.0f, s2_lo = 0.0f;
        // the part of g0 that the FP32 pair cannot hold, restored at the end
        const double g0_rest = (g0 - (double)mu) - (double)mu_lo;
        double chd = 0.0;
        float aS_prev = local ? a0f * pf.S(P.psi0f * P.ellf) : a0S0f;
        RadCell32 carry;
        if (QUANTUM) rad_lookup32(tab32, phf.two_over_aS * mu * fabsf(aS_prev * env32[0]), carry);
        // local amplitude: one spatial factor per step, at psi_{j+2}; the
        // stage-2/3 value at psi_j + h/2 is the quadratic through psi_j,
        // psi_{j+1} and psi_{j+2} (error of order h^3 times the third
        // derivative of S, far below FP32 rounding)
        float aS_next = local ? a0f * pf.S((P.psi0f + P.hf) * P.ellf) : a0S0f;
        for (int j = 0; j < N; ++j) {
            float aSh = a0S0f, aS4 = a0S0f;
            if (local && sp.mid_interp) {
                const float psi2 = fmaf((float)(j + 2), P.hf, P.psi0f);
                const float aS_far = a0f * pf.S(psi2 * P.ellf);
                aS4 = aS_next;
                aSh = fmaf(0.375f, aS_prev, fmaf(0.75f, aS4, -0.125f * aS_far));
                aS_next = aS_far;
            } else if (local) {  // coarse steps: both points exactly
                const float psi = fmaf((float)j, P.hf, P.psi0f);
                aSh = a0f * pf.S(fmaf(0.5f, P.hf, psi) * P.ellf);
                aS4 = a0f * pf.S((psi + P.hf) * P.ellf);
            }
            const float a1 = aS_prev * env32[2 * j];
            const float ah = aSh * env32[2 * j + 1];
            const float a4 = aS4 * env32[2 * j + 2];
            const float chi1 = phf.two_over_aS * mu * fabsf(a1);
            cmx = fmaxf(cmx, chi1);
            bool promote = false;
            if (PREC == PREC_F32MIX) promote = __any(chi1 > P.chi_fp64);
            if (promote) {
                // the whole wavefront runs this step in FP64 (uniform branch)
                const double psid = fma((double)j, P.h, -P.psi_max);
                double A1 = a0S0, Ah = a0S0, A4 = a0S0;
                if (local) {
                    A1 = sp.a0 * pd.S(psid * P.ell_per_psi);
                    Ah = sp.a0 * pd.S(fma(0.5, P.h, psid) * P.ell_per_psi);
                    A4 = sp.a0 * pd.S((psid + P.h) * P.ell_per_psi);
                }
                A1 *= env64[2 * j];
                Ah *= env64[2 * j + 1];
                A4 *= env64[2 * j + 2];
                const double mud = (double)mu + (double)mu_lo;
                const double s2d = (double)s2 + (double)s2_lo;
                double dm, ds;
                rk4_increment<double, QUANTUM>(mud, s2d, A1, Ah, A4, P.h, phd, tabd, dm, ds, chd);
                const double mn = mud + dm, sn = s2d + ds;
                mu = (float)mn;
                mu_lo = (float)(mn - (double)mu);
                s2 = (float)sn;
                s2_lo = (float)(sn - (double)s2);
                // the next FP32 stage 1 needs the cell at the new state
                rad_lookup32(tab32, phf.two_over_aS * mu * fabsf(aS4 * env32[2 * j + 2]), carry);
            } else if (QUANTUM) {
                float dm, ds;
                rk4_q32(mu, s2, a1, ah, a4, P.hf, phf, tab32, carry, dm, ds, chi_hi);
                comp_add(mu, mu_lo, dm);
                comp_add(s2, s2_lo, ds);
            } else {
                float dm, ds;
                rk4_increment<float, false>(mu, s2, a1, ah, a4, P.hf, phf, tabf, dm, ds, chi_hi);
                comp_add(mu, mu_lo, dm);
            }
            aS_prev = aS4;
        }
        mu_f = ((double)mu + (double)mu_lo) + g0_rest;
        s2_f = (double)s2 + (double)s2_lo;
        chi_hi = fmaxf(chi_hi, (float)chd);
    }
    {
        // chi at the end of the last step (the pulse tail)
        const double aN = (local ? sp.a0 * pd.S(P.psi_max * P.ell_per_psi) : a0S0) * env64[2 * N];
        cmx = fmaxf(cmx, (float)(P.two_over_aS * mu_f * fabs(aN)));
    }
    if (QUANTUM && !(chi_hi < chi_top)) flags |= kFlagRange;
    if (!(mu_f > 0.0) || !isfinite(mu_f) || !isfinite(s2_f)) flags |= kFlagNonFinite;
    const int64_t k = sp.state_off + i;
    P.st.mu[k] = mu_f;
    P.st.s2[k] = s2_f;
    P.st.S0[k] = S0;
    P.st.g0[k] = g0;
    P.st.thx[k] = thx;
    P.st.thy[k] = thy;
    P.st.cmx[k] = cmx;
}

template <int PREC, bool QUANTUM, bool LOCAL>
__global__ __launch_bounds__(kPhaseBlock) void phase_kernel(BatchParams P,
                                                            const float *__restrict__ env32,
                                                            const double *__restrict__ env64) {
    constexpr bool kTab32 = QUANTUM && PREC != PREC_F64;
    __shared__ __align__(16) float tab32[kTab32 ? kCells32 * kCellVals : 4];
    __shared__ int64_t slot;
    if (kTab32) {
        const float4 *src = reinterpret_cast<const float4 *>(P.rad32);
        float4 *dst = reinterpret_cast<float4 *>(tab32);
        for (int k = threadIdx.x; k < kCells32 * kCellVals / 4; k += blockDim.x) dst[k] = src[k];
        __syncthreads();
    }
    for (;;) {
        const int64_t item = next_item(&P.queue[0], &slot);
        if (item >= P.n_items) break;
        const int s = __builtin_amdgcn_readfirstlane(find_shot(P.shots, P.n_shots, item, false));
        const ShotParams &sp = P.shots[s];
        const int64_t i = (item - sp.item0) * kPhaseBlock + threadIdx.x;
        if (i < sp.n_samples) {
            int flags = 0;
            phase_sample<PREC, QUANTUM, LOCAL>(P, sp, i, env32, env64, tab32, flags);
            if (flags) atomicOr(&P.flags[s], flags);
        }
    }
}

// ===========================================================================
// Deposit kernel: final states -> observables -> histograms and moments
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

__global__ __launch_bounds__(kDepBlock) void deposit_kernel(BatchParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *hist = reinterpret_cast<unsigned long long *>(smem);
    __shared__ int64_t slot;
    __shared__ double red[kDepBlock / 64][P_N];
    __shared__ float redmax[kDepBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (;;) {
        const int64_t item = next_item(&P.queue[1], &slot);
        if (item >= P.n_ditems) break;
        const int s = __builtin_amdgcn_readfirstlane(find_shot(P.shots, P.n_shots, item, true));
        const ShotParams &sp = P.shots[s];
        const ShotOut &so = P.outs[s];
        const int nh_e = sp.n_e + 2, nh_t = sp.n_th + 2, nh = nh_e + nh_t + sp.n_a;
        for (int k = threadIdx.x; k < nh; k += blockDim.x) hist[k] = 0ull;
        __syncthreads();

        double acc[P_N];
#pragma unroll
        for (int m = 0; m < P_N; ++m) acc[m] = 0.0;
        float chimax = 0.0f;
        int flags = 0;
        const int64_t i0 = (item - sp.ditem0) * kDepTile;
        const int64_t i1 = i0 + kDepTile < sp.n_samples ? i0 + kDepTile : sp.n_samples;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
            const int64_t k = sp.state_off + i;
            const double mu_f = P.st.mu[k], s2_f = P.st.s2[k], S0 = P.st.S0[k], g0 = P.st.g0[k];
            const double thx_m = 1e3 * P.st.thx[k], thy_m = 1e3 * P.st.thy[k];
            const float cmx = P.st.cmx[k];
            if (!(mu_f > 0.0) || !isfinite(mu_f) || !isfinite(s2_f)) {
                flags |= kFlagNonFinite;  // also raised by the phase kernel
                continue;
            }
            chimax = fmaxf(chimax, cmx);
            // Sec. 5.2: the direction is kept, the stochastic broadening
            // c_theta sqrt(2/pi) a0,eff sigma_f / gamma_f^2 acts in x
            const double sigf = sqrt(fmax(s2_f, 0.0));
            const double a_eff = sp.a0 * S0;
            const double sigth =
                1e3 * P.c_theta * 0.79788456080286535588 * a_eff * sigf / (mu_f * mu_f);

            deposit_law(mu_f, sigf, P.deposit, P.ksig_bins, sp.e_lo, sp.e_w, sp.n_e, hist);
            deposit_law(thx_m, sigth, P.deposit, P.ksig_bins, sp.th_lo, sp.th_w, sp.n_th,
                        hist + nh_e);
            {
                int ka = (int)floor(S0 * (double)sp.n_a);
                ka = min(max(ka, 0), sp.n_a - 1);
                atomicAdd(&hist[nh_e + nh_t + ka], kOne);
            }
            const double de = mu_f - sp.gamma0;
            acc[P_S1E] += de;
            acc[P_S2E] += fma(de, de, fmax(s2_f, 0.0));
            acc[P_S1X] += thx_m;
            acc[P_S2X] += fma(thx_m, thx_m, sigth * sigth);
            acc[P_S1Y] += thy_m;
            acc[P_S2Y] += thy_m * thy_m;
            acc[P_SAEFF] += a_eff;
            acc[P_SRAD] += 1.0 - mu_f / g0;
            acc[P_SSIGF] += sigf;

            if (so.samples != nullptr && i % so.rec_stride == 0 && i / so.rec_stride < so.rec_n) {
                double *r = so.samples + (i / so.rec_stride) * 11;
                r[0] = mu_f;
                r[1] = s2_f;
                r[2] = thx_m;
                r[3] = thy_m;
                r[4] = sigth;
                r[5] = a_eff;
                r[6] = cmx;
                r[7] = g0;
                r[8] = 0.0;
                r[9] = 0.0;
                r[10] = 0.0;
            }
        }

        // ---- item reduction of moments (fixed order) ----
#pragma unroll
        for (int m = 0; m < P_N; ++m) {
            const double v = wave_sum(acc[m]);
            if (lane == 0) red[wid][m] = v;
        }
        const float wm = wave_max(chimax);
        if (lane == 0) redmax[wid] = wm;
        if (flags) atomicOr(&P.flags[s], flags);
        __syncthreads();
        double *part = P.partials + (size_t)item * kPartials;
        if (threadIdx.x < P_N) {
            double sum = 0.0;
            for (int w = 0; w < kDepBlock / 64; ++w) sum += red[w][threadIdx.x];
            part[threadIdx.x] = sum;
        }
        if (threadIdx.x == 0) {
            float m = 0.0f;
            for (int w = 0; w < kDepBlock / 64; ++w) m = fmaxf(m, redmax[w]);
            part[P_N] = m;
        }
        for (int k = threadIdx.x; k < nh; k += blockDim.x) {
            const unsigned long long v = hist[k];
            if (v) atomicAdd(&P.hist[sp.hist_off + k], v);
        }
        __syncthreads();  // the next item clears the LDS histogram
    }
}

// ===========================================================================
// Finalize: one block per shot, fixed-order reduction of its item partials
// ===========================================================================
__global__ __launch_bounds__(256) void finalize_kernel(BatchParams P) {
    const int s = blockIdx.x;
    const ShotParams &sp = P.shots[s];
    const ShotOut &so = P.outs[s];
    const int64_t nd = (sp.n_samples + kDepTile - 1) / kDepTile;
    __shared__ double sums[kPartials];
    __shared__ double tree[256];
    // each column: thread t sums items t, t + 256, ... then a fixed tree
    for (int m = 0; m < kPartials; ++m) {
        double acc = 0.0;
        for (int64_t b = threadIdx.x; b < nd; b += blockDim.x) {
            const double v = P.partials[(size_t)(sp.ditem0 + b) * kPartials + m];
            acc = m == P_N ? fmax(acc, v) : acc + v;
        }
        tree[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                const double o = tree[threadIdx.x + w];
                tree[threadIdx.x] = m == P_N ? fmax(tree[threadIdx.x], o) : tree[threadIdx.x] + o;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) sums[m] = tree[0];
        __syncthreads();
    }
    const int nh_e = sp.n_e + 2, nh_t = sp.n_th + 2;
    const unsigned long long *H = P.hist + sp.hist_off;
    const double scale = 1.0 / 4294967296.0;
    for (int k = threadIdx.x; k < nh_e; k += blockDim.x) so.energy_hist[k] = (double)H[k] * scale;
    for (int k = threadIdx.x; k < nh_t; k += blockDim.x)
        so.angle_hist[k] = (double)H[nh_e + k] * scale;
    for (int k = threadIdx.x; k < sp.n_a; k += blockDim.x)
        so.a0eff_hist[k] = (double)H[nh_e + nh_t + k] * scale;
    __syncthreads();
    if (threadIdx.x == 0) {
        double *M = so.moments;
        for (int m = 0; m < 16; ++m) M[m] = 0.0;
        const double W = (double)sp.n_samples;
        M[0] = W;
        if (sp.n_samples > 0) {
            const double m1 = sums[P_S1E] / W;
            M[1] = sp.gamma0 + m1;
            M[2] = sqrt(fmax(sums[P_S2E] / W - m1 * m1, 0.0));
            M[3] = sums[P_S1X] / W;
            M[4] = sqrt(sums[P_S2X] / W);
            M[5] = sums[P_S1Y] / W;
            M[6] = sqrt(sums[P_S2Y] / W);
            M[7] = sums[P_SAEFF] / W;
            M[8] = sums[P_N];
            M[9] = sums[P_SRAD] / W;
            M[10] = sums[P_SSIGF] / W;
        }
        const int fl = P.flags[s];
        *so.status = (fl & kFlagNonFinite) ? 4 : ((fl & kFlagRange) ? 6 : 0);
    }
}

// ===========================================================================
// Set-up kernels: envelope x carrier table, zero fill
// ===========================================================================
__global__ void envelope_kernel(double psi_max, double h, int n_steps, int envelope,
                                double omega_tau, float *env32, double *env64) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > 2 * n_steps) return;
    const double psi = fma((double)k, 0.5 * h, -psi_max);
    double f;
    if (envelope == 0) {
        const double u = psi / omega_tau;
        f = exp(-2.0 * 0.69314718055994530942 * u * u);
    } else {
        if (fabs(psi) > omega_tau) {
            f = 0.0;
        } else {
            const double s = sinpi((psi + omega_tau) / (2.0 * omega_tau));
            f = s * s;
        }
    }
    const double e = f * cos(psi);
    env64[k] = e;
    env32[k] = (float)e;
}

__global__ void zero_kernel(unsigned long long *p, size_t n) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x)
        p[k] = 0ull;
}

// ===========================================================================
// Radiation-function tables.
//
// The LCFA photon emission rate per unit energy fraction xi is proportional
// to (1 - xi + 1/(1 - xi)) K_{2/3}(y) - Int_y^inf K_{1/3}, y = 2 xi / (3 chi
// (1 - xi)).  With the integral representations K_nu(y) = Int_0^inf
// exp(-y cosh t) cosh(nu t) dt and Int_y^inf K_{1/3} = Int_0^inf exp(-y cosh t)
// cosh(t/3) / cosh t dt,
//   g(chi) = sqrt3/(2 pi chi^2) I_0,   h(chi) = 24/(55 pi chi^3) J_0,
//   I_k = Int_0^1 dxi xi Int_0^inf dt (y cosh t)^k e^{-y cosh t}
//         [w cosh(2t/3) - cosh(t/3)/cosh t],   J_0 likewise with xi^2,
// where chi d/dchi acting on e^{-y cosh t} brings down y cosh t, so that
//   chi g' = C (I_1 - 2 I_0),  chi^2 g'' = C (I_2 - 6 I_1 + 6 I_0),  C = sqrt3/(2 pi chi^2).
// The t integrals depend on y only and are tabulated once on a y = e^v
// grid; the xi integral is taken over v with xi = 3 chi y / (2 + 3 chi y).
// Both rules are trapezoidal on doubly-exponentially decaying integrands.
// Each table cell stores the cubic through the values at four Chebyshev
// points of its local coordinate.
// ===========================================================================
constexpr double kVLo = -32.25;  // y from ~1e-14
constexpr double kVHi = 4.125;   // to ~62
constexpr double kDv = 1.0 / 16.0;
constexpr int kNY = (int)((kVHi - kVLo) / kDv) + 1;
constexpr double kDt = 1.0 / 16.0;
constexpr int kYVals = 8;     // per y node: P_0..P_2, Q_0..Q_2, P_3, Q_3
constexpr int kNodeVals = 6;  // per chi node: g, chi g', chi^2 g'', h, chi^3 g''', chi h'

__global__ void rad_y_kernel(double *yf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNY) return;
    const double y = exp(kVLo + i * kDv);
    const double tmax = acosh(fmax(60.0 / y, 1.0)) + kDt;
    const int nt = (int)ceil(tmax / kDt);
    double P0 = 0, P1 = 0, P2 = 0, P3 = 0, Q0 = 0, Q1 = 0, Q2 = 0, Q3 = 0;
    for (int m = 0; m <= nt; ++m) {
        const double t = m * kDt;
        const double c = cosh(t);
        const double u = y * c;
        const double e = exp(-u) * (m == 0 ? 0.5 : 1.0);
        const double p = e * cosh(t * (2.0 / 3.0));
        const double q = e * cosh(t * (1.0 / 3.0)) / c;
        P0 += p;
        P1 += u * p;
        P2 += u * u * p;
        P3 += u * u * u * p;
        Q0 += q;
        Q1 += u * q;
        Q2 += u * u * q;
        Q3 += u * u * u * q;
    }
    double *o = yf + kYVals * i;
    o[0] = P0 * kDt;
    o[1] = P1 * kDt;
    o[2] = P2 * kDt;
    o[3] = Q0 * kDt;
    o[4] = Q1 * kDt;
    o[5] = Q2 * kDt;
    o[6] = P3 * kDt;
    o[7] = Q3 * kDt;
}

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

// vals[node][6] at the four Chebyshev nodes of every cell, cells of the
// FP32 table first, then those of the FP64 table.  The chi dependence of the
// moments I_k (weight (y cosh t)^k) and J_k sits in y cosh t, which scales
// as 1/chi at fixed chi y, so chi d/dchi maps I_k to I_{k+1} - k I_k; with
// g = C I_0 (C ~ chi^-2) and h = C' J_0 (C' ~ chi^-3) that gives
//   chi g' = C (I_1 - 2 I_0),       chi^2 g'' = C (I_2 - 6 I_1 + 6 I_0),
//   chi^3 g''' = C (I_3 - 12 I_2 + 36 I_1 - 24 I_0),   chi h' = C' (J_1 - 3 J_0).
__global__ void rad_node_kernel(const double *yf, double *vals) {
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = 4 * (kCells32 + kCells64);
    if (node >= total) return;
    const int cell_all = node >> 2, m = node & 3;
    const bool t32 = cell_all < kCells32;
    const int cell = t32 ? cell_all : cell_all - kCells32;
    const double chi = cell_chi(cell, cheb_node(m), t32 ? kSB32 : kSB64);
    double I0 = 0, I1 = 0, I2 = 0, I3 = 0, J0 = 0, J1 = 0;
    for (int i = 0; i < kNY; ++i) {
        const double y = exp(kVLo + i * kDv);
        const double q = 2.0 + 3.0 * chi * y;
        const double xi = 3.0 * chi * y / q;
        const double w = 2.0 / q + 0.5 * q;
        const double base = xi * (6.0 * chi / (q * q)) * y;  // xi dxi/dy dy/dv
        const double *f = yf + kYVals * i;
        const double b0 = base * (w * f[0] - f[3]);
        const double b1 = base * (w * f[1] - f[4]);
        I0 += b0;
        I1 += b1;
        I2 += base * (w * f[2] - f[5]);
        I3 += base * (w * f[6] - f[7]);
        J0 += xi * b0;
        J1 += xi * b1;
    }
    I0 *= kDv;
    I1 *= kDv;
    I2 *= kDv;
    I3 *= kDv;
    J0 *= kDv;
    J1 *= kDv;
    const double C = 1.7320508075688772935 / (2.0 * 3.14159265358979323846 * chi * chi);
    const double Cp = 24.0 / (55.0 * 3.14159265358979323846 * chi * chi * chi);
    double *o = vals + kNodeVals * node;
    o[0] = C * I0;
    o[1] = C * (I1 - 2.0 * I0);
    o[2] = C * (I2 - 6.0 * I1 + 6.0 * I0);
    o[3] = Cp * J0;
    o[4] = C * (I3 - 12.0 * I2 + 36.0 * I1 - 24.0 * I0);
    o[5] = Cp * (J1 - 3.0 * J0);
}

// Cubic through the four node values of each cell, in monomials of t.  The
// forward tables take g, chi g', chi^2 g'', h; the derivative tables all six
// functions (same order as the node values).
__global__ void rad_coef_kernel(const double *vals, float *rad32, double *rad64, float *rad32d,
                                double *rad64d) {
    const int cell_all = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell_all >= kCells32 + kCells64) return;
    double tn[4];
    for (int m = 0; m < 4; ++m) tn[m] = cheb_node(m);
    double coef[kNodeVals][4] = {};
    for (int m = 0; m < 4; ++m) {
        double r[3];
        int k = 0;
        double den = 1.0;
        for (int n = 0; n < 4; ++n)
            if (n != m) {
                r[k++] = tn[n];
                den *= tn[m] - tn[n];
            }
        // (t - r0)(t - r1)(t - r2) / den
        const double l3 = 1.0 / den;
        const double l2 = -(r[0] + r[1] + r[2]) / den;
        const double l1 = (r[0] * r[1] + r[0] * r[2] + r[1] * r[2]) / den;
        const double l0 = -(r[0] * r[1] * r[2]) / den;
        for (int f = 0; f < kNodeVals; ++f) {
            const double v = vals[kNodeVals * (4 * cell_all + m) + f];
            coef[f][0] += v * l0;
            coef[f][1] += v * l1;
            coef[f][2] += v * l2;
            coef[f][3] += v * l3;
        }
    }
    if (cell_all < kCells32) {
        // function-major: rad32[(f * kCells32 + cell) * 4 + power], holding the
        // drift combinations g, 2g + chi g', g + 2 chi g' + chi^2 g''/2, h
        for (int c = 0; c < 4; ++c) {
            const double mix[4] = {coef[0][c], 2.0 * coef[0][c] + coef[1][c],
                                   coef[0][c] + 2.0 * coef[1][c] + 0.5 * coef[2][c], coef[3][c]};
            for (int f = 0; f < 4; ++f) rad32[(f * kCells32 + cell_all) * 4 + c] = (float)mix[f];
            // g, E1 = 2g + G1, E2 = 2g + 4 G1 + G2, E3 = 6 G1 + 6 G2 + G3, h, H1
            const double jm[kDerivFuncs] = {
                coef[0][c], 2.0 * coef[0][c] + coef[1][c],
                2.0 * coef[0][c] + 4.0 * coef[1][c] + coef[2][c],
                6.0 * (coef[1][c] + coef[2][c]) + coef[4][c], coef[3][c], coef[5][c]};
            for (int f = 0; f < kDerivFuncs; ++f)
                rad32d[(f * kCells32 + cell_all) * 4 + c] = (float)jm[f];
        }
    } else {
        const int cell = cell_all - kCells32;
        for (int f = 0; f < 4; ++f)
            for (int c = 0; c < 4; ++c) rad64[(size_t)cell * kCellVals + 4 * f + c] = coef[f][c];
        for (int f = 0; f < kDerivFuncs; ++f)
            for (int c = 0; c < 4; ++c)
                rad64d[(size_t)cell * (4 * kDerivFuncs) + 4 * f + c] = coef[f][c];
    }
}

__global__ void rad_eval_kernel(const float *rad32, const double *rad64, int prec, int64_t n,
                                const double *chi, double *out, int *flags) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int fl = (chi[k] < (double)(1 << (kEMax + 1))) ? 0 : kFlagRange;
    if (prec == 0) {
        float T1, T2, T3, h;
        rad_eval32(rad32, (float)chi[k], T1, T2, T3, h);
        const double g = T1, G1 = (double)T2 - 2.0 * T1;
        out[4 * k] = g;
        out[4 * k + 1] = G1;
        out[4 * k + 2] = 2.0 * ((double)T3 - g - 2.0 * G1);
        out[4 * k + 3] = h;
    } else {
        double g, G1, G2, h;
        rad_eval64(rad64, chi[k], g, G1, G2, h);
        out[4 * k] = g;
        out[4 * k + 1] = G1;
        out[4 * k + 2] = G2;
        out[4 * k + 3] = h;
    }
    if (fl) atomicOr(flags, fl);
}

// ===========================================================================
// Adjoint: derivatives of a weighted sum of the energy histogram,
//   L = sum_k w_k H_k   (w = dL/dH from the caller),
// with respect to the eight shot parameters (a0, W0, x and y offsets, delay,
// gamma0, sigma_gamma, divergence).  Every sample's trajectory is integrated
// again together with its tangents: forward-mode derivatives of the discrete
// RK4 map itself, so no trajectory is stored.  The final tangents are
// contracted with the sample's sensitivities dL/dmu_f and dL/dsig2_f, taken
// from its deposited law; the sums over samples are reduced per work item and
// per shot in a fixed order.
//
// Tangent directions.  The sample state depends on the parameters through
// the amplitude a(psi) = a0 S(x_e, y_e, z_e) f(psi) cos psi along the path
// (Sec. 2, eq. a0eff) and through the initial energy.  gamma0 and
// sigma_gamma only enter the initial energy (mu_0 = gamma0 + sigma_gamma n3),
// so the sigma_gamma tangent is n3 times the gamma0 tangent.  With the
// amplitude frozen at a0,eff every amplitude direction forces the system
// with a multiple of S0 f cos psi, so one tangent serves a0 and the four
// geometric parameters.
// ===========================================================================
// Radiation functions in the combinations the Jacobian uses:
//   g,  E1 = 2g + G1,  E2 = 2g + 4 G1 + G2,  E3 = 6 G1 + 6 G2 + G3,  h,  H1
// (G1 = chi g', G2 = chi^2 g'', G3 = chi^3 g''', H1 = chi h').  The FP32
// derivative table stores these combinations; the FP64 one the plain
// functions.
template <class T>
struct RadJ {
    T g, E1, E2, E3, h, H1;
};

// One FP32 derivative-table cell in registers (see RadCell32).
struct RadCell6 {
    float4 q[kDerivFuncs];
    float tw, ts;
};

__device__ __forceinline__ void rad6_lookup32(const float *__restrict__ tab, float chi,
                                              RadCell6 &cell) {
    const uint32_t b = __float_as_uint(chi);
    int c = (int)(b >> (23 - kSB32)) - ((127 + kEMin) << kSB32) + 1;
    float tw = __uint_as_float((uint32_t)(254 + kSB32 - (int)(b >> 23)) << 23);
    float ts = -__uint_as_float(b & ~((1u << (23 - kSB32)) - 1)) * tw;
    if (c < 1) {  // chi < 2^kEMin: the first cell, linear in chi
        c = 0;
        tw = 0x1p20f;
        ts = 0.0f;
    }
    if (c > kCells32 - 1) {  // beyond the table (reported by the caller)
        c = kCells32 - 1;
        tw = 0.0f;
        ts = 1.0f;
    }
    const float4 *T = reinterpret_cast<const float4 *>(tab);
#pragma unroll
    for (int f = 0; f < kDerivFuncs; ++f) cell.q[f] = T[f * kCells32 + c];
    cell.tw = tw;
    cell.ts = ts;
}

__device__ __forceinline__ RadJ<float> rad6_cell_eval(const RadCell6 &cell, float chi) {
    const float t = fmaf(chi, cell.tw, cell.ts);
    float v[kDerivFuncs];
#pragma unroll
    for (int f = 0; f < kDerivFuncs; ++f) {
        const float4 &q = cell.q[f];
        v[f] = fmaf(t, fmaf(t, fmaf(t, q.w, q.z), q.y), q.x);
    }
    return RadJ<float>{v[0], v[1], v[2], v[3], v[4], v[5]};
}

// FP64 table, cell-major [cell][g, G1, G2, h, G3, H1][power]: the plain
// functions, combined here.
__device__ __forceinline__ void rad6_plain64(const double *__restrict__ tab, double chi,
                                             double v[kDerivFuncs]) {
    const uint64_t b = (uint64_t)__double_as_longlong(chi);
    int64_t c = (int64_t)(b >> (52 - kSB64)) - ((int64_t)(1023 + kEMin) << kSB64) + 1;
    double t = __longlong_as_double((long long)(((b & ((1ull << (52 - kSB64)) - 1)) << kSB64) |
                                                0x3ff0000000000000ull)) - 1.0;
    if (c < 1) {
        c = 0;
        t = chi * 0x1p20;
    }
    c = c < kCells64 - 1 ? c : kCells64 - 1;
    const double *q = tab + (size_t)c * (4 * kDerivFuncs);
#pragma unroll
    for (int f = 0; f < kDerivFuncs; ++f)
        v[f] = fma(t, fma(t, fma(t, q[4 * f + 3], q[4 * f + 2]), q[4 * f + 1]), q[4 * f]);
}

__device__ __forceinline__ RadJ<double> radj_eval64(const double *__restrict__ tab, double chi) {
    double v[kDerivFuncs];
    rad6_plain64(tab, chi, v);
    const double g = v[0], G1 = v[1], G2 = v[2], h = v[3], G3 = v[4], H1 = v[5];
    return RadJ<double>{g, fma(2.0, g, G1), fma(4.0, G1, fma(2.0, g, G2)), fma(6.0, G1 + G2, G3),
                        h, H1};
}

// Where a stage takes its radiation functions from.  FP32: the LDS table,
// read at stages 2 and 4 only -- stage 3 reuses stage 2's cell and the next
// step's stage 1 reuses stage 4's (as in the forward phase loop).  FP64: the
// global table at every stage.
template <class T>
struct RadSrc;
template <>
struct RadSrc<float> {
    const float *tab;
    RadCell6 carry, mid;
    __device__ __forceinline__ void init(float chi) { rad6_lookup32(tab, chi, carry); }
    __device__ __forceinline__ RadJ<float> s1(float chi) { return rad6_cell_eval(carry, chi); }
    __device__ __forceinline__ RadJ<float> s2(float chi) {
        rad6_lookup32(tab, chi, mid);
        return rad6_cell_eval(mid, chi);
    }
    __device__ __forceinline__ RadJ<float> s3(float chi) { return rad6_cell_eval(mid, chi); }
    __device__ __forceinline__ RadJ<float> s4(float chi) {
        rad6_lookup32(tab, chi, carry);
        return rad6_cell_eval(carry, chi);
    }
};
template <>
struct RadSrc<double> {
    const double *tab;
    __device__ __forceinline__ void init(double) {}
    __device__ __forceinline__ RadJ<double> s1(double chi) { return radj_eval64(tab, chi); }
    __device__ __forceinline__ RadJ<double> s2(double chi) { return radj_eval64(tab, chi); }
    __device__ __forceinline__ RadJ<double> s3(double chi) { return radj_eval64(tab, chi); }
    __device__ __forceinline__ RadJ<double> s4(double chi) { return radj_eval64(tab, chi); }
};

__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Right-hand side f = (dmu/dpsi, dsig2/dpsi) of the moment system and its
// partial derivatives with respect to mu, sig2 and the amplitude a.  With
// chi d/dchi written D (D g = G1, D G1 = G1 + G2, D G2 = 2 G2 + G3,
// D h = H1) and u = K a^2:
//   f_mu  = -u (mu^2 g + sig2 E2 / 2),      f_s2 = -2 u mu sig2 E1 + C_D |a|^3 mu^4 h,
//   d f_mu / d mu   = -u (mu E1 + sig2 E3 / (2 mu)),
//   d f_mu / d sig2 = -u E2 / 2,
//   d f_s2 / d mu   = -2 u sig2 E2 + C_D |a|^3 mu^3 (4 h + H1),
//   d f_s2 / d sig2 = -2 u mu E1,
//   d f_mu / d a    = -K a (mu^2 E1 + sig2 (E2 + E3 / 2)),
//   d f_s2 / d a    = -2 K a mu sig2 (E1 + E2) + C_D a |a| mu^4 (3 h + H1).
// Classical model (g = 1, no diffusion; sig2 stays 0): f_mu = -u mu^2.
template <class T>
struct Jac {
    T fm, fs;  // f
    T mm, ms, sm, ss;  // d f / d (mu, sig2)
    T ma, sa;  // d f / d a
};

// Per-stage amplitude constants: a, K a, C_D a |a|, 2 |a| / a_S.
template <class T>
struct StageAmp {
    T a, Ka, cda, chi_per_mu;
    __device__ __forceinline__ StageAmp(T a_, const Phys<T> &ph)
        : a(a_), Ka(ph.K * a_), cda(ph.CD * a_ * fabs(a_)), chi_per_mu(ph.two_over_aS * fabs(a_)) {}
};

template <class T>
__device__ __forceinline__ Jac<T> jac_quantum(T mu, T s2, const StageAmp<T> &A, const RadJ<T> &r) {
    Jac<T> J;
    const T u = A.Ka * A.a;
    const T mu2 = mu * mu;
    const T hs = T(0.5) * s2;
    const T c3 = A.cda * mu2;        // C_D a |a| mu^2
    const T c3a = c3 * mu * A.a;     // C_D |a|^3 mu^3
    const T u2 = T(-2) * u;
    J.fm = -u * fma(mu2, r.g, hs * r.E2);
    J.fs = fma(u2 * mu * s2, r.E1, c3a * mu * r.h);
    J.mm = -u * fma(mu, r.E1, hs * r.E3 * recip(mu));
    J.ms = T(-0.5) * u * r.E2;
    J.sm = fma(u2 * s2, r.E2, c3a * fma(T(4), r.h, r.H1));
    J.ss = u2 * mu * r.E1;
    J.ma = -A.Ka * fma(mu2, r.E1, s2 * fma(T(0.5), r.E3, r.E2));
    J.sa = fma(T(-2) * A.Ka * mu * s2, r.E1 + r.E2, c3 * mu2 * fma(T(3), r.h, r.H1));
    return J;
}

template <class T>
__device__ __forceinline__ Jac<T> jac_classical(T mu, const StageAmp<T> &A) {
    Jac<T> J;
    const T u = A.Ka * A.a;
    J.fm = -u * mu * mu;
    J.mm = T(-2) * u * mu;
    J.ma = T(-2) * A.Ka * mu * mu;
    J.fs = J.ms = J.sm = J.ss = J.sa = T(0);
    return J;
}

// 2x2 matrices [[a, b], [c, d]] and 2-vectors acting on (mu, sig2); in the
// classical model only the mu entries are used.
template <class T>
struct Mat2 {
    T a, b, c, d;
};
template <class T>
struct Vec2 {
    T x, y;
};

// K (I + s M) = K + s K M
template <class T, bool Q>
__device__ __forceinline__ Mat2<T> kism(const Jac<T> &K, T s, const Mat2<T> &M) {
    Mat2<T> R;
    if (Q) {
        R.a = fma(s, fma(K.mm, M.a, K.ms * M.c), K.mm);
        R.b = fma(s, fma(K.mm, M.b, K.ms * M.d), K.ms);
        R.c = fma(s, fma(K.sm, M.a, K.ss * M.c), K.sm);
        R.d = fma(s, fma(K.sm, M.b, K.ss * M.d), K.ss);
    } else {
        R.a = fma(s, K.mm * M.a, K.mm);
        R.b = R.c = R.d = T(0);
    }
    return R;
}

// s K v
template <class T, bool Q>
__device__ __forceinline__ Vec2<T> skv(const Jac<T> &K, T s, const Vec2<T> &v) {
    Vec2<T> r;
    if (Q) {
        r.x = s * fma(K.mm, v.x, K.ms * v.y);
        r.y = s * fma(K.sm, v.x, K.ss * v.y);
    } else {
        r.x = s * K.mm * v.x;
        r.y = T(0);
    }
    return r;
}

// One RK4 step of (mu, sig2), linearised.  The tangent of any direction obeys
//   dk1 = K1 V + g1 d1,            dk2 = K2 (V + h/2 dk1) + g2 dh,
//   dk3 = K3 (V + h/2 dk2) + g3 dh, dk4 = K4 (V + h dk3) + g4 d4,
//   V' = V + h/6 (dk1 + 2 dk2 + 2 dk3 + dk4),
// with K_s = d f / d(mu, sig2) and g_s = d f / d a at stage s, and d1, dh, d4
// the direction's amplitude derivatives at psi_j, psi_j + h/2, psi_j + h.
// That map is linear, V' = A V + P1 d1 + Ph dh + P4 d4, and A, P1, Ph, P4 are
// shared by all directions, so they are formed once per step.
template <class T, bool Q>
struct StepLin {
    Mat2<T> A;
    Vec2<T> P1, Ph, P4;
    T dmu, ds2;  // the state increment
};

template <class T, bool Q>
__device__ __forceinline__ StepLin<T, Q> rk4_linear(T mu, T s2, const StageAmp<T> &A1,
                                                    const StageAmp<T> &Ah, const StageAmp<T> &A4,
                                                    T h, RadSrc<T> &rad, T &chi_hi) {
    const T hh = T(0.5) * h, h6 = h * T(1.0 / 6.0);
    StepLin<T, Q> L;
    // stage 1
    Jac<T> K1;
    if (Q) {
        const T chi = A1.chi_per_mu * mu;
        chi_hi = fmax(chi_hi, chi);
        K1 = jac_quantum(mu, s2, A1, rad.s1(chi));
    } else {
        K1 = jac_classical(mu, A1);
    }
    const Vec2<T> g1{K1.ma, K1.sa};
    // stage 2
    const T m2 = fma(hh, K1.fm, mu), s22 = fma(hh, K1.fs, s2);
    Jac<T> K2;
    if (Q) {
        const T chi = Ah.chi_per_mu * m2;
        chi_hi = fmax(chi_hi, chi);
        K2 = jac_quantum(m2, s22, Ah, rad.s2(chi));
    } else {
        K2 = jac_classical(m2, Ah);
    }
    const Mat2<T> M1{K1.mm, K1.ms, K1.sm, K1.ss};
    const Mat2<T> M2 = kism<T, Q>(K2, hh, M1);
    const Vec2<T> e21 = skv<T, Q>(K2, hh, g1);
    const Vec2<T> g2{K2.ma, K2.sa};
    // stage 3
    const T m3 = fma(hh, K2.fm, mu), s23 = fma(hh, K2.fs, s2);
    Jac<T> K3;
    if (Q) {
        const T chi = Ah.chi_per_mu * m3;
        chi_hi = fmax(chi_hi, chi);
        K3 = jac_quantum(m3, s23, Ah, rad.s3(chi));
    } else {
        K3 = jac_classical(m3, Ah);
    }
    const Mat2<T> M3 = kism<T, Q>(K3, hh, M2);
    const Vec2<T> e31 = skv<T, Q>(K3, hh, e21);
    Vec2<T> e3h = skv<T, Q>(K3, hh, g2);
    e3h.x += K3.ma;
    e3h.y += K3.sa;
    // stage 4
    const T m4 = fma(h, K3.fm, mu), s24 = fma(h, K3.fs, s2);
    Jac<T> K4;
    if (Q) {
        const T chi = A4.chi_per_mu * m4;
        chi_hi = fmax(chi_hi, chi);
        K4 = jac_quantum(m4, s24, A4, rad.s4(chi));
    } else {
        K4 = jac_classical(m4, A4);
    }
    const Mat2<T> M4 = kism<T, Q>(K4, h, M3);
    const Vec2<T> e41 = skv<T, Q>(K4, h, e31);
    const Vec2<T> e4h = skv<T, Q>(K4, h, e3h);
    // assemble
    L.A.a = fma(h6, M1.a + T(2) * (M2.a + M3.a) + M4.a, T(1));
    L.A.b = h6 * (M1.b + T(2) * (M2.b + M3.b) + M4.b);
    L.A.c = h6 * (M1.c + T(2) * (M2.c + M3.c) + M4.c);
    L.A.d = fma(h6, M1.d + T(2) * (M2.d + M3.d) + M4.d, T(1));
    L.P1.x = h6 * (g1.x + T(2) * (e21.x + e31.x) + e41.x);
    L.P1.y = h6 * (g1.y + T(2) * (e21.y + e31.y) + e41.y);
    L.Ph.x = h6 * (T(2) * (g2.x + e3h.x) + e4h.x);
    L.Ph.y = h6 * (T(2) * (g2.y + e3h.y) + e4h.y);
    L.P4.x = h6 * K4.ma;
    L.P4.y = h6 * K4.sa;
    L.dmu = h6 * (K1.fm + T(2) * (K2.fm + K3.fm) + K4.fm);
    L.ds2 = h6 * (K1.fs + T(2) * (K2.fs + K3.fs) + K4.fs);
    return L;
}

// Spatial factor of eq. a0eff and its logarithmic derivatives with respect to
// the sample position (x, y, z) and the spot size W0:
//   ln S = -p - ln(q)/2,  p = (x^2 + y^2) / (W0^2 q),  q = 1 + (z / zR)^2,
//   d/dx = -2 x / (W0^2 q),  d/dz = 2 (z / zR^2) (p - 1/2) / q,
//   d/dW0 = (2 / W0) (p - 2 (z/zR)^2 (p - 1/2) / q)   (zR = pi W0^2 / lambda).
template <class T>
struct SpD {
    T S, Lx, Ly, Lz, Lw;
};

__device__ __forceinline__ SpD<float> spatial_d(float x, float y, float z, float inv_w0sq,
                                                float inv_zR, float inv_w0) {
    const float zz = z * inv_zR;
    const float q = fmaf(zz, zz, 1.0f);
    const float rq = __builtin_amdgcn_rsqf(q);
    const float iq = rq * rq;
    const float p = fmaf(x, x, y * y) * inv_w0sq * iq;
    SpD<float> r;
    r.S = __builtin_amdgcn_exp2f(-1.4426950408889634f * p) * rq;
    const float m = -2.0f * inv_w0sq * iq;
    r.Lx = m * x;
    r.Ly = m * y;
    const float B = iq * (p - 0.5f);
    r.Lz = 2.0f * zz * inv_zR * B;
    r.Lw = 2.0f * inv_w0 * fmaf(-2.0f * zz * zz, B, p);
    return r;
}

__device__ __forceinline__ SpD<double> spatial_d(double x, double y, double z, double inv_w0sq,
                                                 double inv_zR, double inv_w0) {
    const double zz = z * inv_zR;
    const double q = fma(zz, zz, 1.0);
    const double iq = 1.0 / q;
    const double p = fma(x, x, y * y) * inv_w0sq * iq;
    SpD<double> r;
    r.S = exp(-p) * sqrt(iq);
    const double m = -2.0 * inv_w0sq * iq;
    r.Lx = m * x;
    r.Ly = m * y;
    const double B = iq * (p - 0.5);
    r.Lz = 2.0 * zz * inv_zR * B;
    r.Lw = 2.0 * inv_w0 * fma(-2.0 * zz * zz, B, p);
    return r;
}

// Directions of the local-amplitude tangents: a0, W0, x offset, y offset,
// delay, gamma0, divergence.
constexpr int kDirLocal = 7;
constexpr int kDirA0eff = 2;  // a0 (all amplitude directions), gamma0

// Geometry of one sample in the adjoint's precision.
template <class T>
struct AdjPath {
    T xc, yc, thx, thy, zstar, hz;     // hz = z / 2
    T dthx, dthy;                      // d theta / d div_mrad = 1e-3 n4, 1e-3 n5
    T inv_w0sq, inv_zR, inv_w0, a0, zfac;  // zfac = d z* / d delay = c / 2
    // amplitude without the carrier and its derivative in each direction
    __device__ __forceinline__ void amp(T ell, T fc, T &a, T *da) const {
        const SpD<T> d = spatial_d(fma(thx, ell, xc), fma(thy, ell, yc), zstar - ell, inv_w0sq,
                                   inv_zR, inv_w0);
        const T Sf = d.S * fc;
        a = a0 * Sf;
        da[0] = Sf;
        da[1] = a * d.Lw;
        da[2] = a * d.Lx;
        da[3] = a * d.Ly;
        da[4] = a * zfac * d.Lz;
        da[5] = T(0);
        da[6] = a * (hz + ell) * fma(dthx, d.Lx, dthy * d.Ly);
    }
};

// Sensitivities of one sample's share of L = sum_k w_k H_k to the centre v
// and the variance sig2 of its energy law.  Writing F for the law's CDF and
// e_j = lo + j width (j = 0..n) for the bin edges, the sample adds F(e_0) to
// the underflow, F(e_{k+1}) - F(e_k) to bin k and 1 - F(e_n) to the overflow,
// so its share is sum_j c_j F(e_j) + w_over with c_j = w_{j-1} - w_j
// (w_{-1} = w_under, w_n = w_over).  For the three laws (with t = e_j - v):
//   Gaussian N(v, s^2):  dF/dv = -phi(t/s)/s,          dF/ds = -(t/s) phi(t/s)/s;
//   box of width b:      dF/dv = -1/b for |t| < b/2,   no s;
//   box (x) N(0, s^2):   dF/dv = -(Phi((t + b/2)/s) - Phi((t - b/2)/s)) / b,
//                        dF/ds = (phi((t + b/2)/s) - phi((t - b/2)/s)) / b.
// Edges beyond 9 standard deviations add nothing at FP64 precision.
__device__ __forceinline__ double phi_pdf(double z) {
    return 0.39894228040143267794 * exp(-0.5 * z * z);
}

__device__ __forceinline__ double phi_diff(double zp, double zm) {  // Phi(zp) - Phi(zm), zp > zm
    const double r = 0.70710678118654752440;
    if (zm > 0.0) return 0.5 * (erfc(zm * r) - erfc(zp * r));
    if (zp < 0.0) return 0.5 * (erfc(-zp * r) - erfc(-zm * r));
    return 1.0 - 0.5 * (erfc(zp * r) + erfc(-zm * r));
}

__device__ void law_sensitivity(double v, double s2, int dep, double ksig, double lo, double wb,
                                int n, const double *__restrict__ W, double &lv, double &ls2) {
    lv = 0.0;
    ls2 = 0.0;
    const double s = sqrt(fmax(s2, 0.0));
    const double half = 0.5 * wb;
    int mode;
    double se = s, dse = 0.0;  // law width and d se / d sig2
    if (dep == 2) {            // GAUSS
        const double ks = ksig * wb;
        se = sqrt(s * s + ks * ks);
        mode = se > 0.0 ? 2 : 0;
        if (s2 > 0.0) dse = 0.5 / se;
    } else if (dep == 1) {  // CIC
        mode = s > 0.0 ? 3 : 1;
        if (s > 0.0) dse = 0.5 / s;
    } else {
        mode = s > 0.0 ? 2 : 0;
        if (s > 0.0) dse = 0.5 / s;
    }
    if (mode == 0) return;
    const double reach = mode == 1 ? half : (mode == 2 ? 9.0 * se : 9.0 * se + half);
    const int ja = (int)fmin(fmax(ceil((v - reach - lo) / wb), 0.0), (double)n + 1.0);
    const int jb = (int)fmin(fmax(floor((v + reach - lo) / wb), -1.0), (double)n);
    const double inv_se = mode >= 2 ? 1.0 / se : 0.0;
    double sv = 0.0, ss = 0.0;
    for (int j = ja; j <= jb; ++j) {
        const double wl = j == 0 ? W[n] : W[j - 1];
        const double wr = j == n ? W[n + 1] : W[j];
        const double c = wl - wr;
        if (c == 0.0) continue;
        const double t = fma((double)j, wb, lo) - v;
        double p, q = 0.0;
        if (mode == 1) {
            p = fabs(t) < half ? 1.0 / wb : 0.0;
        } else if (mode == 2) {
            const double z = t * inv_se;
            const double f = phi_pdf(z) * inv_se;
            p = f;
            q = -z * f;
        } else {
            const double zp = (t + half) * inv_se, zm = (t - half) * inv_se;
            p = phi_diff(zp, zm) / wb;
            q = (phi_pdf(zp) - phi_pdf(zm)) / wb;
        }
        sv = fma(c, p, sv);
        ss = fma(c, q, ss);
    }
    lv = -sv;
    ls2 = ss * dse;
}

// Final state of one sample and its derivatives along the eight parameters
// (order of the grad outputs: a0, W0, x offset, y offset, delay, gamma0,
// sigma_gamma, divergence).
struct SampleTangent {
    double mu, s2;
    double dmu[kGradParams], ds2[kGradParams];
    double S0, g0, thx, thy;
    float cmx;
};

// One sample: trajectory, tangents, and the chain to the eight parameters.
template <int PREC, bool QUANTUM, bool LOCAL>
__device__ __forceinline__ void tangent_sample(const BatchParams &P, const ShotParams &sp,
                                               int64_t i, const float *__restrict__ env32,
                                               const double *__restrict__ env64,
                                               const float *tab32, SampleTangent &o,
                                               int &flags) {
    using T = typename std::conditional<PREC == PREC_F64, double, float>::type;
    constexpr int ND = LOCAL ? kDirLocal : kDirA0eff;
    constexpr int GD = LOCAL ? 5 : 1;  // the gamma0 direction: no amplitude forcing
    constexpr double kHalfC = 0.5 * 0.299792458;  // d z* / d delay [um/fs]
    const int N = P.n_steps;
    RadSrc<T> rad;
    if constexpr (PREC == PREC_F64)
        rad.tab = P.rad64d;
    else
        rad.tab = tab32;
    const T *env;
    if constexpr (PREC == PREC_F64)
        env = env64;
    else
        env = env32;
    Phys<T> ph;
    ph.K = (T)P.K;
    ph.CD = (T)P.CD;
    ph.two_over_aS = (T)P.two_over_aS;
    const float chi_top = (float)(1 << (kEMax + 1));

    // ---- sample and geometry (FP64) ----
    double nrm[6];
    sample_normals((uint32_t)i, (uint32_t)sp.shot_word, P.key0, P.key1, nrm);
    const double x = fma(sp.sigma_r, nrm[0], sp.x_off);
    const double y = fma(sp.sigma_r, nrm[1], sp.y_off);
    const double z = sp.sigma_z * nrm[2];
    const double g0 = fma(sp.sigma_gamma, nrm[3], sp.gamma0);
    const double thx = sp.div_rad * nrm[4];
    const double thy = sp.div_rad * nrm[5];
    const double inv_w0 = sqrt(sp.inv_w0sq);
    const double xc = fma(thx, 0.5 * z, x), yc = fma(thy, 0.5 * z, y);
    const double zstar = fma(0.5, z, sp.z_delay);
    const SpD<double> d0 = spatial_d(xc, yc, zstar, sp.inv_w0sq, sp.inv_zR, inv_w0);

    AdjPath<T> pth;
    pth.xc = (T)xc;
    pth.yc = (T)yc;
    pth.thx = (T)thx;
    pth.thy = (T)thy;
    pth.zstar = (T)zstar;
    pth.hz = (T)(0.5 * z);
    pth.dthx = (T)(1e-3 * nrm[4]);
    pth.dthy = (T)(1e-3 * nrm[5]);
    pth.inv_w0sq = (T)sp.inv_w0sq;
    pth.inv_zR = (T)sp.inv_zR;
    pth.inv_w0 = (T)inv_w0;
    pth.a0 = (T)sp.a0;
    pth.zfac = (T)kHalfC;
    const T S0 = (T)d0.S;
    const T ell_per_psi = (T)P.ell_per_psi;
    const T h = (T)P.h;
    const T psi0 = (T)(-P.psi_max);

    T vm[ND], vs[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) vm[d] = vs[d] = T(0);
    vm[GD] = T(1);  // d mu_0 / d gamma0

    T mu = (T)g0, mu_lo = T(0), s2 = T(0), s2_lo = T(0);
    double g0_rest = 0.0;
    if constexpr (PREC != PREC_F64) {
        mu_lo = (T)(g0 - (double)mu);
        g0_rest = (g0 - (double)mu) - (double)mu_lo;
    }
    T chi_hi = T(0);
    float cmx = 0.0f;  // largest chi at a step start
    T a1, da1[ND];
    if (LOCAL) {
        pth.amp(psi0 * ell_per_psi, env[0], a1, da1);
    } else {
        const T Sf = S0 * env[0];
        a1 = pth.a0 * Sf;
        da1[0] = Sf;
        da1[1] = T(0);
    }
    StageAmp<T> A1(a1, ph);
    if (QUANTUM) rad.init(A1.chi_per_mu * mu);
    for (int j = 0; j < N; ++j) {
        const T psi = fma((T)j, h, psi0);
        cmx = fmaxf(cmx, (float)(A1.chi_per_mu * mu));
        T ah, a4, dah[ND], da4[ND];
        if (LOCAL) {
            pth.amp(fma(T(0.5), h, psi) * ell_per_psi, env[2 * j + 1], ah, dah);
            pth.amp((psi + h) * ell_per_psi, env[2 * j + 2], a4, da4);
        } else {
            const T Sh = S0 * env[2 * j + 1], S4 = S0 * env[2 * j + 2];
            ah = pth.a0 * Sh;
            a4 = pth.a0 * S4;
            dah[0] = Sh;
            da4[0] = S4;
            dah[1] = da4[1] = T(0);
        }
        const StageAmp<T> Ah(ah, ph), A4(a4, ph);
        const StepLin<T, QUANTUM> L = rk4_linear<T, QUANTUM>(mu, s2, A1, Ah, A4, h, rad, chi_hi);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            T fm = T(0), fs = T(0);
            if (d != GD) {
                fm = fma(L.P1.x, da1[d], fma(L.Ph.x, dah[d], L.P4.x * da4[d]));
                fs = fma(L.P1.y, da1[d], fma(L.Ph.y, dah[d], L.P4.y * da4[d]));
            }
            const T m0 = vm[d];
            if (QUANTUM) {
                const T s0 = vs[d];
                vm[d] = fma(L.A.a, m0, fma(L.A.b, s0, fm));
                vs[d] = fma(L.A.c, m0, fma(L.A.d, s0, fs));
            } else {
                vm[d] = fma(L.A.a, m0, fm);
            }
        }
        if constexpr (PREC == PREC_F64) {
            mu += L.dmu;
            s2 += L.ds2;
        } else {
            comp_add(mu, mu_lo, L.dmu);
            comp_add(s2, s2_lo, L.ds2);
        }
        A1 = A4;
#pragma unroll
        for (int d = 0; d < ND; ++d) da1[d] = da4[d];
    }
    o.mu = ((double)mu + (double)mu_lo) + g0_rest;
    o.s2 = (double)s2 + (double)s2_lo;
    o.cmx = fmaxf(cmx, (float)(A1.chi_per_mu * mu));  // the end of the last step
    o.S0 = d0.S;
    o.g0 = g0;
    o.thx = thx;
    o.thy = thy;
    if (QUANTUM && !((float)chi_hi < chi_top)) flags |= kFlagRange;
    if (!(o.mu > 0.0) || !isfinite(o.mu) || !isfinite(o.s2)) flags |= kFlagNonFinite;

    // ---- chain to the eight parameters ----
    const double dthx_dd = 1e-3 * nrm[4], dthy_dd = 1e-3 * nrm[5];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T *v = c == 0 ? vm : vs;
        double *d = c == 0 ? o.dmu : o.ds2;
        if (c == 1 && !QUANTUM) {
#pragma unroll
            for (int p = 0; p < kGradParams; ++p) d[p] = 0.0;
            continue;
        }
        if (LOCAL) {
            d[0] = v[0];
            d[1] = v[1];
            d[2] = v[2];
            d[3] = v[3];
            d[4] = v[4];
            d[5] = v[5];
            d[6] = nrm[3] * (double)v[5];
            d[7] = v[6];
        } else {
            // every amplitude direction is a multiple of the a0 tangent
            const double b = sp.a0 * (double)v[0];
            d[0] = v[0];
            d[1] = b * d0.Lw;
            d[2] = b * d0.Lx;
            d[3] = b * d0.Ly;
            d[4] = b * kHalfC * d0.Lz;
            d[5] = v[1];
            d[6] = nrm[3] * (double)v[1];
            d[7] = b * (0.5 * z) * fma(dthx_dd, d0.Lx, dthy_dd * d0.Ly);
        }
    }
}

// Fixed-order reduction of the block's eight sums into the item's partials.
__device__ __forceinline__ void grad_item_reduce(const BatchParams &P, int64_t item,
                                                 const double *g, double (*red)[kGradParams]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < kGradParams; ++p) {
        const double v = wave_sum(g[p]);
        if (lane == 0) red[wid][p] = v;
    }
    __syncthreads();
    if (threadIdx.x < kGradParams) {
        double sum = 0.0;
        for (int w = 0; w < kPhaseBlock / 64; ++w) sum += red[w][threadIdx.x];
        P.partials[(size_t)item * kGradParams + threadIdx.x] = sum;
    }
    // red is rewritten only after the next item's barriers
}

// TAPE = false: the adjoint -- each sample's derivatives contracted at once
// with its law sensitivities, summed per item.  TAPE = true: the forward pass
// that also records the derivatives: final states for the deposit kernel and
// the tape (mu, sig2 and their eight derivatives, structure of arrays).
template <int PREC, bool QUANTUM, bool LOCAL, bool TAPE>
__global__ __launch_bounds__(kPhaseBlock) void tangent_kernel(BatchParams P,
                                                              const float *__restrict__ env32,
                                                              const double *__restrict__ env64) {
    constexpr bool kTab32 = QUANTUM && PREC != PREC_F64;
    __shared__ __align__(16) float tab32[kTab32 ? kCells32 * 4 * kDerivFuncs : 4];
    __shared__ int64_t slot;
    __shared__ double red[kPhaseBlock / 64][kGradParams];
    if (kTab32) {
        const float4 *src = reinterpret_cast<const float4 *>(P.rad32d);
        float4 *dst = reinterpret_cast<float4 *>(tab32);
        for (int k = threadIdx.x; k < kCells32 * kDerivFuncs; k += blockDim.x) dst[k] = src[k];
        __syncthreads();
    }
    for (;;) {
        const int64_t item = next_item(&P.queue[0], &slot);
        if (item >= P.n_items) break;
        const int s = __builtin_amdgcn_readfirstlane(find_shot(P.shots, P.n_shots, item, false));
        const ShotParams &sp = P.shots[s];
        const int64_t i = (item - sp.item0) * kPhaseBlock + threadIdx.x;
        double g[kGradParams];
#pragma unroll
        for (int p = 0; p < kGradParams; ++p) g[p] = 0.0;
        if (i < sp.n_samples) {
            int flags = 0;
            SampleTangent o;
            tangent_sample<PREC, QUANTUM, LOCAL>(P, sp, i, env32, env64, tab32, o, flags);
            if (TAPE) {
                const int64_t k = sp.state_off + i;
                P.st.mu[k] = o.mu;
                P.st.s2[k] = o.s2;
                P.st.S0[k] = o.S0;
                P.st.g0[k] = o.g0;
                P.st.thx[k] = o.thx;
                P.st.thy[k] = o.thy;
                P.st.cmx[k] = o.cmx;
                double *t = P.tape + k;
                const int64_t n = P.tape_n;
                t[0] = o.mu;
                t[n] = o.s2;
#pragma unroll
                for (int p = 0; p < kGradParams; ++p) {
                    t[(2 + p) * n] = o.dmu[p];
                    t[(2 + kGradParams + p) * n] = o.ds2[p];
                }
            } else if (!(flags & kFlagNonFinite)) {
                double lv, ls;
                law_sensitivity(o.mu, o.s2, P.deposit, P.ksig_bins, sp.e_lo, sp.e_w, sp.n_e,
                                P.gouts[s].d_energy, lv, ls);
#pragma unroll
                for (int p = 0; p < kGradParams; ++p) g[p] = fma(lv, o.dmu[p], ls * o.ds2[p]);
            }
            if (flags) atomicOr(&P.flags[s], flags);
        }
        if (!TAPE) grad_item_reduce(P, item, g, red);
    }
}

// The adjoint from a tape: contraction of the recorded derivatives with the
// law sensitivities (memory-bound: 144 bytes a sample).
__global__ __launch_bounds__(kPhaseBlock) void contract_kernel(BatchParams P) {
    __shared__ int64_t slot;
    __shared__ double red[kPhaseBlock / 64][kGradParams];
    for (;;) {
        const int64_t item = next_item(&P.queue[0], &slot);
        if (item >= P.n_items) break;
        const int s = __builtin_amdgcn_readfirstlane(find_shot(P.shots, P.n_shots, item, false));
        const ShotParams &sp = P.shots[s];
        const int64_t i = (item - sp.item0) * kPhaseBlock + threadIdx.x;
        double g[kGradParams];
#pragma unroll
        for (int p = 0; p < kGradParams; ++p) g[p] = 0.0;
        if (i < sp.n_samples) {
            const int64_t n = P.tape_n;
            const double *t = P.tape + sp.state_off + i;
            const double mu = t[0], s2 = t[n];
            if (mu > 0.0 && isfinite(mu) && isfinite(s2)) {
                double lv, ls;
                law_sensitivity(mu, s2, P.deposit, P.ksig_bins, sp.e_lo, sp.e_w, sp.n_e,
                                P.gouts[s].d_energy, lv, ls);
#pragma unroll
                for (int p = 0; p < kGradParams; ++p)
                    g[p] = fma(lv, t[(2 + p) * n], ls * t[(2 + kGradParams + p) * n]);
            } else {
                atomicOr(&P.flags[s], kFlagNonFinite);
            }
        }
        grad_item_reduce(P, item, g, red);
    }
}

// One block per shot: fixed-order sum of the shot's item partials.
__global__ __launch_bounds__(256) void grad_finalize_kernel(BatchParams P) {
    const int s = blockIdx.x;
    const ShotParams &sp = P.shots[s];
    const ShotGrad &so = P.gouts[s];
    const int64_t ni = (sp.n_samples + kPhaseBlock - 1) / kPhaseBlock;
    __shared__ double tree[256];
    for (int p = 0; p < kGradParams; ++p) {
        double acc = 0.0;
        for (int64_t b = threadIdx.x; b < ni; b += blockDim.x)
            acc += P.partials[(size_t)(sp.item0 + b) * kGradParams + p];
        tree[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) tree[threadIdx.x] += tree[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) so.grad[p] = tree[0];
        __syncthreads();
    }
    if (threadIdx.x == 0 && so.status) {
        const int fl = P.flags[s];
        *so.status = (fl & kFlagNonFinite) ? 4 : ((fl & kFlagRange) ? 6 : 0);
    }
}

__global__ void rad_derivs_kernel(const float *rad32d, const double *rad64d, int prec, int64_t n,
                                  const double *chi, double *out, int *flags) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int fl = (chi[k] < (double)(1 << (kEMax + 1))) ? 0 : kFlagRange;
    double v[kDerivFuncs];
    if (prec == 0) {
        // the FP32 table holds combinations: undo them
        RadCell6 cell;
        rad6_lookup32(rad32d, (float)chi[k], cell);
        const RadJ<float> r = rad6_cell_eval(cell, (float)chi[k]);
        const double g = r.g, G1 = (double)r.E1 - 2.0 * g;
        const double G2 = (double)r.E2 - 2.0 * g - 4.0 * G1;
        v[0] = g;
        v[1] = G1;
        v[2] = G2;
        v[3] = r.h;
        v[4] = (double)r.E3 - 6.0 * (G1 + G2);
        v[5] = r.H1;
    } else {
        rad6_plain64(rad64d, chi[k], v);
    }
    for (int f = 0; f < kDerivFuncs; ++f) out[kDerivFuncs * k + f] = v[f];
    if (fl) atomicOr(flags, fl);
}

// ===========================================================================
// Photon spectrum (Sec. 4).  Along each sample's trajectory every RK4 stage
// (weights h/6, h/3, h/3, h/6) emits the LCFA spectrum of its state:
//   d2N / (dpsi dxi) = C_ph F(xi, chi) / mu,   C_ph = alpha a_S / (2 sqrt3 pi),
// so that a stage adds c h C_ph (chi / mu) [Phi(e_{k+1}/mu; chi) -
// Phi(e_k/mu; chi)] / chi to photon-energy bin k, Phi(xi; chi) = Int_0^xi F.
// Evaluating Phi at every bin edge for every stage would cost the bin count
// per stage, so each stage instead deposits its weight c (chi / mu) =
// c 2|a| / a_S, bilinearly, into an emission grid over (ln chi, ln mu) kept
// in LDS in fixed point (order-independent sums); a finalize kernel then
// evaluates Phi / chi once per grid node and bin edge.  The grid spacing
// (0.2 in ln chi, at most ~0.05 in ln mu for the shot's energy range) sets the
// accuracy, about 1e-3 of the spectrum in L1.  Stages whose chi lies below
// the grid emit photons below the first bin (the host sizes the grid so): they
// add only their photon number, (5 pi / 2) chi (1 - 8 chi / (5 sqrt3)) per
// unit C_ph c / mu, to the lowest bin.  The emitted photon energy itself,
// c h (-A) summed over the stages (A: the drift), is accumulated exactly.
// ===========================================================================
__device__ __forceinline__ double ph_dz() { return cbrt(kPhYMax) / kPhNZ; }
__device__ __forceinline__ float ph_ln(float x) {
    return __builtin_amdgcn_logf(x) * 0.69314718055994530942f;
}
__device__ __forceinline__ float ph_ln(double x) { return (float)log(x); }

// K_{2/3} and K_{1/3} at the 5 Gauss-Legendre nodes of every z interval.
__constant__ double kGLx[5] = {-0.9061798459386640, -0.5384693101056831, 0.0,
                               0.5384693101056831, 0.9061798459386640};
__constant__ double kGLw[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                               0.4786286704993665, 0.2369268850561891};

__device__ __forceinline__ double ph_node_z(int g) {
    return ph_dz() * ((g / 5) + 0.5 + 0.5 * kGLx[g % 5]);
}

__global__ void ph_bessel_kernel(double *k23, double *k13) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 5 * kPhNZ) return;
    const double z = ph_node_z(g);
    const double y = z * z * z;
    // K_nu(y) = Int_0^inf exp(-y cosh t) cosh(nu t) dt (trapezoid, doubly
    // exponential decay)
    const double dt = 1.0 / 32.0;
    const double tmax = acosh(fmax(60.0 / y, 1.0)) + dt;
    const int nt = (int)ceil(tmax / dt);
    double s23 = 0.0, s13 = 0.0;
    for (int m = 0; m <= nt; ++m) {
        const double t = m * dt;
        const double e = exp(-y * cosh(t)) * (m == 0 ? 0.5 : 1.0);
        s23 += e * cosh(t * (2.0 / 3.0));
        s13 += e * cosh(t * (1.0 / 3.0));
    }
    k23[g] = s23 * dt;
    k13[g] = s13 * dt;
}

// Int_{y(z_j)}^inf K_{1/3}, accumulated downwards (y beyond kPhYMax: < 1e-34).
__global__ void ph_i13_kernel(const double *k13, double *i13) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const double dz = ph_dz();
    i13[kPhNZ] = 0.0;
    for (int j = kPhNZ - 1; j >= 0; --j) {
        double s = 0.0;
        for (int q = 0; q < 5; ++q) {
            const double z = ph_node_z(5 * j + q);
            s += kGLw[q] * k13[5 * j + q] * 3.0 * z * z;
        }
        i13[j] = i13[j + 1] + 0.5 * dz * s;
    }
}

// One row per thread: Phi / chi at the z nodes,
//   Phi = Int_0^y [w K_{2/3} xi_y - xi K_{1/3}] dy' - xi Int_y^inf K_{1/3}
// (the Int K_{1/3} term of F integrated by parts).
__global__ void ph_row_kernel(const double *k23, const double *k13, const double *i13,
                              double *phtab) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= kPhRows) return;
    const double chi = exp(kPhU0 + r * kPhDu);
    const double dz = ph_dz();
    double *row = phtab + (size_t)r * (kPhNZ + 1);
    double A = 0.0;
    // stored: Phi / (chi z), smooth at z = 0 where it tends to
    // 9 2^(-1/3) Gamma(2/3) (K_{2/3}(y) ~ Gamma(2/3)/2 (y/2)^(-2/3))
    row[0] = 9.0 * 0.79370052598409973738 * 1.3541179394264004169;
    for (int j = 0; j < kPhNZ; ++j) {
        double s = 0.0;
        for (int q = 0; q < 5; ++q) {
            const int g = 5 * j + q;
            const double z = ph_node_z(g);
            const double y = z * z * z;
            const double qq = 2.0 + 3.0 * chi * y;
            const double xi = 3.0 * chi * y / qq;
            const double w = 2.0 / qq + 0.5 * qq;
            const double xi_y = 6.0 * chi / (qq * qq);
            s += kGLw[q] * (w * k23[g] * xi_y - xi * k13[g]) * 3.0 * z * z;
        }
        A += 0.5 * dz * s;
        const double z1 = (j + 1) * dz, y1 = z1 * z1 * z1;
        const double xi1 = 3.0 * chi * y1 / (2.0 + 3.0 * chi * y1);
        row[j + 1] = (A - xi1 * i13[j + 1]) / (chi * z1);
    }
}

// Phi / chi on global row r at xi: the stored Phi / (chi z) interpolated by a
// cubic in z, times z (xi >= 1 and y >= kPhYMax give the row's total).
__device__ __forceinline__ double ph_cdf_row(const double *__restrict__ phtab, int r, double chi,
                                             double xi) {
    if (!(xi > 0.0)) return 0.0;
    const double *row = phtab + (size_t)r * (kPhNZ + 1);
    const double zmax = kPhNZ * ph_dz();
    if (xi >= 1.0) return row[kPhNZ] * zmax;
    const double y = 2.0 * xi / (3.0 * chi * (1.0 - xi));
    if (!(y < kPhYMax)) return row[kPhNZ] * zmax;
    const double z = cbrt(y);
    const double t = z / ph_dz();
    int j = (int)t - 1;
    j = j < 0 ? 0 : (j > kPhNZ - 3 ? kPhNZ - 3 : j);
    const double x = t - j;
    const double w0 = -(x - 1.0) * (x - 2.0) * (x - 3.0) * (1.0 / 6.0);
    const double w1 = x * (x - 2.0) * (x - 3.0) * 0.5;
    const double w2 = -x * (x - 1.0) * (x - 3.0) * 0.5;
    const double w3 = x * (x - 1.0) * (x - 2.0) * (1.0 / 6.0);
    return (w0 * row[j] + w1 * row[j + 1] + w2 * row[j + 2] + w3 * row[j + 3]) * z;
}

// Diagnostic: Phi(xi; chi) with cubic interpolation across rows as well.
__global__ void ph_cdf_kernel(const double *phtab, int64_t n, const double *chi,
                              const double *xi, double *out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double c = chi[k];
    const double s = (log(c) - kPhU0) / kPhDu;
    if (!(c > 0.0) || !(s >= 0.0) || !(s <= kPhRows - 1)) {
        out[k] = nan("");
        return;
    }
    int r = (int)s - 1;
    r = r < 0 ? 0 : (r > kPhRows - 4 ? kPhRows - 4 : r);
    const double x = s - r;
    const double wr[4] = {-(x - 1.0) * (x - 2.0) * (x - 3.0) / 6.0, x * (x - 2.0) * (x - 3.0) / 2.0,
                          -x * (x - 1.0) * (x - 3.0) / 2.0, x * (x - 1.0) * (x - 2.0) / 6.0};
    double acc = 0.0;
    for (int a = 0; a < 4; ++a) acc += wr[a] * ph_cdf_row(phtab, r + a, c, xi[k]);
    out[k] = acc * c;
}

// Emission of one stage: c = the stage weight over h, mu and a its state and
// amplitude, A its drift.
struct PhotAcc {
    double e_ph, soft;
    int flags;
};

template <class T>
__device__ __forceinline__ void ph_emit(T c, T mu, T a, T A, T h, T two_over_aS, T inv_a0,
                                        const ShotPhot &sp, unsigned long long *grid, PhotAcc &acc) {
    acc.e_ph += (double)(c * h * -A);
    const T aa = fabs(a);
    if (!(aa > T(0))) return;
    const T chi = two_over_aS * mu * aa;
    const T D = c * aa * inv_a0;  // deposit, in units of 2 a0 / a_S
    const float ru = (ph_ln(chi) - (float)(kPhU0 + sp.r_lo * kPhDu)) * (float)(1.0 / kPhDu);
    if (ru < 0.0f) {  // below the grid: photon number only
        acc.soft += (double)D * (1.0 - 0.92376043070340122 * (double)chi);
        return;
    }
    const float rv = (ph_ln(mu) - (float)sp.v_lo) / (float)sp.dv;
    float fu = ru, fv = rv;
    if (!(fu <= (float)(sp.nu - 1)) || !(fv >= 0.0f) || !(fv <= (float)(sp.nv - 1))) {
        acc.flags |= kFlagRange;
        fu = fminf(fmaxf(fu, 0.0f), (float)(sp.nu - 1));
        fv = fminf(fmaxf(fv, 0.0f), (float)(sp.nv - 1));
    }
    int n = min((int)fu, sp.nu - 2), m = min((int)fv, sp.nv - 2);
    const float du = fu - (float)n, dv = fv - (float)m;
    const double q = (double)D * kPhScale;
    unsigned long long *g = grid + n * sp.nv + m;
    const unsigned long long q00 = (unsigned long long)llrint(q * (double)((1.0f - du) * (1.0f - dv)));
    const unsigned long long q01 = (unsigned long long)llrint(q * (double)((1.0f - du) * dv));
    const unsigned long long q10 = (unsigned long long)llrint(q * (double)(du * (1.0f - dv)));
    const unsigned long long q11 = (unsigned long long)llrint(q * (double)(du * dv));
    if (q00) atomicAdd(g, q00);
    if (q01) atomicAdd(g + 1, q01);
    if (q10) atomicAdd(g + sp.nv, q10);
    if (q11) atomicAdd(g + sp.nv + 1, q11);
}

// Stage right-hand side with the drift A (the photon energy per unit phase is
// -A).  FP32 quantum: the forward table's combinations T1 = g, T2 = 2g +
// chi g', T3 = g + 2 chi g' + chi^2 g''/2, T4 = h.
template <class T, bool QUANTUM>
__device__ __forceinline__ void stage_rhs(T mu, T s2, T a, const Phys<T> &ph, const T *tab,
                                          T &dmu, T &ds2, T &A, T &chi_hi) {
    const T a2 = a * a;
    const T u = ph.K * a2;
    const T mu2 = mu * mu;
    if (!QUANTUM) {
        A = -u * mu2;
        dmu = A;
        ds2 = T(0);
        return;
    }
    const T aa = fabs(a);
    const T chi = ph.two_over_aS * mu * aa;
    chi_hi = fmax(chi_hi, chi);
    const T D = ph.CD * aa * a2 * mu2 * mu2;
    if constexpr (std::is_same<T, float>::value) {
        float T1, T2, T3, T4;
        rad_eval32(tab, chi, T1, T2, T3, T4);
        A = -u * mu2 * T1;
        dmu = -u * fmaf(mu2, T1, s2 * T3);
        ds2 = fmaf(-2.0f * u * mu * s2, T2, D * T4);
    } else {
        double g, G1, G2, hq;
        rad_eval64(tab, chi, g, G1, G2, hq);
        A = -u * mu2 * g;
        dmu = fma(-0.5 * u * (2.0 * g + 4.0 * G1 + G2), s2, A);
        ds2 = fma(-2.0 * u * mu * (2.0 * g + G1), s2, D * hq);
    }
}

template <int PREC, bool QUANTUM, bool LOCAL>
__device__ __forceinline__ void photon_sample(const BatchParams &P, const ShotParams &sp,
                                              const ShotPhot &pp, int64_t i,
                                              const float *__restrict__ env32,
                                              const double *__restrict__ env64,
                                              const float *tab32, unsigned long long *grid,
                                              PhotAcc &acc, double &loss) {
    using T = typename std::conditional<PREC == PREC_F64, double, float>::type;
    const T *env;
    const T *tab;
    if constexpr (PREC == PREC_F64) {
        env = env64;
        tab = P.rad64;
    } else {
        env = env32;
        tab = tab32;
    }
    Phys<T> ph;
    ph.K = (T)P.K;
    ph.CD = (T)P.CD;
    ph.two_over_aS = (T)P.two_over_aS;
    const int N = P.n_steps;
    const bool local = LOCAL && !sp.plane_wave;

    double nrm[6];
    sample_normals((uint32_t)i, (uint32_t)sp.shot_word, P.key0, P.key1, nrm);
    const double x = fma(sp.sigma_r, nrm[0], sp.x_off);
    const double y = fma(sp.sigma_r, nrm[1], sp.y_off);
    const double z = sp.sigma_z * nrm[2];
    const double g0 = fma(sp.sigma_gamma, nrm[3], sp.gamma0);
    const double thx = sp.div_rad * nrm[4];
    const double thy = sp.div_rad * nrm[5];
    Path<double> pd;
    pd.xc = fma(thx, 0.5 * z, x);
    pd.yc = fma(thy, 0.5 * z, y);
    pd.thx = thx;
    pd.thy = thy;
    pd.zstar = fma(0.5, z, sp.z_delay);
    pd.inv_w0sq = sp.inv_w0sq;
    pd.inv_zR = sp.inv_zR;
    const double S0 = sp.plane_wave ? 1.0 : pd.S(0.0);
    Path<T> pt;
    pt.xc = (T)pd.xc;
    pt.yc = (T)pd.yc;
    pt.thx = (T)thx;
    pt.thy = (T)thy;
    pt.zstar = (T)pd.zstar;
    pt.inv_w0sq = (T)sp.inv_w0sq;
    pt.inv_zR = (T)sp.inv_zR;

    const T a0 = (T)sp.a0, a0S0 = (T)(sp.a0 * S0);
    const T inv_a0 = sp.a0 > 0.0 ? (T)(1.0 / sp.a0) : T(0);
    const T h = (T)P.h, hh = T(0.5) * h, psi0 = (T)(-P.psi_max), ell = (T)P.ell_per_psi;
    const T c16 = T(1.0 / 6.0), c13 = T(1.0 / 3.0);
    T mu = (T)g0, mu_lo = T(0), s2 = T(0), s2_lo = T(0);
    double g0_rest = 0.0;
    if constexpr (PREC != PREC_F64) {
        mu_lo = (T)(g0 - (double)mu);
        g0_rest = (g0 - (double)mu) - (double)mu_lo;
    }
    T chi_hi = T(0);
    T aS_prev = local ? a0 * pt.S(psi0 * ell) : a0S0;
    for (int j = 0; j < N; ++j) {
        const T psi = fma((T)j, h, psi0);
        T aSh = a0S0, aS4 = a0S0;
        if (local) {
            aSh = a0 * pt.S(fma(T(0.5), h, psi) * ell);
            aS4 = a0 * pt.S((psi + h) * ell);
        }
        const T a1 = aS_prev * env[2 * j], ah = aSh * env[2 * j + 1], a4 = aS4 * env[2 * j + 2];
        T k1m, k1s, A1, k2m, k2s, A2, k3m, k3s, A3, k4m, k4s, A4;
        stage_rhs<T, QUANTUM>(mu, s2, a1, ph, tab, k1m, k1s, A1, chi_hi);
        ph_emit(c16, mu, a1, A1, h, ph.two_over_aS, inv_a0, pp, grid, acc);
        const T m2 = fma(hh, k1m, mu);
        stage_rhs<T, QUANTUM>(m2, fma(hh, k1s, s2), ah, ph, tab, k2m, k2s, A2, chi_hi);
        ph_emit(c13, m2, ah, A2, h, ph.two_over_aS, inv_a0, pp, grid, acc);
        const T m3 = fma(hh, k2m, mu);
        stage_rhs<T, QUANTUM>(m3, fma(hh, k2s, s2), ah, ph, tab, k3m, k3s, A3, chi_hi);
        ph_emit(c13, m3, ah, A3, h, ph.two_over_aS, inv_a0, pp, grid, acc);
        const T m4 = fma(h, k3m, mu);
        stage_rhs<T, QUANTUM>(m4, fma(h, k3s, s2), a4, ph, tab, k4m, k4s, A4, chi_hi);
        ph_emit(c16, m4, a4, A4, h, ph.two_over_aS, inv_a0, pp, grid, acc);
        const T h6 = h * c16;
        const T dm = h6 * (k1m + T(2) * (k2m + k3m) + k4m);
        const T ds = h6 * (k1s + T(2) * (k2s + k3s) + k4s);
        if constexpr (PREC == PREC_F64) {
            mu += dm;
            s2 += ds;
        } else {
            comp_add(mu, mu_lo, dm);
            comp_add(s2, s2_lo, ds);
        }
        aS_prev = aS4;
    }
    const double mu_f = ((double)mu + (double)mu_lo) + g0_rest;
    if (QUANTUM && !((float)chi_hi < (float)(1 << (kEMax + 1)))) acc.flags |= kFlagRange;
    if (!(mu_f > 0.0) || !isfinite(mu_f)) {
        acc.flags |= kFlagNonFinite;
        return;
    }
    loss += g0 - mu_f;
}

__device__ __forceinline__ int find_phot(const ShotPhot *ph, int n_shots, int64_t item) {
    int lo = 0, hi = n_shots - 1;  // largest s whose first item is <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ph[mid].pitem0 <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int PREC, bool QUANTUM, bool LOCAL>
__global__ __launch_bounds__(kDepBlock) void photon_kernel(BatchParams P,
                                                           const float *__restrict__ env32,
                                                           const double *__restrict__ env64) {
    constexpr bool kTab32 = QUANTUM && PREC != PREC_F64;
    __shared__ __align__(16) float tab32[kTab32 ? kCells32 * kCellVals : 4];
    __shared__ unsigned long long grid[kPhNodes];
    __shared__ int64_t slot;
    __shared__ double red[kDepBlock / 64][kPhotPartials];
    if (kTab32) {
        const float4 *src = reinterpret_cast<const float4 *>(P.rad32);
        float4 *dst = reinterpret_cast<float4 *>(tab32);
        for (int k = threadIdx.x; k < kCells32 * kCellVals / 4; k += blockDim.x) dst[k] = src[k];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (;;) {
        const int64_t item = next_item(&P.queue[0], &slot);
        if (item >= P.n_pitems) break;
        const int s = __builtin_amdgcn_readfirstlane(find_phot(P.phot, P.n_shots, item));
        const ShotParams &sp = P.shots[s];
        const ShotPhot &pp = P.phot[s];
        const int nodes = pp.nu * pp.nv;
        for (int k = threadIdx.x; k < nodes; k += blockDim.x) grid[k] = 0ull;
        __syncthreads();
        PhotAcc acc{0.0, 0.0, 0};
        double loss = 0.0;
        const int64_t i0 = (item - pp.pitem0) * kPhotTile;
        const int64_t i1 = i0 + kPhotTile < sp.n_samples ? i0 + kPhotTile : sp.n_samples;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x)
            photon_sample<PREC, QUANTUM, LOCAL>(P, sp, pp, i, env32, env64, tab32, grid, acc,
                                                loss);
        if (acc.flags) atomicOr(&P.flags[s], acc.flags);
        const double v[kPhotPartials] = {acc.e_ph, loss, acc.soft};
#pragma unroll
        for (int m = 0; m < kPhotPartials; ++m) {
            const double w = wave_sum(v[m]);
            if (lane == 0) red[wid][m] = w;
        }
        __syncthreads();
        if (threadIdx.x < kPhotPartials) {
            double sum = 0.0;
            for (int w = 0; w < kDepBlock / 64; ++w) sum += red[w][threadIdx.x];
            P.partials[(size_t)item * kPhotPartials + threadIdx.x] = sum;
        }
        for (int k = threadIdx.x; k < nodes; k += blockDim.x) {
            const unsigned long long w = grid[k];
            if (w) atomicAdd(&P.pgrid[pp.grid_off + k], w);
        }
        __syncthreads();  // the next item clears the grid
    }
}

// One block per shot: the item sums in a fixed order, then the spectrum.
// With S_k = sum over grid nodes of W_node Phi(e_k / mu_node; chi_node) / chi_node
// (nodes in index order), bin k holds C (S_{k+1} - S_k), the underflow C S_0
// and the overflow C (S_total - S_n), C = 2^-24 (2 a0 / a_S) h C_ph.
constexpr int kPhMaxEdgesPerThread = (4096 + 2 + 255) / 256;

__global__ __launch_bounds__(256) void photon_finalize_kernel(BatchParams P, double c_ph) {
    const int s = blockIdx.x;
    const ShotParams &sp = P.shots[s];
    const ShotPhot &pp = P.phot[s];
    __shared__ double tree[256];
    __shared__ double sums[kPhotPartials];
    __shared__ double nzw[kPhNodes + 2];   // weights of the non-zero nodes, then S_k
    __shared__ unsigned short nzi[kPhNodes];
    __shared__ int cnt[257];
    const int tid = threadIdx.x;
    const int64_t ni = (sp.n_samples + kPhotTile - 1) / kPhotTile;
    for (int m = 0; m < kPhotPartials; ++m) {
        double a = 0.0;
        for (int64_t b = tid; b < ni; b += blockDim.x)
            a += P.partials[(size_t)(pp.pitem0 + b) * kPhotPartials + m];
        tree[tid] = a;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) tree[tid] += tree[tid + w];
            __syncthreads();
        }
        if (tid == 0) sums[m] = tree[0];
        __syncthreads();
    }
    // compact the non-zero nodes in index order
    const int nodes = pp.nu * pp.nv;
    const unsigned long long *G = P.pgrid + pp.grid_off;
    constexpr int kPer = kPhNodes / 256;
    int mine = 0;
    for (int q = 0; q < kPer; ++q) {
        const int k = tid * kPer + q;
        if (k < nodes && G[k]) ++mine;
    }
    cnt[tid + 1] = mine;
    if (tid == 0) cnt[0] = 0;
    __syncthreads();
    if (tid == 0)
        for (int t = 1; t <= 256; ++t) cnt[t] += cnt[t - 1];
    __syncthreads();
    int pos = cnt[tid];
    for (int q = 0; q < kPer; ++q) {
        const int k = tid * kPer + q;
        if (k < nodes && G[k]) {
            nzi[pos] = (unsigned short)k;
            nzw[pos] = (double)G[k];
            ++pos;
        }
    }
    __syncthreads();
    const int nnz = cnt[256];
    // edge sums: thread tid owns edges tid, tid + 256, ...; index n_ph + 1
    // stands for the total
    const int n_edges = pp.n_ph + 2;
    double S[kPhMaxEdgesPerThread];
    for (int q = 0; q < kPhMaxEdgesPerThread; ++q) S[q] = 0.0;
    for (int z = 0; z < nnz; ++z) {
        const int k = nzi[z];
        const int n = k / pp.nv, m = k - n * pp.nv;
        const int r = pp.r_lo + n;
        const double chi = exp(kPhU0 + r * kPhDu);
        const double inv_mu = exp(-(pp.v_lo + m * pp.dv));
        const double w = nzw[z];
        for (int q = 0; q < kPhMaxEdgesPerThread; ++q) {
            const int e = tid + 256 * q;
            if (e >= n_edges) break;
            const double xi = e == pp.n_ph + 1 ? 2.0 : (pp.ph_lo + e * pp.ph_w) * inv_mu;
            S[q] = fma(w, ph_cdf_row(P.phtab, r, chi, xi), S[q]);
        }
    }
    __syncthreads();  // nzw is reused for S
    for (int q = 0; q < kPhMaxEdgesPerThread; ++q) {
        const int e = tid + 256 * q;
        if (e < n_edges) nzw[e] = S[q];
    }
    __syncthreads();
    const double C = (1.0 / kPhScale) * (2.0 * sp.a0 * P.two_over_aS * 0.5) * P.h * c_ph;
    // C = 2^-24 (2 a0 / a_S) h C_ph  (two_over_aS / 2 = 1 / a_S)
    const double soft = sums[2] * (2.0 * sp.a0 * P.two_over_aS * 0.5) * P.h * c_ph *
                        (5.0 * 3.14159265358979323846 / 2.0);
    const int n = pp.n_ph;
    for (int k = tid; k < n + 2; k += blockDim.x) {
        double v;
        if (k < n)
            v = C * (nzw[k + 1] - nzw[k]);
        else if (k == n)
            v = C * nzw[0];
        else
            v = C * (nzw[n + 1] - nzw[n]);
        if (pp.ph_lo > 0.0 ? k == n : k == 0) v += soft;
        pp.hist[k] = v;
    }
    if (tid == 0) {
        pp.energy[0] = sums[0];
        pp.energy[1] = sums[1];
        if (pp.status) {
            const int fl = P.flags[s];
            *pp.status = (fl & kFlagNonFinite) ? 4 : ((fl & kFlagRange) ? 6 : 0);
        }
    }
}

// ===========================================================================
// Launchers
// ===========================================================================
size_t radiation_work_doubles() {
    return (size_t)kNY * kYVals + (size_t)4 * kNodeVals * (kCells32 + kCells64);
}

hipError_t build_radiation_tables(float *rad32, double *rad64, float *rad32d, double *rad64d,
                                  double *work, size_t work_doubles, hipStream_t s) {
    if (work_doubles < radiation_work_doubles()) return hipErrorInvalidValue;
    double *yf = work, *vals = work + (size_t)kNY * kYVals;
    rad_y_kernel<<<(kNY + 63) / 64, 64, 0, s>>>(yf);
    const int nodes = 4 * (kCells32 + kCells64);
    rad_node_kernel<<<(nodes + 63) / 64, 64, 0, s>>>(yf, vals);
    const int cells = kCells32 + kCells64;
    rad_coef_kernel<<<(cells + 63) / 64, 64, 0, s>>>(vals, rad32, rad64, rad32d, rad64d);
    return hipGetLastError();
}

hipError_t launch_envelope(double psi_max, double h, int n_steps, int envelope, double omega_tau,
                           float *env32, double *env64, hipStream_t s) {
    const int n = 2 * n_steps + 1;
    envelope_kernel<<<(n + 255) / 256, 256, 0, s>>>(psi_max, h, n_steps, envelope, omega_tau,
                                                    env32, env64);
    return hipGetLastError();
}

hipError_t launch_zero(unsigned long long *p, size_t n64, hipStream_t s) {
    if (n64 == 0) return hipSuccess;
    const int grid = (int)((n64 + 255) / 256 < 1024 ? (n64 + 255) / 256 : 1024);
    zero_kernel<<<grid, 256, 0, s>>>(p, n64);
    return hipGetLastError();
}

template <int PREC, bool QUANTUM, bool LOCAL>
static const void *phase_ptr() {
    return reinterpret_cast<const void *>(&phase_kernel<PREC, QUANTUM, LOCAL>);
}

static const void *select_phase(int prec, int rr, int amp) {
    const bool q = rr == 1, l = amp == 1;
    if (prec == PREC_F32MIX && !q) prec = PREC_F32;  // no radiation table, no promotion
#define QS_SEL(P)                                              \
    if (prec == P) {                                           \
        if (q && l) return phase_ptr<P, true, true>();         \
        if (q && !l) return phase_ptr<P, true, false>();       \
        if (!q && l) return phase_ptr<P, false, true>();       \
        return phase_ptr<P, false, false>();                   \
    }
    QS_SEL(PREC_F32)
    QS_SEL(PREC_F64)
    if (prec == PREC_F32MIX) {
        if (l) return phase_ptr<PREC_F32MIX, true, true>();
        return phase_ptr<PREC_F32MIX, true, false>();
    }
#undef QS_SEL
    return nullptr;
}

static hipError_t resident_grid(const void *fn, int block, size_t lds, int64_t items, int *grid) {
    int device = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds);
    if (e != hipSuccess) return e;
    int64_t g = (int64_t)(per_cu < 1 ? 1 : per_cu) * ncu;
    if (g > items) g = items;
    *grid = (int)(g < 1 ? 1 : g);
    return hipSuccess;
}

hipError_t launch_phase(const BatchParams &p, const float *env32, const double *env64, int prec,
                        int rr, int amp, hipStream_t s) {
    const void *fn = select_phase(prec, rr, amp);
    if (!fn) return hipErrorInvalidValue;
    int grid = 0;
    hipError_t e = resident_grid(fn, kPhaseBlock, 0, p.n_items, &grid);
    if (e != hipSuccess) return e;
    BatchParams pc = p;
    const float *e32 = env32;
    const double *e64 = env64;
    void *args[] = {&pc, &e32, &e64};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kPhaseBlock), args, 0, s);
}

size_t deposit_lds_bytes(int max_hist_words) { return (size_t)max_hist_words * 8; }

hipError_t launch_deposit(const BatchParams &p, int max_hist_words, hipStream_t s) {
    const void *fn = reinterpret_cast<const void *>(&deposit_kernel);
    const size_t lds = deposit_lds_bytes(max_hist_words);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int grid = 0;
    e = resident_grid(fn, kDepBlock, lds, p.n_ditems, &grid);
    if (e != hipSuccess) return e;
    deposit_kernel<<<grid, kDepBlock, lds, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_finalize(const BatchParams &p, hipStream_t s) {
    finalize_kernel<<<p.n_shots, 256, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_radiation_eval(const float *rad32, const double *rad64, int prec, int64_t n,
                                 const double *chi, double *out, int *flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    rad_eval_kernel<<<(unsigned)blocks, 256, 0, s>>>(rad32, rad64, prec, n, chi, out, flags);
    return hipGetLastError();
}

template <int PREC, bool QUANTUM, bool LOCAL, bool TAPE>
static const void *tangent_ptr() {
    return reinterpret_cast<const void *>(&tangent_kernel<PREC, QUANTUM, LOCAL, TAPE>);
}

template <bool TAPE>
static const void *select_tangent(int prec, int rr, int amp) {
    const bool q = rr == 1, l = amp == 1;
    if (prec == PREC_F64)
        return q ? (l ? tangent_ptr<PREC_F64, true, true, TAPE>()
                      : tangent_ptr<PREC_F64, true, false, TAPE>())
                 : (l ? tangent_ptr<PREC_F64, false, true, TAPE>()
                      : tangent_ptr<PREC_F64, false, false, TAPE>());
    return q ? (l ? tangent_ptr<PREC_F32, true, true, TAPE>()
                  : tangent_ptr<PREC_F32, true, false, TAPE>())
             : (l ? tangent_ptr<PREC_F32, false, true, TAPE>()
                  : tangent_ptr<PREC_F32, false, false, TAPE>());
}

hipError_t launch_tangent(const BatchParams &p, const float *env32, const double *env64, int prec,
                          int rr, int amp, bool tape, hipStream_t s) {
    const void *fn = tape ? select_tangent<true>(prec, rr, amp) : select_tangent<false>(prec, rr, amp);
    int grid = 0;
    hipError_t e = resident_grid(fn, kPhaseBlock, 0, p.n_items, &grid);
    if (e != hipSuccess) return e;
    BatchParams pc = p;
    const float *e32 = env32;
    const double *e64 = env64;
    void *args[] = {&pc, &e32, &e64};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kPhaseBlock), args, 0, s);
}

hipError_t launch_contract(const BatchParams &p, hipStream_t s) {
    const void *fn = reinterpret_cast<const void *>(&contract_kernel);
    int grid = 0;
    hipError_t e = resident_grid(fn, kPhaseBlock, 0, p.n_items, &grid);
    if (e != hipSuccess) return e;
    contract_kernel<<<grid, kPhaseBlock, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_grad_finalize(const BatchParams &p, hipStream_t s) {
    grad_finalize_kernel<<<p.n_shots, 256, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_radiation_derivs(const float *rad32d, const double *rad64d, int prec, int64_t n,
                                   const double *chi, double *out, int *flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    rad_derivs_kernel<<<(unsigned)blocks, 256, 0, s>>>(rad32d, rad64d, prec, n, chi, out, flags);
    return hipGetLastError();
}

size_t photon_work_doubles() { return (size_t)2 * 5 * kPhNZ + (kPhNZ + 1); }

hipError_t build_photon_table(double *phtab, double *work, size_t work_doubles, hipStream_t s) {
    if (work_doubles < photon_work_doubles()) return hipErrorInvalidValue;
    double *k23 = work, *k13 = work + 5 * kPhNZ, *i13 = work + 10 * kPhNZ;
    ph_bessel_kernel<<<(5 * kPhNZ + 63) / 64, 64, 0, s>>>(k23, k13);
    ph_i13_kernel<<<1, 1, 0, s>>>(k13, i13);
    ph_row_kernel<<<(kPhRows + 63) / 64, 64, 0, s>>>(k23, k13, i13, phtab);
    return hipGetLastError();
}

template <int PREC, bool QUANTUM, bool LOCAL>
static const void *photon_ptr() {
    return reinterpret_cast<const void *>(&photon_kernel<PREC, QUANTUM, LOCAL>);
}

hipError_t launch_photon(const BatchParams &p, const float *env32, const double *env64, int prec,
                         int rr, int amp, hipStream_t s) {
    const bool q = rr == 1, l = amp == 1;
    const void *fn;
    if (prec == PREC_F64)
        fn = q ? (l ? photon_ptr<PREC_F64, true, true>() : photon_ptr<PREC_F64, true, false>())
               : (l ? photon_ptr<PREC_F64, false, true>() : photon_ptr<PREC_F64, false, false>());
    else
        fn = q ? (l ? photon_ptr<PREC_F32, true, true>() : photon_ptr<PREC_F32, true, false>())
               : (l ? photon_ptr<PREC_F32, false, true>() : photon_ptr<PREC_F32, false, false>());
    int grid = 0;
    hipError_t e = resident_grid(fn, kDepBlock, 0, p.n_pitems, &grid);
    if (e != hipSuccess) return e;
    BatchParams pc = p;
    const float *e32 = env32;
    const double *e64 = env64;
    void *args[] = {&pc, &e32, &e64};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kDepBlock), args, 0, s);
}

hipError_t launch_photon_finalize(const BatchParams &p, double c_ph, hipStream_t s) {
    photon_finalize_kernel<<<p.n_shots, 256, 0, s>>>(p, c_ph);
    return hipGetLastError();
}

hipError_t launch_photon_cdf(const double *phtab, int64_t n, const double *chi, const double *xi,
                             double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    ph_cdf_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(phtab, n, chi, xi, out);
    return hipGetLastError();
}

}  // namespace qs
