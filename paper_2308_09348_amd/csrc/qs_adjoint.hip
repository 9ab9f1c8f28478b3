// qs_adjoint.hip -- derivatives of the energy histogram with respect to the
// eight shot parameters: the tangent kernel (adjoint, or forward pass with a
// derivative tape), the tape contraction and the per-shot reduction.
#include "qs_device.h"

namespace qs {

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

// Index from chi clamped to the octave cells, as rad_lookup32 (the first
// octave cell extrapolates linearly down to chi = 0).
__device__ __forceinline__ void rad6_lookup32(const float *__restrict__ tab, float chi,
                                              RadCell6 &cell) {
    const float xc = fminf(fmaxf(chi, 0x1p-20f), 0x1.fffffep7f);
    const uint32_t b = __float_as_uint(xc);
    const uint32_t c = ((b - ((uint32_t)(127 + kEMin) << 23)) >> (23 - kSB32)) + 1u;
    const float tw = __uint_as_float((uint32_t)(254 + kSB32 - (int)(b >> 23)) << 23);
    const float ts = -__uint_as_float(b & ~((1u << (23 - kSB32)) - 1)) * tw;
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

__device__ __forceinline__ RadJ<double> radj_combine(const double v[kDerivFuncs]) {
    const double g = v[0], G1 = v[1], G2 = v[2], h = v[3], G3 = v[4], H1 = v[5];
    return RadJ<double>{g, fma(2.0, g, G1), fma(4.0, G1, fma(2.0, g, G2)), fma(6.0, G1 + G2, G3),
                        h, H1};
}

__device__ __forceinline__ RadJ<double> radj_eval64(const double *__restrict__ tab, double chi) {
    double v[kDerivFuncs];
    rad6_plain64(tab, chi, v);
    return radj_combine(v);
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

template <class T, bool Q, class Src = RadSrc<T>>
__device__ __forceinline__ StepLin<T, Q> rk4_linear(T mu, T s2, const StageAmp<T> &A1,
                                                    const StageAmp<T> &Ah, const StageAmp<T> &A4,
                                                    T h, Src &rad, T &chi_hi) {
    // The stage matrices M_s = K_s (I + c_s M_{s-1}) and the forcing chains
    // e_s1 = c_s K_s e_{s-1,1}, e_sh = c_s K_s e_{s-1,h} (+ g_s) are summed
    // with the RK4 weights as they are formed, so only the running sums and
    // the latest stage stay live.
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
    Mat2<T> M{K1.mm, K1.ms, K1.sm, K1.ss};
    Mat2<T> SA = M;                  // M1 + 2 M2 + 2 M3 + M4
    Vec2<T> e1{K1.ma, K1.sa};        // g1, e21, e31, e41
    Vec2<T> S1 = e1;                 // g1 + 2 e21 + 2 e31 + e41
    T Sm = K1.fm, Ss = K1.fs;        // k1 + 2 k2 + 2 k3 + k4
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
    M = kism<T, Q>(K2, hh, M);
    SA = Mat2<T>{fma(T(2), M.a, SA.a), fma(T(2), M.b, SA.b), fma(T(2), M.c, SA.c),
                 fma(T(2), M.d, SA.d)};
    e1 = skv<T, Q>(K2, hh, e1);
    S1 = Vec2<T>{fma(T(2), e1.x, S1.x), fma(T(2), e1.y, S1.y)};
    Vec2<T> eh{K2.ma, K2.sa};                        // g2, e3h, e4h
    Vec2<T> Sh{T(2) * eh.x, T(2) * eh.y};           // 2 g2 + 2 e3h + e4h
    Sm = fma(T(2), K2.fm, Sm);
    Ss = fma(T(2), K2.fs, Ss);
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
    M = kism<T, Q>(K3, hh, M);
    SA = Mat2<T>{fma(T(2), M.a, SA.a), fma(T(2), M.b, SA.b), fma(T(2), M.c, SA.c),
                 fma(T(2), M.d, SA.d)};
    e1 = skv<T, Q>(K3, hh, e1);
    S1 = Vec2<T>{fma(T(2), e1.x, S1.x), fma(T(2), e1.y, S1.y)};
    eh = skv<T, Q>(K3, hh, eh);
    eh.x += K3.ma;
    eh.y += K3.sa;
    Sh = Vec2<T>{fma(T(2), eh.x, Sh.x), fma(T(2), eh.y, Sh.y)};
    Sm = fma(T(2), K3.fm, Sm);
    Ss = fma(T(2), K3.fs, Ss);
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
    M = kism<T, Q>(K4, h, M);
    e1 = skv<T, Q>(K4, h, e1);
    eh = skv<T, Q>(K4, h, eh);
    // assemble
    L.A.a = fma(h6, SA.a + M.a, T(1));
    L.A.b = h6 * (SA.b + M.b);
    L.A.c = h6 * (SA.c + M.c);
    L.A.d = fma(h6, SA.d + M.d, T(1));
    L.P1.x = h6 * (S1.x + e1.x);
    L.P1.y = h6 * (S1.y + e1.y);
    L.Ph.x = h6 * (Sh.x + eh.x);
    L.Ph.y = h6 * (Sh.y + eh.y);
    L.P4.x = h6 * K4.ma;
    L.P4.y = h6 * K4.sa;
    L.dmu = h6 * (Sm + K4.fm);
    L.ds2 = h6 * (Ss + K4.fs);
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

// A sample's draw, its path in FP64 and the spatial factor at its collision
// point with the log-derivatives.  The tangent loop recomputes this where it
// needs it (FP64 steps, the chain to the parameters at the end) instead of
// carrying it through the phase steps: the draw is a few hundred operations
// against the thousands a step costs, and the registers go to the loop.
struct AdjSample {
    SampleCoords sc;
    AdjPath<double> p;
    SpD<double> d0;
};

// The sample index hidden from the optimiser, so that a recomputation is not
// merged with an earlier one into values kept live in between.
__device__ __forceinline__ int64_t opaque_index(int64_t i) {
    asm volatile("" : "+v"(i));
    return i;
}

__device__ __forceinline__ void adj_sample(const BatchParams &P, const ShotParams &sp, int64_t i,
                                           AdjSample &s) {
    constexpr double kHalfC = 0.5 * 0.299792458;  // d z* / d delay [um/fs]
    sample_coords(sp, P.key0, P.key1, i, s.sc);
    const double z = s.sc.z;
    s.p.xc = fma(s.sc.thx, 0.5 * z, s.sc.x);
    s.p.yc = fma(s.sc.thy, 0.5 * z, s.sc.y);
    s.p.thx = s.sc.thx;
    s.p.thy = s.sc.thy;
    s.p.zstar = fma(0.5, z, sp.z_delay);
    s.p.hz = 0.5 * z;
    s.p.dthx = 1e-3 * s.sc.n[4];
    s.p.dthy = 1e-3 * s.sc.n[5];
    s.p.inv_w0sq = sp.inv_w0sq;
    s.p.inv_zR = sp.inv_zR;
    s.p.inv_w0 = sqrt(sp.inv_w0sq);
    s.p.a0 = sp.a0;
    s.p.zfac = kHalfC;
    s.d0 = spatial_d(s.p.xc, s.p.yc, s.p.zstar, sp.inv_w0sq, sp.inv_zR, s.p.inv_w0);
}

template <class T>
__device__ __forceinline__ AdjPath<T> adj_path_cast(const AdjPath<double> &p) {
    AdjPath<T> r;
    r.xc = (T)p.xc;
    r.yc = (T)p.yc;
    r.thx = (T)p.thx;
    r.thy = (T)p.thy;
    r.zstar = (T)p.zstar;
    r.hz = (T)p.hz;
    r.dthx = (T)p.dthx;
    r.dthy = (T)p.dthy;
    r.inv_w0sq = (T)p.inv_w0sq;
    r.inv_zR = (T)p.inv_zR;
    r.inv_w0 = (T)p.inv_w0;
    r.a0 = (T)p.a0;
    r.zfac = (T)p.zfac;
    return r;
}

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
    if (mode == 2) {
        // the Gaussian density along the edges by multiplications:
        // phi(z + dz) = phi(z) r, r = exp(-z dz - dz^2 / 2), and r itself
        // advances by exp(-dz^2) (exact in the arithmetic; FP64 rounding adds
        // an ulp or two an edge)
        const double dz = wb * inv_se;
        const double q = exp(-dz * dz);
        double z = (fma((double)ja, wb, lo) - v) * inv_se;
        double f = phi_pdf(z) * inv_se;
        double r = exp(fma(-z, dz, -0.5 * dz * dz));
        for (int j = ja; j <= jb; ++j) {
            const double wl = j == 0 ? W[n] : W[j - 1];
            const double wr = j == n ? W[n + 1] : W[j];
            const double c = wl - wr;
            sv = fma(c, f, sv);
            ss = fma(c, -z * f, ss);
            f *= r;
            r *= q;
            z += dz;
        }
        lv = -sv;
        ls2 = ss * dse;
        return;
    }
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

// Share of one sample in the angle-histogram and moment terms of L, as
// derivatives along the eight parameters added to g.  The sample's energy
// state (mu, sig2) and its derivatives come from the trajectory; the draw
// gives the rest: theta = div n (derivative n in mrad per mrad), gamma0,i =
// gamma0 + sigma_gamma n3, and a0,eff = a0 S0 with S0 at the collision point
// (ln S0 derivatives of spatial_d; the divergence moves the collision point
// by theta z / 2).  The angle law is N(theta_x, sig_th^2) with sig_th^2 =
// C^2 a0,eff^2 max(sig2, 0) / mu^4 (Sec. 5.2), deposited like the energy law;
// the moments are those of the finalize kernel:
//   mean gamma = sum mu / W,   std^2 = sum (mu^2 + sig2^+) / W - mean^2,
//   mean and rms of theta_x (rms with sig_th^2) and theta_y, mean a0,eff,
//   mean 1 - mu / gamma0,i, mean sqrt(sig2^+);
// the weight, the largest chi and the FP64-shadow fields carry no derivative.
__device__ void observable_sensitivity(const BatchParams &P, const ShotParams &sp,
                                       const ShotGrad &go, int64_t i, double mu, double s2,
                                       const double *dmu, const double *ds2, double *g) {
    if (!go.d_angle && !go.d_moments) return;
    constexpr double kHalfC = 0.5 * 0.299792458;  // d z* / d delay [um/fs]
    SampleCoords sc;
    sample_coords(sp, P.key0, P.key1, i, sc);
    const double *nrm = sc.n;
    const double z = sc.z;
    const double xc = fma(sc.thx, 0.5 * z, sc.x), yc = fma(sc.thy, 0.5 * z, sc.y);
    const double zstar = fma(0.5, z, sp.z_delay);
    const SpD<double> d0 = spatial_d(xc, yc, zstar, sp.inv_w0sq, sp.inv_zR, sqrt(sp.inv_w0sq));
    const double aeff = sp.a0 * d0.S;
    double da[kGradParams];
    da[0] = d0.S;
    da[1] = aeff * d0.Lw;
    da[2] = aeff * d0.Lx;
    da[3] = aeff * d0.Ly;
    da[4] = aeff * kHalfC * d0.Lz;
    da[5] = 0.0;
    da[6] = 0.0;
    da[7] = aeff * (0.5 * z) * fma(1e-3 * nrm[4], d0.Lx, 1e-3 * nrm[5] * d0.Ly);
    const double thx = 1e3 * sc.thx, thy = 1e3 * sc.thy;
    const double s2p = fmax(s2, 0.0), sigf = sqrt(s2p);
    const double C = 1e3 * P.c_theta * 0.79788456080286535588;
    const double q = C * C / (mu * mu * mu * mu);
    const double sig_th = sqrt(q * aeff * aeff * s2p);
    // dL = Lmu dmu + Ls2 dsig2^+ + Lx dtheta_x + Ly dtheta_y + Lq dsig_th^2
    //      + La da0eff + Lg dgamma0,i
    double Lmu = 0.0, Ls2 = 0.0, Lx = 0.0, Ly = 0.0, Lq = 0.0, La = 0.0, Lg = 0.0;
    if (go.d_angle) {
        double lv, ls;
        law_sensitivity(thx, sig_th * sig_th, P.deposit, P.ksig_bins, sp.th_lo, sp.th_w, sp.n_th,
                        go.d_angle, lv, ls);
        Lx += lv;
        Lq += ls;
    }
    if (go.d_moments) {
        const double *u = go.d_moments, *M = go.moments;
        const double iW = 1.0 / (double)sp.n_samples;
        Lmu += u[1] * iW;
        if (M[2] > 0.0) {
            Lmu += u[2] * (mu - M[1]) * iW / M[2];
            Ls2 += u[2] * 0.5 * iW / M[2];
        }
        Lx += u[3] * iW;
        if (M[4] > 0.0) {
            Lx += u[4] * thx * iW / M[4];
            Lq += u[4] * 0.5 * iW / M[4];
        }
        Ly += u[5] * iW;
        if (M[6] > 0.0) Ly += u[6] * thy * iW / M[6];
        La += u[7] * iW;
        Lmu -= u[9] * iW / sc.g0;
        Lg += u[9] * iW * mu / (sc.g0 * sc.g0);
        if (sigf > 0.0) Ls2 += u[10] * iW * 0.5 / sigf;
    }
    const double a2 = aeff * aeff;
#pragma unroll
    for (int p = 0; p < kGradParams; ++p) {
        const double ds2p = s2 > 0.0 ? ds2[p] : 0.0;
        const double dq = q * fma(2.0 * aeff * s2p, da[p], fma(a2, ds2p, -4.0 * a2 * s2p * dmu[p] / mu));
        const double dth_x = p == 7 ? nrm[4] : 0.0, dth_y = p == 7 ? nrm[5] : 0.0;
        const double dg = p == 5 ? 1.0 : (p == 6 ? nrm[3] : 0.0);
        g[p] += Lmu * dmu[p] + Ls2 * ds2p + Lx * dth_x + Ly * dth_y + Lq * dq + La * da[p] +
                Lg * dg;
    }
}

// One step of the tangents of every direction: V' = A V + P1 d1 + Ph dh + P4 d4
// (d1, dh, d4: the direction's amplitude derivatives at the three stage
// points; the gamma0 direction GD has none).
template <class T, bool QUANTUM, int ND, int GD>
__device__ __forceinline__ void tangent_update(const StepLin<T, QUANTUM> &L, const T *da1,
                                               const T *dah, const T *da4, T *vm, T *vs) {
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
}

// FP64 steps of the mixed-precision tangent loop, from step j on for as long
// as some lane of the wavefront has chi above the threshold at a step start
// (the rule of the forward pass).  The state advances by the forward pass's
// FP64 step (FP64 amplitudes, the FP64 table read a wavefront at a time);
// the tangents by the FP32 step linearisation at the state rounded to FP32,
// with the FP32 amplitude derivatives and derivative table as in the FP32
// steps (the linearisation is rounded to FP32 either way), with the FP32
// loop's table cells carried from stage to stage as there.  A1, da1 and those
// cells carry over to the step the segment returns, the first not taken.
template <bool LOCAL, int ND, int GD>
__device__ __forceinline__ int tangent_fp64_segment(
    const BatchParams &P, const AdjPath<double> &pd, double S0d, const AdjPath<float> &pf,
    float S0f, const float *__restrict__ env32, const double *__restrict__ env64, double2 *stage,
    RadSrc<float> &rad, const Phys<float> &phf, int j, double &mu, double &s2, float *vm,
    float *vs, float *da1, StageAmp<float> &A1, float &cmx, float &chi_hi, double &chd) {
    const RadTabWave tabd(P.rad64, stage);
    const Phys<double> phd{P.K, P.CD, P.two_over_aS};
    const int N = P.n_steps;
    const double h = P.h, psi0 = -P.psi_max, ell = P.ell_per_psi;
    const float hf = (float)P.h, psi0f = (float)(-P.psi_max), ellf = (float)P.ell_per_psi;
    auto amp64 = [&](double psi, double fc) {
        if (LOCAL) {
            const double e = psi * ell;
            return pd.a0 * spatial(fma(pd.thx, e, pd.xc), fma(pd.thy, e, pd.yc), pd.zstar - e,
                                   pd.inv_w0sq, pd.inv_zR) * fc;
        }
        return pd.a0 * S0d * fc;
    };
    auto amp32 = [&](float psi, float fc, float &a, float *da) {
        if (LOCAL) {
            pf.amp(psi * ellf, fc, a, da);
        } else {
            const float Sf = S0f * fc;
            a = pf.a0 * Sf;
            da[0] = Sf;
            da[1] = 0.0f;
        }
    };
    double a1 = amp64(fma((double)j, h, psi0), env64[2 * j]);
    for (;;) {
        // tangents: FP32 linearisation at the rounded state
        const float psif = fmaf((float)j, hf, psi0f);
        float ahf, a4f, dah[ND], da4[ND];
        amp32(fmaf(0.5f, hf, psif), env32[2 * j + 1], ahf, dah);
        amp32(psif + hf, env32[2 * j + 2], a4f, da4);
        const StageAmp<float> Ah(ahf, phf), A4(a4f, phf);
        const StepLin<float, true> L =
            rk4_linear<float, true>((float)mu, (float)s2, A1, Ah, A4, hf, rad, chi_hi);
        tangent_update<float, true, ND, GD>(L, da1, dah, da4, vm, vs);
        A1 = A4;
#pragma unroll
        for (int d = 0; d < ND; ++d) da1[d] = da4[d];
        // state: the forward pass's FP64 step
        const double psi = fma((double)j, h, psi0);
        const double ah = amp64(fma(0.5, h, psi), env64[2 * j + 1]);
        const double a4 = amp64(psi + h, env64[2 * j + 2]);
        double dm, ds;
        rk4_increment<double, true, RadTabWave>(mu, s2, a1, ah, a4, h, phd, tabd, dm, ds, chd);
        mu += dm;
        s2 += ds;
        a1 = a4;
        ++j;
        if (j >= N) break;
        const double chi = phd.two_over_aS * mu * fabs(a1);
        cmx = fmaxf(cmx, (float)chi);
        if (!__any(chi > (double)P.chi_fp64)) break;
    }
    return j;
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
                                               const float *tab32, double2 *stage,
                                               SampleTangent &o, int &flags) {
    using T = typename std::conditional<PREC == PREC_F64, double, float>::type;
    // FP32 with FP64 steps where chi is above the threshold (quantum only;
    // stage: the wavefront's staging rows for the FP64 table, every lane
    // active)
    constexpr bool MIX = PREC == PREC_F32MIX;
    static_assert(!MIX || QUANTUM, "FP64 steps are a quantum-model option");
    constexpr int ND = LOCAL ? kDirLocal : kDirA0eff;
    constexpr int GD = LOCAL ? 5 : 1;  // the gamma0 direction: no amplitude forcing
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
    AdjSample smp;
    adj_sample(P, sp, i, smp);
    const double g0 = smp.sc.g0;
    AdjPath<T> pth = adj_path_cast<T>(smp.p);
    const T S0 = (T)smp.d0.S;
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
    double chd = 0.0;  // largest chi of the FP64 steps
    for (int j = 0; j < N;) {
        const T chi1 = A1.chi_per_mu * mu;
        cmx = fmaxf(cmx, (float)chi1);
        if constexpr (MIX) {
            if (__any(chi1 > P.chi_fp64)) {
                // FP64 steps while some lane of the wavefront has chi above
                // the threshold; the FP32 pair takes the state back at the
                // exit step (amplitude, derivatives and cells carry over)
                double mud = ((double)mu + (double)mu_lo) + g0_rest;
                double s2d = (double)s2 + (double)s2_lo;
                g0_rest = 0.0;  // now held by the state
                AdjSample sd;
                adj_sample(P, sp, opaque_index(i), sd);
                j = tangent_fp64_segment<LOCAL, ND, GD>(P, sd.p, sd.d0.S, pth, S0, env32, env64,
                                                        stage, rad, ph, j, mud, s2d, vm, vs, da1,
                                                        A1, cmx, chi_hi, chd);
                mu = (float)mud;
                mu_lo = (float)(mud - (double)mu);
                s2 = (float)s2d;
                s2_lo = (float)(s2d - (double)s2);
                continue;
            }
        }
        const T psi = fma((T)j, h, psi0);
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
        tangent_update<T, QUANTUM, ND, GD>(L, da1, dah, da4, vm, vs);
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
        ++j;
    }
    if constexpr (MIX) chi_hi = fmax(chi_hi, (T)chd);
    o.mu = ((double)mu + (double)mu_lo) + g0_rest;
    o.s2 = (double)s2 + (double)s2_lo;
    o.cmx = fmaxf(cmx, (float)(A1.chi_per_mu * mu));  // the end of the last step
    // the draw again for the chain (not carried through the loop)
    AdjSample se;
    adj_sample(P, sp, opaque_index(i), se);
    const double *nrm = se.sc.n;
    const SpD<double> &d0 = se.d0;
    const double z = se.sc.z;
    o.S0 = d0.S;
    o.g0 = se.sc.g0;
    o.thx = se.sc.thx;
    o.thy = se.sc.thy;
    if (QUANTUM && !((float)chi_hi < chi_top)) flags |= kFlagRange;
    if (!(o.mu > 0.0) || !isfinite(o.mu) || !isfinite(o.s2)) flags |= kFlagNonFinite;

    // ---- chain to the eight parameters ----
    constexpr double kHalfC = 0.5 * 0.299792458;  // d z* / d delay [um/fs]
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
// Occupancy: the FP32 tape pass is latency-bound and fits 168 VGPRs, three
// waves per SIMD; every other pass is held to 256 (two waves): the FP64 ones
// would otherwise take a few registers more and run one wave per SIMD, and
// the mixed ones are held to two by the FP64 table staging in LDS anyway.
// Mixed precision (FP64 steps): the work items are groups of kChiGroup
// samples taken in rounds in order of their chi scale; every lane of a
// wavefront runs, lanes past the group's end repeat its last sample.
template <int PREC, bool QUANTUM, bool LOCAL, bool TAPE>
__global__ __launch_bounds__(kPhaseBlock)
__attribute__((amdgpu_waves_per_eu((TAPE && PREC == PREC_F32) ? 3 : 2))) void tangent_kernel(
    BatchParams P, const float *__restrict__ env32, const double *__restrict__ env64) {
    constexpr bool kTab32 = QUANTUM && PREC != PREC_F64;
    constexpr bool kWave64 = PREC == PREC_F32MIX;
    __shared__ __align__(16) float tab32[kTab32 ? kCells32 * 4 * kDerivFuncs : 4];
    __shared__ double2 stage[kWave64 ? (kPhaseBlock / 64) * kStageChunks : 1];
    __shared__ int64_t slot;
    __shared__ double red[kPhaseBlock / 64][kGradParams];
    // FP64 steps where chi is high: the group's samples in order of their chi
    // scale, as the forward pass orders its items (chi_order)
    __shared__ float okey[kWave64 ? kChiGroup : 1];
    __shared__ unsigned short oidx[kWave64 ? kChiGroup : 1];
    double2 *wstage = stage + (kWave64 ? (threadIdx.x >> 6) * kStageChunks : 0);
    if (kTab32) {
        const float4 *src = reinterpret_cast<const float4 *>(P.rad32d);
        float4 *dst = reinterpret_cast<float4 *>(tab32);
        for (int k = threadIdx.x; k < kCells32 * kDerivFuncs; k += blockDim.x) dst[k] = src[k];
        __syncthreads();
    }
    // one sample: the tape entries and final state (TAPE), else its terms
    // of the gradient added to g
    auto one = [&](const ShotParams &sp, int s, int64_t i, bool live, double *g) {
        int flags = 0;
        SampleTangent o;
        tangent_sample<PREC, QUANTUM, LOCAL>(P, sp, i, env32, env64, tab32, wstage, o, flags);
        if (!live) return;  // ran for the wavefront's table reads only
        if (TAPE) {
            const int64_t k = sp.state_off + i;
            P.st.mu[k] = o.mu;
            P.st.s2[k] = o.s2;
            P.st.S0[k] = o.S0;
            P.st.g0[k] = o.g0;
            P.st.thx[k] = o.thx;
            P.st.thy[k] = o.thy;
            P.st.cmx[k] = o.cmx;
            double *tp = P.tape + k;
            const int64_t n = P.tape_n;
            tp[0] = o.mu;
            tp[n] = o.s2;
#pragma unroll
            for (int p = 0; p < kGradParams; ++p) {
                tp[(2 + p) * n] = o.dmu[p];
                tp[(2 + kGradParams + p) * n] = o.ds2[p];
            }
        } else if (!(flags & kFlagNonFinite)) {
            const ShotGrad &go = P.gouts[s];
            double gi[kGradParams];
#pragma unroll
            for (int p = 0; p < kGradParams; ++p) gi[p] = 0.0;
            if (go.d_energy) {
                double lv, ls;
                law_sensitivity(o.mu, o.s2, P.deposit, P.ksig_bins, sp.e_lo, sp.e_w, sp.n_e,
                                go.d_energy, lv, ls);
#pragma unroll
                for (int p = 0; p < kGradParams; ++p) gi[p] = fma(lv, o.dmu[p], ls * o.ds2[p]);
            }
            observable_sensitivity(P, sp, go, i, o.mu, o.s2, o.dmu, o.ds2, gi);
#pragma unroll
            for (int p = 0; p < kGradParams; ++p) g[p] += gi[p];
        }
        if (flags) atomicOr(&P.flags[s], flags);
    };
    for (;;) {
        const int64_t item = next_item(&P.queue[0], &slot);
        double g[kGradParams];
#pragma unroll
        for (int p = 0; p < kGradParams; ++p) g[p] = 0.0;
        if constexpr (kWave64) {
            if (item >= P.n_gitems) break;
            const int s = __builtin_amdgcn_readfirstlane(find_group_shot(P.shots, P.n_shots, item));
            const ShotParams &sp = P.shots[s];
            const int64_t base = (item - sp.gitem0) * kChiGroup;
            const int cnt = (int)min((int64_t)kChiGroup, sp.n_samples - base);
            chi_order<kChiGroup, kPhaseBlock>(sp, P.key0, P.key1, base, sp.n_samples, okey, oidx);
            for (int r = 0; r * kPhaseBlock < cnt; ++r) {
                const int rank = r * kPhaseBlock + (int)threadIdx.x;
                if (r * kPhaseBlock + (int)(threadIdx.x & ~63u) >= cnt) continue;  // whole wavefront
                const bool live = rank < cnt;
                one(sp, s, base + oidx[live ? rank : cnt - 1], live, g);
            }
        } else {
            if (item >= P.n_items) break;
            const int s = __builtin_amdgcn_readfirstlane(find_shot(P.shots, P.n_shots, item, false));
            const ShotParams &sp = P.shots[s];
            const int64_t i = (item - sp.item0) * kPhaseBlock + threadIdx.x;
            if (i < sp.n_samples) one(sp, s, i, true, g);
        }
        if (!TAPE) grad_item_reduce(P, item, g, red);
    }
}

// The adjoint from a tape: contraction of the recorded derivatives with the
// law sensitivities (memory-bound: 144 bytes a sample).
// OBS: some shot also has angle-histogram or moment weights (the memory-bound
// contraction of the energy terms alone keeps its small register budget).
// GROUPED: the tape of a pass with FP64 steps, summed over the groups of its
// tangent pass in the same order (rounds in chi order, each lane adding its
// samples' terms round by round, then the block reduction), so that the
// result equals the recomputing adjoint's bit for bit.
template <bool OBS, bool GROUPED>
__global__ __launch_bounds__(kPhaseBlock) void contract_kernel(BatchParams P) {
    // the energy-histogram weights of the block's current shot (n_e + 2
    // words), read from LDS by every edge of every sample's law
    extern __shared__ double wsh[];
    __shared__ int64_t slot;
    __shared__ double red[kPhaseBlock / 64][kGradParams];
    __shared__ float okey[GROUPED ? kChiGroup : 1];
    __shared__ unsigned short oidx[GROUPED ? kChiGroup : 1];
    int s_w = -1;  // the shot whose weights wsh holds (block-uniform)
    auto load_w = [&](int s, const ShotParams &sp) {
        if (s == s_w) return;
        // the previous item's reads ended at its reduction's barrier
        const double *W = P.gouts[s].d_energy;
        if (W)
            for (int k = threadIdx.x; k < sp.n_e + 2; k += blockDim.x) wsh[k] = W[k];
        __syncthreads();
        s_w = s;
    };
    auto one = [&](const ShotParams &sp, int s, int64_t i, double *g) {
        const int64_t n = P.tape_n;
        const double *t = P.tape + sp.state_off + i;
        const double mu = t[0], s2 = t[n];
        if (mu > 0.0 && isfinite(mu) && isfinite(s2)) {
            const ShotGrad &go = P.gouts[s];
            double dm[kGradParams], ds[kGradParams], gi[kGradParams];
#pragma unroll
            for (int p = 0; p < kGradParams; ++p) {
                dm[p] = t[(2 + p) * n];
                ds[p] = t[(2 + kGradParams + p) * n];
                gi[p] = 0.0;
            }
            if (go.d_energy) {
                double lv, ls;
                law_sensitivity(mu, s2, P.deposit, P.ksig_bins, sp.e_lo, sp.e_w, sp.n_e, wsh,
                                lv, ls);
#pragma unroll
                for (int p = 0; p < kGradParams; ++p) gi[p] = fma(lv, dm[p], ls * ds[p]);
            }
            if (OBS) observable_sensitivity(P, sp, go, i, mu, s2, dm, ds, gi);
#pragma unroll
            for (int p = 0; p < kGradParams; ++p) g[p] += gi[p];
        } else {
            atomicOr(&P.flags[s], kFlagNonFinite);
        }
    };
    for (;;) {
        const int64_t item = next_item(&P.queue[0], &slot);
        double g[kGradParams];
#pragma unroll
        for (int p = 0; p < kGradParams; ++p) g[p] = 0.0;
        if constexpr (GROUPED) {
            if (item >= P.n_gitems) break;
            const int s = __builtin_amdgcn_readfirstlane(find_group_shot(P.shots, P.n_shots, item));
            const ShotParams &sp = P.shots[s];
            const int64_t base = (item - sp.gitem0) * kChiGroup;
            const int cnt = (int)min((int64_t)kChiGroup, sp.n_samples - base);
            load_w(s, sp);
            chi_order<kChiGroup, kPhaseBlock>(sp, P.key0, P.key1, base, sp.n_samples, okey, oidx);
            for (int r = 0; r * kPhaseBlock < cnt; ++r) {
                const int rank = r * kPhaseBlock + (int)threadIdx.x;
                if (rank < cnt) one(sp, s, base + oidx[rank], g);
            }
        } else {
            if (item >= P.n_items) break;
            const int s = __builtin_amdgcn_readfirstlane(find_shot(P.shots, P.n_shots, item, false));
            const ShotParams &sp = P.shots[s];
            const int64_t i = (item - sp.item0) * kPhaseBlock + threadIdx.x;
            load_w(s, sp);
            if (i < sp.n_samples) one(sp, s, i, g);
        }
        grad_item_reduce(P, item, g, red);
    }
}

// One block per shot: fixed-order sum of the shot's item partials.
__global__ __launch_bounds__(256) void grad_finalize_kernel(BatchParams P) {
    const int s = blockIdx.x;
    const ShotParams &sp = P.shots[s];
    const ShotGrad &so = P.gouts[s];
    // partials per group with FP64 steps, else per phase item
    const bool grouped = P.prec == PREC_F32MIX;
    const int64_t ni = grouped ? (sp.n_samples + kChiGroup - 1) / kChiGroup
                               : (sp.n_samples + kPhaseBlock - 1) / kPhaseBlock;
    const int64_t first = grouped ? sp.gitem0 : sp.item0;
    __shared__ double tree[256];
    for (int p = 0; p < kGradParams; ++p) {
        double acc = 0.0;
        for (int64_t b = threadIdx.x; b < ni; b += blockDim.x)
            acc += P.partials[(size_t)(first + b) * kGradParams + p];
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

// FP64-shadow report of each shot: the batch is the FP64 view pass, the FP32
// view pass's gradients sit span doubles before its own (span 0: zeros).
__global__ __launch_bounds__(256) void grad_shadow_kernel(BatchParams P, int64_t span) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P.n_shots) return;
    const ShotGrad &so = P.gouts[s];
    double *o = so.errors;
    if (!o) return;
    if (span == 0) {
        for (int q = 0; q < 1 + 2 * kGradParams; ++q) o[q] = 0.0;
        return;
    }
    o[0] = (double)P.shots[s].n_samples;
    for (int p = 0; p < kGradParams; ++p) {
        const double g64 = so.grad[p], g32 = so.grad[p - span];
        o[1 + p] = g32 - g64;
        o[1 + kGradParams + p] = g64;
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
// Launchers
// ===========================================================================
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
    if (prec == PREC_F32MIX && q)  // FP64 steps are a quantum-model option
        return l ? tangent_ptr<PREC_F32MIX, true, true, TAPE>()
                 : tangent_ptr<PREC_F32MIX, true, false, TAPE>();
    return q ? (l ? tangent_ptr<PREC_F32, true, true, TAPE>()
                  : tangent_ptr<PREC_F32, true, false, TAPE>())
             : (l ? tangent_ptr<PREC_F32, false, true, TAPE>()
                  : tangent_ptr<PREC_F32, false, false, TAPE>());
}

hipError_t launch_tangent(const BatchParams &p, const float *env32, const double *env64, int prec,
                          int rr, int amp, bool tape, hipStream_t s) {
    const void *fn = tape ? select_tangent<true>(prec, rr, amp) : select_tangent<false>(prec, rr, amp);
    const bool grouped = prec == PREC_F32MIX && rr == 1;
    int grid = 0;
    hipError_t e = resident_grid(fn, kPhaseBlock, 0, grouped ? p.n_gitems : p.n_items, &grid);
    if (e != hipSuccess) return e;
    BatchParams pc = p;
    const float *e32 = env32;
    const double *e64 = env64;
    void *args[] = {&pc, &e32, &e64};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kPhaseBlock), args, 0, s);
}

hipError_t launch_contract(const BatchParams &p, bool obs, int max_ne, hipStream_t s) {
    // a tape of a pass with FP64 steps is summed over that pass's groups
    const bool grouped = p.prec == PREC_F32MIX;
    const void *fn =
        grouped ? (obs ? reinterpret_cast<const void *>(&contract_kernel<true, true>)
                       : reinterpret_cast<const void *>(&contract_kernel<false, true>))
                : (obs ? reinterpret_cast<const void *>(&contract_kernel<true, false>)
                       : reinterpret_cast<const void *>(&contract_kernel<false, false>));
    const size_t lds = (size_t)(max_ne + 2) * sizeof(double);  // at most 32 KB (n_e <= 4096)
    int grid = 0;
    hipError_t e = resident_grid(fn, kPhaseBlock, lds, grouped ? p.n_gitems : p.n_items, &grid);
    if (e != hipSuccess) return e;
    BatchParams pc = p;
    void *args[] = {&pc};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kPhaseBlock), args, lds, s);
}

hipError_t launch_grad_finalize(const BatchParams &p, hipStream_t s) {
    grad_finalize_kernel<<<p.n_shots, 256, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_grad_shadow(const BatchParams &p, int64_t span, hipStream_t s) {
    grad_shadow_kernel<<<(p.n_shots + 255) / 256, 256, 0, s>>>(p, span);
    return hipGetLastError();
}

hipError_t launch_radiation_derivs(const float *rad32d, const double *rad64d, int prec, int64_t n,
                                   const double *chi, double *out, int *flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    rad_derivs_kernel<<<(unsigned)blocks, 256, 0, s>>>(rad32d, rad64d, prec, n, chi, out, flags);
    return hipGetLastError();
}

}  // namespace qs
