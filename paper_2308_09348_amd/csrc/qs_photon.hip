// qs_photon.hip -- the approximate photon spectrum of Sec. 4: the LCFA number
// CDF table, the emission kernel and the per-shot contraction.
#include "qs_device.h"

namespace qs {

// ===========================================================================
// Photon spectrum (Sec. 4).  Along each sample's trajectory every RK4 stage
// (weights h/6, h/3, h/3, h/6) emits the LCFA spectrum of its state:
//   d2N / (dpsi dxi) = C_ph F(xi, chi) / mu,   C_ph = alpha a_S / (2 sqrt3 pi),
// so that a stage adds c h C_ph (chi / mu) [Phi(e_{k+1}/mu; chi) -
// Phi(e_k/mu; chi)] / chi to photon-energy bin k, Phi(xi; chi) = Int_0^xi F.
// Evaluating Phi at every bin edge for every stage would cost the bin count
// per stage, so each stage instead deposits its weight c (chi / mu) =
// c 2|a| / a_S, bilinearly, into an emission grid over (u, t) = (ln chi,
// sqrt(mu)) kept in LDS in fixed point (order-independent sums); a finalize
// kernel then evaluates Phi / chi once per grid node and bin edge.
//
// Bilinear deposit followed by evaluation at the nodes is the bin content f
// integrated against the emission density smoothed by a tent of one node
// spacing in each direction: to second order, f + (du^2/12) f_uu + (dt^2/12)
// f_tt.  The contraction removes that term by weighting the nodes with the
// deposit convolved with [-1/12, 7/6, -1/12] along each axis (the inverse of
// the tent's [1/12, 5/6, 1/12] node average to second order), leaving an
// error of fourth order in the spacings.  The emission density in t is set
// by the beam's energy spread near the initial energy, where t = sqrt(mu)
// gives finer columns than ln mu over the same range.  The host keeps the
// outer columns empty and the row above the largest chi; the row below the
// grid's first is a table row too, so the convolution needs no node the
// table lacks.
//
// Stages whose chi lies below the grid emit photons below the first bin (the
// host sizes the grid so): they add only their photon number, (5 pi / 2) chi
// (1 - 8 chi / (5 sqrt3)) per unit C_ph c / mu, to the lowest bin.  The
// emitted photon energy itself, c h (-A) summed over the stages (A: the
// drift), is accumulated exactly.
// ===========================================================================
__device__ __forceinline__ double ph_dz() { return cbrt(kPhYMax) / kPhNZ; }
__device__ __forceinline__ float ph_ln(float x) {
    return __builtin_amdgcn_logf(x) * 0.69314718055994530942f;
}
__device__ __forceinline__ float ph_ln(double x) { return (float)log(x); }
// Grid coordinates need a few 1e-7 relative: the hardware square root (1 ulp).
__device__ __forceinline__ float ph_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// ln of the geometric mean of two stage energies from their product.  Like
// the deposit below, evaluated without contracting a product into a later
// sum, so that every instantiation of the photon step (FP64 pass, FP64
// steps of the mixed pass) places a deposit at the same grid coordinates.
__device__ __forceinline__ float ph_half_ln(float pm) {
#pragma clang fp contract(off)
    return 0.5f * ph_ln(pm);
}

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

// Deposit of emission weight D (in units of 2 a0 / a_S per unit h) at
// u = ln chi = la + lm (la = ln(2 |a| / a_S), lm = ln mu) and t = sqrt(mu),
// bilinear in (u, t); below the grid only the photon number is kept.
struct PhotAcc {
    double e_ph, soft;
    int flags;
    // Sec. 5.1 angular sums (in units that the finalize kernel scales):
    // sum c |a| Phi(1; chi)/chi (photon number), the same times theta_x^2 and
    // theta_y^2; sum c (-A) (energy), the same times theta_x^2, theta_y^2
    double nn, nx, ny, ee, ex, ey;
};

// Phi(1; chi) / chi, the LCFA photon number over all energies per unit chi,
// from the number CDF table's last node on each row (z_max Phi/(chi z) at
// y = kPhYMax, beyond which the spectrum is below 1e-34), cubic in ln chi; below
// the first row the small-chi series (5 pi / 2)(1 - 8 chi / (5 sqrt3)).
__device__ __forceinline__ float ph_total(const float *tot, float chi) {
    const float s = (__logf(chi) - (float)kPhU0) * (float)(1.0 / kPhDu);
    if (!(s > 0.0f)) return 7.85398163397448310f * fmaf(-0.92376043070340122f, chi, 1.0f);
    const int i = min(max((int)s - 1, 0), kPhRows - 4);
    const float t = s - (float)i;
    const float w0 = -(t - 1.0f) * (t - 2.0f) * (t - 3.0f) * (1.0f / 6.0f);
    const float w1 = t * (t - 2.0f) * (t - 3.0f) * 0.5f;
    const float w2 = -t * (t - 1.0f) * (t - 3.0f) * 0.5f;
    const float w3 = t * (t - 1.0f) * (t - 2.0f) * (1.0f / 6.0f);
    return fmaf(w0, tot[i], fmaf(w1, tot[i + 1], fmaf(w2, tot[i + 2], w3 * tot[i + 3])));
}

// Phi(1; chi) / chi in FP64 from the rows, as ph_total does in FP32.
__device__ double ph_total64(const double *phtab, double chi) {
    const double s = (log(chi) - kPhU0) * (1.0 / kPhDu);
    if (!(s > 0.0)) return 7.85398163397448310 * (1.0 - 0.92376043070340122 * chi);
    const int i = min(max((int)s - 1, 0), kPhRows - 4);
    const double t = s - (double)i;
    const double w[4] = {-(t - 1.0) * (t - 2.0) * (t - 3.0) / 6.0, t * (t - 2.0) * (t - 3.0) / 2.0,
                         -t * (t - 1.0) * (t - 3.0) / 2.0, t * (t - 1.0) * (t - 2.0) / 6.0};
    double v = 0.0;
    for (int k = 0; k < 4; ++k)
        v = fma(w[k], cbrt(kPhYMax) * phtab[(size_t)(i + k) * (kPhNZ + 1) + kPhNZ], v);
    return v;
}

// The cubic in the cell coordinate of each FP32 radiation-table cell through
// Phi(1; chi) / chi at the cell's four Chebyshev nodes (from the rows): the
// FP32 photon kernel reads it with the cell it already holds for g and h.
__global__ void ph_cell_kernel(const double *phtab, float *cells) {
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= kCells32) return;
    double coef[4] = {0.0, 0.0, 0.0, 0.0};
    for (int m = 0; m < 4; ++m) {
        const double v = ph_total64(phtab, cell_chi(cell, cheb_node(m), kSB32));
        double l[4];
        cheb_basis(m, l);
        for (int k = 0; k < 4; ++k) coef[k] = fma(v, l[k], coef[k]);
    }
    for (int k = 0; k < 4; ++k) cells[4 * cell + k] = (float)coef[k];
}

// One stage's share of the angular sums: weight c (the stage's quadrature
// weight over h), amplitude a, mean energy mu, drift A; the emission angle is
// theta_x + a/mu in x and theta_y in y, plus a 1/mu cone in each plane.
template <class T>
struct AngStep {
    T n, nx, ny, e, ex, ey;
    // nf: Phi(1; chi) / chi at the stage's chi
    __device__ __forceinline__ void add(T c, T a, T mu, T A, T thx, T thy, T nf) {
        const T aa = fabs(a);
        T imu;
        if constexpr (sizeof(T) == 4) {
            imu = __builtin_amdgcn_rcpf(mu);  // about one ulp
        } else {
            // the hardware reciprocal refined by two Newton steps (each
            // squares the relative error): FP64 rounding for mu >= 1
            imu = __builtin_amdgcn_rcp(mu);
            imu = fma(fma(-mu, imu, 1.0), imu, imu);
            imu = fma(fma(-mu, imu, 1.0), imu, imu);
        }
        const T tx = fma(a, imu, thx), cone = imu * imu;
        const T x2 = fma(tx, tx, cone), y2 = fma(thy, thy, cone);
        const T dn = c * aa * nf;
        const T de = -c * A;
        n += dn;
        nx = fma(dn, x2, nx);
        ny = fma(dn, y2, ny);
        e += de;
        ex = fma(de, x2, ex);
        ey = fma(de, y2, ey);
    }
};

// LDS row stride of the emission grid: one word more than a row, so that
// nodes of one column in neighbouring rows fall in different LDS banks (the
// lanes of a wavefront deposit at similar energies in neighbouring rows)
constexpr int kPhLdsRow = kPhNV + 1;
constexpr int kPhLdsNodes = kPhNU * kPhLdsRow;

// Weights in units of 2^-24 (kPhScale): D <= 2/3, so every node weight is
// below 2^24 and its FP32 product is within half a unit of the exact one
// before rounding to an integer; the grid words sum them in any order alike.
__device__ __forceinline__ void ph_deposit(float D, float lm, float t, float la, float chi,
                                           const ShotPhot &sp, unsigned long long *grid,
                                           PhotAcc &acc) {
#pragma clang fp contract(off)
    const float ru = (la + lm - (float)(kPhU0 + sp.r_lo * kPhDu)) * (float)(1.0 / kPhDu);
    if (ru < 0.0f) {  // below the grid: photon number only
        acc.soft += (double)D * (1.0 - 0.92376043070340122 * (double)chi);
        return;
    }
    float fu = ru, fv = (t - sp.t_lof) * sp.inv_dt;
    if (!(fu <= (float)(sp.nu - 1)) || !(fv >= 0.0f) || !(fv <= (float)(sp.nv - 1))) {
        acc.flags |= kFlagRange;
        fu = fminf(fmaxf(fu, 0.0f), (float)(sp.nu - 1));
        fv = fminf(fmaxf(fv, 0.0f), (float)(sp.nv - 1));
    }
    const int n = min((int)fu, sp.nu - 2), m = min((int)fv, sp.nv - 2);
    const float du = fu - (float)n, dv = fv - (float)m;
    const float q = D * (float)kPhScale;
    const float qu = q * du, ql = q - qu;  // the two rows' shares
    unsigned long long *g = grid + n * kPhLdsRow + m;
    atomicAdd(g, (unsigned long long)(unsigned int)rintf(ql - ql * dv));
    atomicAdd(g + 1, (unsigned long long)(unsigned int)rintf(ql * dv));
    atomicAdd(g + kPhLdsRow, (unsigned long long)(unsigned int)rintf(qu - qu * dv));
    atomicAdd(g + kPhLdsRow + 1, (unsigned long long)(unsigned int)rintf(qu * dv));
}

// Radiation functions per stage in the forward table's combinations
// T1 = g, T2 = 2g + chi g', T3 = g + 2 chi g' + chi^2 g''/2, T4 = h.  FP32:
// the LDS table read at stages 2 and 4 only, stage 3 and the next stage 1
// reusing those cells; FP64: the global table at every stage.
template <class T>
struct FwdRad;
// With ncell (FP32 angular moments) the cells also bring the photon-number
// cubic of the same cell: num() gives Phi(1; chi) / chi of the last stage.
template <>
struct FwdRad<float> {
    const float *tab;
    const float4 *ncell = nullptr;
    RadCell32 carry, mid;
    float4 ncarry, nmid;
    float nf = 0.0f;
    __device__ __forceinline__ void init(float chi) { rad_lookup32(tab, chi, carry, ncell, &ncarry); }
    __device__ __forceinline__ void number(const RadCell32 &c, const float4 &q, float chi) {
        if (ncell) {
            const float t = fmaf(chi, c.tw, c.ts);
            nf = fmaf(t, fmaf(t, fmaf(t, q.w, q.z), q.y), q.x);
        }
    }
    __device__ __forceinline__ void s1(float chi, float *t) {
        rad_cell_eval(carry, chi, t[0], t[1], t[2], t[3]);
        number(carry, ncarry, chi);
    }
    __device__ __forceinline__ void s2(float chi, float *t) {
        rad_lookup32(tab, chi, mid, ncell, &nmid);
        rad_cell_eval(mid, chi, t[0], t[1], t[2], t[3]);
        number(mid, nmid, chi);
    }
    __device__ __forceinline__ void s3(float chi, float *t) {
        rad_cell_eval(mid, chi, t[0], t[1], t[2], t[3]);
        number(mid, nmid, chi);
    }
    __device__ __forceinline__ void s4(float chi, float *t) {
        rad_lookup32(tab, chi, carry, ncell, &ncarry);
        rad_cell_eval(carry, chi, t[0], t[1], t[2], t[3]);
        number(carry, ncarry, chi);
    }
};
template <>
struct FwdRad<double> {
    const double *tab;
    double nf = 0.0;  // unused: the FP64 pass takes the number from the rows
    __device__ __forceinline__ void init(double) {}
    __device__ __forceinline__ void ev(double chi, double *t) {
        double g, G1, G2, hq;
        rad_eval64(tab, chi, g, G1, G2, hq);
        t[0] = g;
        t[1] = fma(2.0, g, G1);
        t[2] = fma(0.5, G2, fma(2.0, G1, g));
        t[3] = hq;
    }
    __device__ __forceinline__ void s1(double chi, double *t) { ev(chi, t); }
    __device__ __forceinline__ void s2(double chi, double *t) { ev(chi, t); }
    __device__ __forceinline__ void s3(double chi, double *t) { ev(chi, t); }
    __device__ __forceinline__ void s4(double chi, double *t) { ev(chi, t); }
};
// The same values from the FP64 table read a wavefront at a time
// (RadTabWave; every lane of the wavefront active): the FP64 steps of
// mixed-precision passes.
struct FwdRadWave {
    RadTabWave tw;
    double nf = 0.0;  // unused: FP64 steps take the number from the rows
    __device__ __forceinline__ FwdRadWave(const double *tab, double2 *stage) : tw(tab, stage) {}
    __device__ __forceinline__ void init(double) {}
    __device__ __forceinline__ void ev(double chi, double *t) {
        double g, G1, G2, hq;
        tw.eval(chi, g, G1, G2, hq);
        t[0] = g;
        t[1] = fma(2.0, g, G1);
        t[2] = fma(0.5, G2, fma(2.0, G1, g));
        t[3] = hq;
    }
    __device__ __forceinline__ void s1(double chi, double *t) { ev(chi, t); }
    __device__ __forceinline__ void s2(double chi, double *t) { ev(chi, t); }
    __device__ __forceinline__ void s3(double chi, double *t) { ev(chi, t); }
    __device__ __forceinline__ void s4(double chi, double *t) { ev(chi, t); }
};

// One stage: slopes and the drift A (the photon energy per unit phase is -A).
template <class T, bool QUANTUM, int S, class R = FwdRad<T>>
__device__ __forceinline__ void photon_stage(T mu, T s2, T a, const Phys<T> &ph, R &rad,
                                             T &dmu, T &ds2, T &A, T &chi_hi, T &nf) {
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
    T t[4];
    if (S == 1) rad.s1(chi, t);
    if (S == 2) rad.s2(chi, t);
    if (S == 3) rad.s3(chi, t);
    if (S == 4) rad.s4(chi, t);
    nf = (T)rad.nf;
    A = -u * mu2 * t[0];
    dmu = -u * fma(mu2, t[0], s2 * t[2]);
    ds2 = fma(T(-2) * u * mu * s2, t[1], ph.CD * aa * a2 * mu2 * mu2 * t[3]);
}

// Per-sample constants of the photon pass in precision T.
template <class T>
struct PhotCtx {
    const T *env;
    Path<T> pt;
    Phys<T> ph;
    T a0, a0S0, h, psi0, ell, thx, thy;
    float inv_a0, tas;
    bool local, mid, angles, cell_number;
    bool live;  // the lane's sample is real (else it runs for the wavefront's table reads only)
    const float4 *ncell = nullptr;  // photon-number cubics of the FP32 cells (FP64 steps of mixed passes)
};

// Phi(1; chi) / chi from the photon-number cubic of the FP32 radiation-table
// cell of chi (the index map of rad_lookup32; below the first octave its cubic
// extrapolated down to chi = 0).
__device__ __forceinline__ float ph_number32(const float4 *ncell, float chi) {
    const float xc = fminf(fmaxf(chi, 0x1p-20f), 0x1.fffffep7f);
    const uint32_t b = __float_as_uint(xc);
    const uint32_t c = ((b - ((uint32_t)(127 + kEMin) << 23)) >> (23 - kSB32)) + 1u;
    const float tw = __uint_as_float((uint32_t)(254 + kSB32 - (int)(b >> 23)) << 23);
    const float ts = -__uint_as_float(b & ~((1u << (23 - kSB32)) - 1)) * tw;
    const float4 q = ncell[c];
    const float t = fmaf(chi, tw, ts);
    return fmaf(t, fmaf(t, fmaf(t, q.w, q.z), q.y), q.x);
}

// The state carried from step to step (mu_lo, s2_lo: the FP32 pairs' lower
// parts, unused in FP64): the amplitude factors a0 S at psi_j (and psi_{j+1}
// with the quadratic midpoint), the previous step's stage-4 energy.
template <class T>
struct PhotState {
    T mu, mu_lo, s2, s2_lo, aS_prev, aS_next, m4_prev, chi_hi;
};

// Step j of the photon pass: the four RK4 stages with their emission, the
// deposits of stage 1 with the previous step's stage 4 (same amplitude) and
// of stages 2 and 3, the emitted energy and the Sec. 5.1 angular sums.
// ANG32: the angular sums' terms in FP32 with the photon number from the FP32
// cells' cubics (the FP64 steps of a mixed-precision pass, whose angular
// moments are held to the FP32 pass's bar; the FP64 pass takes them in FP64).
template <class T, bool QUANTUM, class R = FwdRad<T>, bool ANG32 = false>
__device__ __forceinline__ void photon_step(const PhotCtx<T> &c, const ShotPhot &pp,
                                            const float *tot, int j, PhotState<T> &st, R &rad,
                                            unsigned long long *grid, PhotAcc &acc) {
    const T h = c.h, hh = T(0.5) * h;
    const T c16 = T(1.0 / 6.0), c13 = T(1.0 / 3.0);
    const T psi = fma((T)j, h, c.psi0);
    T aSh = c.a0S0, aS4 = c.a0S0;
    if (c.mid) {
        const T aS_far = c.a0 * c.pt.S(fma((T)(j + 2), h, c.psi0) * c.ell);
        aS4 = st.aS_next;
        aSh = fma(T(0.375), st.aS_prev, fma(T(0.75), aS4, T(-0.125) * aS_far));
        st.aS_next = aS_far;
    } else if (c.local) {
        aSh = c.a0 * c.pt.S(fma(T(0.5), h, psi) * c.ell);
        aS4 = c.a0 * c.pt.S((psi + h) * c.ell);
    }
    const T a1 = st.aS_prev * c.env[2 * j], ah = aSh * c.env[2 * j + 1], a4 = aS4 * c.env[2 * j + 2];
    const T mu = st.mu, s2 = st.s2;
    // stage 4 of the previous step with stage 1 of this one (same
    // amplitude): one deposit at the geometric mean of the two energies
    if (j > 0 && c.live) {
        const float aa = fabsf((float)a1);
        if (aa > 0.0f) {
            const float pm = (float)st.m4_prev * (float)mu;
            ph_deposit((float)c13 * aa * c.inv_a0, ph_half_ln(pm), ph_sqrt(ph_sqrt(pm)),
                       ph_ln(c.tas * aa), c.tas * (float)mu * aa, pp, grid, acc);
        }
    }
    T k1m, k1s, A1, k2m, k2s, A2, k3m, k3s, A3, k4m, k4s, A4;
    T n1 = T(0), n2 = T(0), n3 = T(0), n4 = T(0);
    photon_stage<T, QUANTUM, 1, R>(mu, s2, a1, c.ph, rad, k1m, k1s, A1, st.chi_hi, n1);
    const T m2 = fma(hh, k1m, mu);
    photon_stage<T, QUANTUM, 2, R>(m2, fma(hh, k1s, s2), ah, c.ph, rad, k2m, k2s, A2, st.chi_hi, n2);
    const T m3 = fma(hh, k2m, mu);
    photon_stage<T, QUANTUM, 3, R>(m3, fma(hh, k2s, s2), ah, c.ph, rad, k3m, k3s, A3, st.chi_hi, n3);
    const T m4 = fma(h, k3m, mu);
    photon_stage<T, QUANTUM, 4, R>(m4, fma(h, k3s, s2), a4, c.ph, rad, k4m, k4s, A4, st.chi_hi, n4);
    if (c.live) acc.e_ph += (double)(h * -(c16 * (A1 + A4) + c13 * (A2 + A3)));
    if constexpr (ANG32) {
        if (c.angles && c.live) {
            auto num = [&](T m, T a) {
                const float aa = fabsf((float)a);
                return aa > 0.0f ? ph_number32(c.ncell, c.tas * (float)m * aa) : 0.0f;
            };
            const float thx = (float)c.thx, thy = (float)c.thy;
            AngStep<float> an{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            an.add((float)c16, (float)a1, (float)mu, (float)A1, thx, thy, num(mu, a1));
            an.add((float)c13, (float)ah, (float)m2, (float)A2, thx, thy, num(m2, ah));
            an.add((float)c13, (float)ah, (float)m3, (float)A3, thx, thy, num(m3, ah));
            an.add((float)c16, (float)a4, (float)m4, (float)A4, thx, thy, num(m4, a4));
            acc.nn += an.n;
            acc.nx += an.nx;
            acc.ny += an.ny;
            acc.ee += an.e;
            acc.ex += an.ex;
            acc.ey += an.ey;
        }
    } else if (c.angles && c.live) {
        if (!c.cell_number) {  // from the rows
            auto rows = [&](T m, T a) {
                const float aa = fabsf((float)a);
                return aa > 0.0f ? (T)ph_total(tot, c.tas * (float)m * aa) : T(0);
            };
            n1 = rows(mu, a1);
            n2 = rows(m2, ah);
            n3 = rows(m3, ah);
            n4 = rows(m4, a4);
        }
        AngStep<T> an{T(0), T(0), T(0), T(0), T(0), T(0)};
        an.add(c16, a1, mu, A1, c.thx, c.thy, n1);
        an.add(c13, ah, m2, A2, c.thx, c.thy, n2);
        an.add(c13, ah, m3, A3, c.thx, c.thy, n3);
        an.add(c16, a4, m4, A4, c.thx, c.thy, n4);
        acc.nn += an.n;
        acc.nx += an.nx;
        acc.ny += an.ny;
        acc.ee += an.e;
        acc.ex += an.ex;
        acc.ey += an.ey;
    }
    if (c.live) {  // stages 2 and 3 (same amplitude)
        const float aa = fabsf((float)ah);
        if (aa > 0.0f) {
            const float pm = (float)m2 * (float)m3;
            ph_deposit(2.0f * (float)c13 * aa * c.inv_a0, ph_half_ln(pm), ph_sqrt(ph_sqrt(pm)),
                       ph_ln(c.tas * aa), c.tas * (float)m2 * aa, pp, grid, acc);
        }
    }
    const T h6 = h * c16;
    const T dm = h6 * (k1m + T(2) * (k2m + k3m) + k4m);
    const T ds = h6 * (k1s + T(2) * (k2s + k3s) + k4s);
    if constexpr (sizeof(T) == 8) {
        st.mu += dm;
        st.s2 += ds;
    } else {
        comp_add(st.mu, st.mu_lo, dm);
        comp_add(st.s2, st.s2_lo, ds);
    }
    st.m4_prev = m4;
    st.aS_prev = aS4;
}

template <int PREC, bool QUANTUM, bool LOCAL>
__device__ __forceinline__ void photon_sample(const BatchParams &P, const ShotParams &sp,
                                              const ShotPhot &pp, int64_t i,
                                              const float *__restrict__ env32,
                                              const double *__restrict__ env64,
                                              const float *tab32, unsigned long long *grid,
                                              const float *tot, const float4 *ncell,
                                              double2 *stage, bool live, PhotAcc &acc,
                                              double &loss) {
    using T = typename std::conditional<PREC == PREC_F64, double, float>::type;
    // FP32 with FP64 steps where chi is above the threshold (quantum only;
    // every lane of the wavefront runs, live says whether the lane's sample
    // is real and deposits, stage holds the wavefront's FP64 table rows)
    constexpr bool MIX = PREC == PREC_F32MIX;
    static_assert(!MIX || QUANTUM, "FP64 steps are a quantum-model option");
    const bool angles = pp.angles != nullptr;
    const int N = P.n_steps;
    const bool local = LOCAL && !sp.plane_wave;

    SampleCoords sc;
    sample_coords(sp, P.key0, P.key1, i, sc);
    const double x = sc.x, y = sc.y, z = sc.z;
    const double g0 = sc.g0;
    const double thx = sc.thx;
    const double thy = sc.thy;
    Path<double> pd;
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
    const double S0 = sp.plane_wave ? 1.0 : pd.S(0.0);

    PhotCtx<T> c;
    if constexpr (PREC == PREC_F64)
        c.env = env64;
    else
        c.env = env32;
    c.pt.xc = (T)pd.xc;
    c.pt.yc = (T)pd.yc;
    c.pt.thx = (T)thx;
    c.pt.thy = (T)thy;
    c.pt.zstar = (T)pd.zstar;
    c.pt.inv_w0sq = (T)sp.inv_w0sq;
    c.pt.inv_zR = (T)sp.inv_zR;
    c.pt.mode = sp.mode;
    c.pt.mm = sp.mode_m;
    c.pt.mn = sp.mode_n;
    c.pt.inv_norm = (T)sp.mode_inv_norm;
    c.ph = Phys<T>{(T)P.K, (T)P.CD, (T)P.two_over_aS};
    c.a0 = (T)sp.a0;
    c.a0S0 = (T)(sp.a0 * S0);
    c.h = (T)P.h;
    c.psi0 = (T)(-P.psi_max);
    c.ell = (T)P.ell_per_psi;
    c.thx = (T)thx;
    c.thy = (T)thy;
    c.inv_a0 = sp.a0 > 0.0 ? (float)(1.0 / sp.a0) : 0.0f;
    c.tas = (float)P.two_over_aS;
    c.local = local;
    // FP32 with fine steps: one spatial factor a step, the midpoint from the
    // quadratic through three step points (as in the phase kernel)
    c.mid = PREC != PREC_F64 && local && sp.mid_interp;
    c.angles = angles;
    // FP32 quantum passes take the photon number from the radiation cells
    c.cell_number = PREC != PREC_F64 && QUANTUM && angles;
    c.live = MIX ? live : true;

    FwdRad<T> rad;
    if constexpr (PREC == PREC_F64) {
        rad.tab = P.rad64;
    } else {
        rad.tab = tab32;
        if (c.cell_number) rad.ncell = ncell;
    }
    PhotState<T> st;
    st.mu = (T)g0;
    st.mu_lo = T(0);
    st.s2 = T(0);
    st.s2_lo = T(0);
    st.chi_hi = T(0);
    st.m4_prev = T(0);  // the previous step's stage-4 state, deposited with this step's stage 1
    double g0_rest = 0.0;
    if constexpr (PREC != PREC_F64) {
        st.mu_lo = (T)(g0 - (double)st.mu);
        g0_rest = (g0 - (double)st.mu) - (double)st.mu_lo;
    }
    st.aS_prev = local ? c.a0 * c.pt.S(c.psi0 * c.ell) : c.a0S0;
    st.aS_next = c.mid ? c.a0 * c.pt.S((c.psi0 + c.h) * c.ell) : c.a0S0;
    if (QUANTUM) rad.init(c.ph.two_over_aS * st.mu * fabs(st.aS_prev * c.env[0]));
    // the first stage of the first step deposits alone
    if (c.live) {
        const float aa = fabsf((float)(st.aS_prev * c.env[0]));
        if (aa > 0.0f)
            ph_deposit((1.0f / 6.0f) * aa * c.inv_a0, ph_ln((float)st.mu), ph_sqrt((float)st.mu),
                       ph_ln(c.tas * aa), c.tas * (float)st.mu * aa, pp, grid, acc);
    }
    double chd = 0.0;  // largest chi of the FP64 steps
    for (int j = 0; j < N;) {
        if constexpr (MIX) {
            const float chi1 = c.ph.two_over_aS * st.mu * fabsf(st.aS_prev * env32[2 * j]);
            if (__any(chi1 > P.chi_fp64)) {
                // FP64 steps while some lane of the wavefront has chi above
                // the threshold at a step start (the forward pass's rule);
                // the FP32 pair, amplitudes and cell are rebuilt at the exit
                PhotCtx<double> cd;
                cd.env = env64;
                cd.pt = pd;
                cd.ph = Phys<double>{P.K, P.CD, P.two_over_aS};
                cd.a0 = sp.a0;
                cd.a0S0 = sp.a0 * S0;
                cd.h = P.h;
                cd.psi0 = -P.psi_max;
                cd.ell = P.ell_per_psi;
                cd.thx = thx;
                cd.thy = thy;
                cd.inv_a0 = c.inv_a0;
                cd.tas = c.tas;
                cd.local = local;
                cd.mid = false;
                cd.angles = angles;
                cd.cell_number = false;
                cd.ncell = ncell;
                cd.live = c.live;
                PhotState<double> sd;
                sd.mu = ((double)st.mu + (double)st.mu_lo) + g0_rest;
                g0_rest = 0.0;  // now held by the state
                sd.s2 = (double)st.s2 + (double)st.s2_lo;
                sd.mu_lo = sd.s2_lo = 0.0;
                sd.aS_prev = local ? sp.a0 * pd.S(fma((double)j, P.h, -P.psi_max) * P.ell_per_psi)
                                   : cd.a0S0;
                sd.aS_next = 0.0;
                sd.m4_prev = (double)st.m4_prev;
                sd.chi_hi = 0.0;
                FwdRadWave radd(P.rad64, stage);
                for (;;) {
                    photon_step<double, QUANTUM, FwdRadWave, true>(cd, pp, tot, j, sd, radd, grid,
                                                                   acc);
                    ++j;
                    if (j >= N) break;
                    const double chi = P.two_over_aS * sd.mu * fabs(sd.aS_prev * env64[2 * j]);
                    if (!__any(chi > (double)P.chi_fp64)) break;
                }
                st.mu = (float)sd.mu;
                st.mu_lo = (float)(sd.mu - (double)st.mu);
                st.s2 = (float)sd.s2;
                st.s2_lo = (float)(sd.s2 - (double)st.s2);
                st.m4_prev = (float)sd.m4_prev;
                chd = fmax(chd, sd.chi_hi);
                if (local) {
                    st.aS_prev = c.a0 * c.pt.S(fmaf((float)j, c.h, c.psi0) * c.ell);
                    if (c.mid) st.aS_next = c.a0 * c.pt.S(fmaf((float)(j + 1), c.h, c.psi0) * c.ell);
                }
                if (j < N) rad.init(c.ph.two_over_aS * st.mu * fabsf(st.aS_prev * env32[2 * j]));
                continue;
            }
        }
        photon_step<T, QUANTUM>(c, pp, tot, j, st, rad, grid, acc);
        ++j;
    }
    if (!c.live) return;
    {  // the last stage 4 deposits alone
        const float aa = fabsf((float)(st.aS_prev * c.env[2 * N]));
        if (aa > 0.0f)
            ph_deposit((1.0f / 6.0f) * aa * c.inv_a0, ph_ln((float)st.m4_prev),
                       ph_sqrt((float)st.m4_prev), ph_ln(c.tas * aa),
                       c.tas * (float)st.m4_prev * aa, pp, grid, acc);
    }
    const double mu_f = ((double)st.mu + (double)st.mu_lo) + g0_rest;
    const double chi_hi = fmax((double)st.chi_hi, chd);
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

// Block size of the photon kernel: mixed-precision passes read the FP64 table
// a wavefront at a time and stage it in LDS (5 KB a wavefront), which beside
// the table, grid and photon-number cells (about 69 KB) fits one block of 512
// a CU; the others run blocks of 256, two a CU.  Either way two waves per
// SIMD, and the registers are held to that (the FP64 and mixed-precision
// passes would otherwise take a few more and run one).
template <int PREC>
constexpr int phot_block() {
    return PREC == PREC_F32MIX ? 2 * kDepBlock : kDepBlock;
}

template <int PREC, bool QUANTUM, bool LOCAL>
__global__ __launch_bounds__(phot_block<PREC>()) __attribute__((amdgpu_waves_per_eu(2))) void photon_kernel(
    BatchParams P, const float *__restrict__ env32, const double *__restrict__ env64) {
    constexpr int kBlock = phot_block<PREC>();
    // mixed precision: every lane of a wavefront runs (lanes past an item's
    // end repeat its last sample without depositing), for the table reads
    constexpr bool kWave64 = PREC == PREC_F32MIX;
    constexpr bool kTab32 = QUANTUM && PREC != PREC_F64;
    __shared__ __align__(16) float tab32[kTab32 ? kCells32 * kCellVals : 4];
    // mixed precision: two copies of the grid, the even lanes of a wavefront
    // depositing into one and the odd lanes into the other (the lanes hold
    // samples of similar chi, so neighbours often hit the same node; the copy
    // is offset by 32 banks), summed when the grid is flushed
    constexpr int kRep = kWave64 ? 2 : 1;
    constexpr int kRepStride = kPhLdsNodes + 16;
    __shared__ unsigned long long grid[(kRep - 1) * kRepStride + kPhLdsNodes];
    unsigned long long *lgrid = grid + (kRep > 1 ? (threadIdx.x & 1) * kRepStride : 0);
    __shared__ float tot[kPhRows];  // Phi(1; chi) / chi on the table rows
    // ... and as a cubic on each FP32 radiation cell
    __shared__ float4 ncell[kTab32 ? kCells32 : 1];
    __shared__ int64_t slot;
    __shared__ double red[kBlock / 64][kPhotPartials];
    __shared__ double2 stage[kWave64 ? (kBlock / 64) * kStageChunks : 1];
    // FP64 steps where chi is high: the lanes take the item's samples in
    // order of their chi scale (chi_order over the whole item)
    __shared__ float okey[kWave64 ? kPhotTile : 1];
    __shared__ unsigned short oidx[kWave64 ? kPhotTile : 1];
    double2 *wstage = stage + (kWave64 ? (threadIdx.x >> 6) * kStageChunks : 0);
    for (int r = threadIdx.x; r < kPhRows; r += blockDim.x)
        tot[r] = (float)(cbrt(kPhYMax) * P.phtab[(size_t)r * (kPhNZ + 1) + kPhNZ]);
    if (kTab32) {
        const float4 *src = reinterpret_cast<const float4 *>(P.rad32);
        float4 *dst = reinterpret_cast<float4 *>(tab32);
        for (int k = threadIdx.x; k < kCells32 * kCellVals / 4; k += blockDim.x) dst[k] = src[k];
        const float4 *nsrc = reinterpret_cast<const float4 *>(P.phtab + kPhCellOff);
        for (int k = threadIdx.x; k < kCells32; k += blockDim.x) ncell[k] = nsrc[k];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (;;) {
        const int64_t item = next_item(&P.queue[0], &slot);
        if (item >= P.n_pitems) break;
        const int s = __builtin_amdgcn_readfirstlane(find_phot(P.phot, P.n_shots, item));
        const ShotParams &sp = P.shots[s];
        const ShotPhot &pp = P.phot[s];
        const int nodes = pp.nu * pp.nv, lnodes = pp.nu * kPhLdsRow;
        for (int r = 0; r < kRep; ++r)
            for (int k = threadIdx.x; k < lnodes; k += blockDim.x) grid[r * kRepStride + k] = 0ull;
        __syncthreads();
        PhotAcc acc{0.0, 0.0, 0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double loss = 0.0;
        const int64_t i0 = (item - pp.pitem0) * kPhotTile;
        const int64_t i1 = i0 + kPhotTile < sp.n_samples ? i0 + kPhotTile : sp.n_samples;
        if constexpr (kWave64) {
            chi_order<kPhotTile, kBlock>(sp, P.key0, P.key1, i0, i1, okey, oidx);
            for (int64_t b = 0; b < i1 - i0; b += kBlock) {
                const int64_t i = i0 + oidx[b + threadIdx.x];
                const bool live = i < i1;
                photon_sample<PREC, QUANTUM, LOCAL>(P, sp, pp, live ? i : i1 - 1, env32, env64,
                                                    tab32, lgrid, tot, ncell, wstage, live, acc,
                                                    loss);
            }
        } else {
            for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x)
                photon_sample<PREC, QUANTUM, LOCAL>(P, sp, pp, i, env32, env64, tab32, grid, tot,
                                                    ncell, wstage, true, acc, loss);
        }
        if (acc.flags) atomicOr(&P.flags[s], acc.flags);
        const double v[kPhotPartials] = {acc.e_ph, loss, acc.soft, acc.nn, acc.nx,
                                         acc.ny, acc.ee, acc.ex, acc.ey};
#pragma unroll
        for (int m = 0; m < kPhotPartials; ++m) {
            const double w = wave_sum(v[m]);
            if (lane == 0) red[wid][m] = w;
        }
        __syncthreads();
        if (threadIdx.x < kPhotPartials) {
            double sum = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) sum += red[w][threadIdx.x];
            P.partials[(size_t)item * kPhotPartials + threadIdx.x] = sum;
        }
        for (int k = threadIdx.x; k < nodes; k += blockDim.x) {
            const int l = (k / pp.nv) * kPhLdsRow + k % pp.nv;
            unsigned long long w = grid[l];
            for (int r = 1; r < kRep; ++r) w += grid[r * kRepStride + l];
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
    // weights of the non-zero nodes (the grid and a row above and below),
    // then S_k
    __shared__ double nzw[kPhNodes + 2 * kPhNV + 2];
    __shared__ unsigned short nzi[kPhNodes + 2 * kPhNV];
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
    // node weights: the grid convolved with [-1/12, 7/6, -1/12] along each
    // axis (the deposit's tent deconvolved to second order), over the grid's
    // rows and the table rows just below and above it; columns beyond the
    // grid's are left out (the host keeps its outer columns empty); the
    // non-zero nodes compacted in index order
    const int nv = pp.nv, nu = pp.nu;
    const int nodes = (nu + 2) * nv;  // extended row e = grid row e - 1
    const unsigned long long *G = P.pgrid + pp.grid_off;
    auto node_weight = [&](int k) -> double {
        const int e = k / nv, m = k - e * nv;
        const int r = pp.r_lo + e - 1;
        if (r < 0 || r >= kPhRows) return 0.0;
        double acc = 0.0;
        for (int a = -1; a <= 1; ++a) {
            const int n = e - 1 + a;
            if (n < 0 || n >= nu) continue;
            double row = 0.0;
            for (int b = -1; b <= 1; ++b) {
                const int mm = m + b;
                if (mm < 0 || mm >= nv) continue;
                row += (b == 0 ? 7.0 / 6.0 : -1.0 / 12.0) * (double)G[n * nv + mm];
            }
            acc += (a == 0 ? 7.0 / 6.0 : -1.0 / 12.0) * row;
        }
        return acc;
    };
    const int kPer = (nodes + 255) / 256;
    int mine = 0;
    for (int q = 0; q < kPer; ++q) {
        const int k = tid * kPer + q;
        if (k < nodes && node_weight(k) != 0.0) ++mine;
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
        if (k >= nodes) break;
        const double w = node_weight(k);
        if (w != 0.0) {
            nzi[pos] = (unsigned short)k;
            nzw[pos] = w;
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
        const int e = k / nv, m = k - e * nv;
        const int r = pp.r_lo + e - 1;
        const double chi = exp(kPhU0 + r * kPhDu);
        const double t = pp.t_lo + m * pp.dt;
        const double inv_mu = 1.0 / (t * t);
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
        if (pp.angles) {
            // number: C_ph (2 / a_S) h sum c |a| Phi(1; chi)/chi; energy: h sum c (-A)
            double *o = pp.angles;
            const double nn = sums[3], ee = sums[6];
            o[0] = c_ph * P.two_over_aS * P.h * nn;
            o[1] = nn > 0.0 ? 1e3 * sqrt(sums[4] / nn) : 0.0;
            o[2] = nn > 0.0 ? 1e3 * sqrt(sums[5] / nn) : 0.0;
            o[3] = P.h * ee;
            o[4] = ee > 0.0 ? 1e3 * sqrt(sums[7] / ee) : 0.0;
            o[5] = ee > 0.0 ? 1e3 * sqrt(sums[8] / ee) : 0.0;
        }
        if (pp.status) {
            const int fl = P.flags[s];
            *pp.status = (fl & kFlagNonFinite) ? 4 : ((fl & kFlagRange) ? 6 : 0);
        }
    }
}

// FP64-shadow report of one shot.  The batch is the FP64 view pass; the FP32
// view pass wrote the same layout span doubles earlier (span 0: no shadow,
// zeros).  Relative differences are signed, against the FP64 value.
__device__ __forceinline__ double rel_diff(double a, double b) {
    return b != 0.0 ? (a - b) / b : 0.0;
}

__global__ __launch_bounds__(256) void photon_shadow_kernel(BatchParams P, int64_t span) {
    const ShotPhot &pp = P.phot[blockIdx.x];
    double *o = pp.errors;
    if (!o) return;
    const int tid = threadIdx.x;
    constexpr int kOut = 14;  // QS_PE_N
    if (span == 0) {
        if (tid < kOut) o[tid] = 0.0;
        return;
    }
    const double *h64 = pp.hist, *h32 = pp.hist - span;
    double l1 = 0.0, mx = 0.0, tot = 0.0;
    for (int k = tid; k < pp.n_ph + 2; k += blockDim.x) {
        const double d = fabs(h32[k] - h64[k]);
        l1 += d;
        mx = fmax(mx, d);
        tot += h64[k];
    }
    __shared__ double r_l1[256], r_mx[256], r_tot[256];
    r_l1[tid] = l1;
    r_mx[tid] = mx;
    r_tot[tid] = tot;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            r_l1[tid] += r_l1[tid + w];
            r_mx[tid] = fmax(r_mx[tid], r_mx[tid + w]);
            r_tot[tid] += r_tot[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double T = r_tot[0];
        o[0] = (double)P.shots[blockIdx.x].n_samples;
        o[1] = T > 0.0 ? r_l1[0] / T : 0.0;
        o[2] = T > 0.0 ? r_mx[0] / T : 0.0;
        const double *e64 = pp.energy, *e32 = pp.energy - span;
        o[3] = rel_diff(e32[0], e64[0]);
        o[4] = rel_diff(e32[1], e64[1]);
        for (int j = 0; j < 6; ++j)
            o[5 + j] = pp.angles ? rel_diff(pp.angles[j - span], pp.angles[j]) : 0.0;
        o[11] = T;
        o[12] = e64[0];
        o[13] = e64[1];
    }
}

// ===========================================================================
// Launchers
// ===========================================================================
size_t photon_work_doubles() { return (size_t)2 * 5 * kPhNZ + (kPhNZ + 1); }

hipError_t build_photon_table(double *phtab, double *work, size_t work_doubles, hipStream_t s) {
    if (work_doubles < photon_work_doubles()) return hipErrorInvalidValue;
    double *k23 = work, *k13 = work + 5 * kPhNZ, *i13 = work + 10 * kPhNZ;
    ph_bessel_kernel<<<(5 * kPhNZ + 63) / 64, 64, 0, s>>>(k23, k13);
    ph_i13_kernel<<<1, 1, 0, s>>>(k13, i13);
    ph_row_kernel<<<(kPhRows + 63) / 64, 64, 0, s>>>(k23, k13, i13, phtab);
    ph_cell_kernel<<<(kCells32 + 63) / 64, 64, 0, s>>>(
        phtab, reinterpret_cast<float *>(phtab + kPhCellOff));
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
    else if (prec == PREC_F32MIX && q)  // FP64 steps are a quantum-model option
        fn = l ? photon_ptr<PREC_F32MIX, true, true>() : photon_ptr<PREC_F32MIX, true, false>();
    else
        fn = q ? (l ? photon_ptr<PREC_F32, true, true>() : photon_ptr<PREC_F32, true, false>())
               : (l ? photon_ptr<PREC_F32, false, true>() : photon_ptr<PREC_F32, false, false>());
    const int block = prec == PREC_F32MIX && q ? phot_block<PREC_F32MIX>() : kDepBlock;
    int grid = 0;
    hipError_t e = resident_grid(fn, block, 0, p.n_pitems, &grid);
    if (e != hipSuccess) return e;
    BatchParams pc = p;
    const float *e32 = env32;
    const double *e64 = env64;
    void *args[] = {&pc, &e32, &e64};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(block), args, 0, s);
}

hipError_t launch_photon_finalize(const BatchParams &p, double c_ph, hipStream_t s) {
    photon_finalize_kernel<<<p.n_shots, 256, 0, s>>>(p, c_ph);
    return hipGetLastError();
}

hipError_t launch_photon_shadow(const BatchParams &p, int64_t span, hipStream_t s) {
    photon_shadow_kernel<<<p.n_shots, 256, 0, s>>>(p, span);
    return hipGetLastError();
}

hipError_t launch_photon_cdf(const double *phtab, int64_t n, const double *chi, const double *xi,
                             double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    ph_cdf_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(phtab, n, chi, xi, out);
    return hipGetLastError();
}

}  // namespace qs
