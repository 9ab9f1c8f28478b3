// qs_tables.hip -- construction of the radiation-function tables on the
// device (g, chi g', chi^2 g'', h for the forward pass; with the third
// derivative term and chi h' for the adjoint) and their diagnostic evaluation.
#include "qs_device.h"

namespace qs {

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
    double coef[kNodeVals][4] = {};
    for (int m = 0; m < 4; ++m) {
        double l[4];
        cheb_basis(m, l);
        for (int f = 0; f < kNodeVals; ++f) {
            const double v = vals[kNodeVals * (4 * cell_all + m) + f];
            for (int k = 0; k < 4; ++k) coef[f][k] += v * l[k];
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

hipError_t launch_radiation_eval(const float *rad32, const double *rad64, int prec, int64_t n,
                                 const double *chi, double *out, int *flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    rad_eval_kernel<<<(unsigned)blocks, 256, 0, s>>>(rad32, rad64, prec, n, chi, out, flags);
    return hipGetLastError();
}

}  // namespace qs
