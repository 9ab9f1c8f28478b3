/*
 * qso.cpp -- FP64 CPU oracle for the QScatter beam-phase-space integration.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg.  Shares nothing with the HIP library.
 *
 * The steps follow the paper (Amaro & Vranic, arXiv 2308.09348) in its order:
 *   1. samples of the beam phase space          -- Sec. 2 (volume elements)
 *   2. the focused laser seen by each sample    -- eq. a0eff, Table 1 offsets
 *   3. radiation-reaction evolution along phase -- eq. dpdtRR, eq. PWCRR
 *   4. per-sample observables                   -- Sec. 5.2 divergence
 *   5. deposit into spectra and moments         -- eq. dNda2dNdgf
 * Readings of points the paper leaves open are stated where they are used.
 */
#include "qso.h"

#include <cmath>
#include <functional>
#include <cstring>
#include <mutex>
#include <vector>
#include <omp.h>

namespace {

/* ---- physical constants (CODATA 2018) -------------------------------- */
const double kPi = 3.14159265358979323846;
const double kAlpha = 7.2973525693e-3;            /* fine-structure constant */
const double kLambdaBarC_um = 3.8615926796e-7;    /* reduced Compton wavelength */
const double kC_um_per_fs = 0.299792458;          /* speed of light          */

/* ---- forward-mode dual numbers ----------------------------------------- */
/* A value and its derivatives with respect to the eight differentiable
 * parameters (a0, w0, x_off, y_off, delay, gamma0, sigma_gamma, divergence).
 * The per-sample path below is written once for a scalar type T and
 * instantiated with double (the forward pass) and with Dual (its exact
 * derivative, by the chain rule applied operation by operation). */
const int kNP = 8;
struct Dual {
    double v;
    double d[kNP];
    Dual(double x = 0.0) : v(x) { for (int k = 0; k < kNP; ++k) d[k] = 0.0; }
};
inline double val(double x) { return x; }
inline double val(const Dual &x) { return x.v; }
inline Dual operator+(const Dual &a, const Dual &b) {
    Dual r(a.v + b.v); for (int k = 0; k < kNP; ++k) r.d[k] = a.d[k] + b.d[k]; return r;
}
inline Dual operator-(const Dual &a, const Dual &b) {
    Dual r(a.v - b.v); for (int k = 0; k < kNP; ++k) r.d[k] = a.d[k] - b.d[k]; return r;
}
inline Dual operator-(const Dual &a) {
    Dual r(-a.v); for (int k = 0; k < kNP; ++k) r.d[k] = -a.d[k]; return r;
}
inline Dual operator*(const Dual &a, const Dual &b) {
    Dual r(a.v * b.v); for (int k = 0; k < kNP; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r;
}
inline Dual operator/(const Dual &a, const Dual &b) {
    Dual r(a.v / b.v);
    for (int k = 0; k < kNP; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
}
inline Dual operator+(const Dual &a, double b) { Dual r = a; r.v += b; return r; }
inline Dual operator+(double a, const Dual &b) { return b + a; }
inline Dual operator-(const Dual &a, double b) { Dual r = a; r.v -= b; return r; }
inline Dual operator-(double a, const Dual &b) { return -b + a; }
inline Dual operator*(const Dual &a, double b) {
    Dual r(a.v * b); for (int k = 0; k < kNP; ++k) r.d[k] = a.d[k] * b; return r;
}
inline Dual operator*(double a, const Dual &b) { return b * a; }
inline Dual operator/(const Dual &a, double b) {
    Dual r(a.v / b); for (int k = 0; k < kNP; ++k) r.d[k] = a.d[k] / b; return r;
}
inline Dual operator/(double a, const Dual &b) { return Dual(a) / b; }
inline Dual &operator+=(Dual &a, const Dual &b) { a = a + b; return a; }
inline Dual chain(const Dual &a, double f, double df) {
    Dual r(f); for (int k = 0; k < kNP; ++k) r.d[k] = df * a.d[k]; return r;
}
inline Dual exp(const Dual &a) { const double e = std::exp(a.v); return chain(a, e, e); }
inline Dual log(const Dual &a) { return chain(a, std::log(a.v), 1.0 / a.v); }
inline Dual sqrt(const Dual &a) {
    if (a.v == 0.0) return Dual(0.0);  /* sqrt(max(sig2, 0)) at sig2 = 0: flat */
    const double s = std::sqrt(a.v);
    return chain(a, s, 0.5 / s);
}
inline Dual fabs(const Dual &a) { return a.v < 0 ? -a : a; }
inline Dual erfc(const Dual &a) {
    return chain(a, std::erfc(a.v), -2.0 / std::sqrt(kPi) * std::exp(-a.v * a.v));
}
inline Dual fmax(const Dual &a, const Dual &b) { return a.v >= b.v ? a : b; }
inline Dual fmin(const Dual &a, const Dual &b) { return a.v <= b.v ? a : b; }
using std::exp; using std::log; using std::sqrt; using std::fabs; using std::erfc;
using std::fmax; using std::fmin;

/* ---- operation counting ------------------------------------------------ */
/* A value that counts the floating-point operations performed on it (per
 * thread): the per-sample path instantiated with it gives the method's own
 * operation tally.  Each add, subtract, multiply, divide counts one; each
 * exp, log, sqrt or erfc counts one transcendental; sign changes, absolute
 * values, maxima and comparisons count nothing.  Arithmetic on plain doubles
 * (quantities shared by every sample, such as the envelope at a phase) is not
 * counted. */
struct OpCount { double add, mul, div, trans; };
thread_local OpCount g_ops = {0.0, 0.0, 0.0, 0.0};
struct Counted {
    double v;
    Counted(double x = 0.0) : v(x) {}
};
inline double val(const Counted &x) { return x.v; }
inline Counted operator+(const Counted &a, const Counted &b) { g_ops.add += 1; return Counted(a.v + b.v); }
inline Counted operator-(const Counted &a, const Counted &b) { g_ops.add += 1; return Counted(a.v - b.v); }
inline Counted operator-(const Counted &a) { return Counted(-a.v); }
inline Counted operator*(const Counted &a, const Counted &b) { g_ops.mul += 1; return Counted(a.v * b.v); }
inline Counted operator/(const Counted &a, const Counted &b) { g_ops.div += 1; return Counted(a.v / b.v); }
inline Counted operator+(const Counted &a, double b) { g_ops.add += 1; return Counted(a.v + b); }
inline Counted operator+(double a, const Counted &b) { g_ops.add += 1; return Counted(a + b.v); }
inline Counted operator-(const Counted &a, double b) { g_ops.add += 1; return Counted(a.v - b); }
inline Counted operator-(double a, const Counted &b) { g_ops.add += 1; return Counted(a - b.v); }
inline Counted operator*(const Counted &a, double b) { g_ops.mul += 1; return Counted(a.v * b); }
inline Counted operator*(double a, const Counted &b) { g_ops.mul += 1; return Counted(a * b.v); }
inline Counted operator/(const Counted &a, double b) { g_ops.div += 1; return Counted(a.v / b); }
inline Counted operator/(double a, const Counted &b) { g_ops.div += 1; return Counted(a / b.v); }
inline Counted &operator+=(Counted &a, const Counted &b) { a = a + b; return a; }
inline Counted exp(const Counted &a) { g_ops.trans += 1; return Counted(std::exp(a.v)); }
inline Counted log(const Counted &a) { g_ops.trans += 1; return Counted(std::log(a.v)); }
inline Counted sqrt(const Counted &a) { g_ops.trans += 1; return Counted(std::sqrt(a.v)); }
inline Counted erfc(const Counted &a) { g_ops.trans += 1; return Counted(std::erfc(a.v)); }
inline Counted fabs(const Counted &a) { return Counted(std::fabs(a.v)); }
inline Counted fmax(const Counted &a, const Counted &b) { return Counted(std::fmax(a.v, b.v)); }
inline Counted fmin(const Counted &a, const Counted &b) { return Counted(std::fmin(a.v, b.v)); }

/* ---- Philox4x32-10 ----------------------------------------------------- */
/* Counter-based generator of Salmon et al. (SC'11): ten rounds of two
 * 32x32->64 multiplies with the key bumped by the Weyl constants between
 * rounds. */
void philox_round(uint32_t c[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

/* ---- problem-derived scalars ----------------------------------------- */
struct Derived {
    double omega0;   /* laser angular frequency [rad/fs]                    */
    double aS;       /* normalised Schwinger vector potential m c^2/(hbar w0) */
    double K;        /* drift constant: dgamma/dpsi = -K a^2 gamma^2 g(chi)  */
    double CD;       /* diffusion constant: D = CD |a|^3 gamma^4 h(chi)      */
    double zR;       /* Rayleigh length [um]                                */
    double psi_max;  /* half-width of the integration window [rad]          */
    double h;        /* phase step                                          */
};

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

int validate(const qso_problem *p) {
    if (!p) return -1;
    const double vals[] = {p->a0, p->lambda_um, p->w0_um, p->tau_fs, p->x_off_um,
                           p->y_off_um, p->delay_fs, p->gamma0, p->sigma_gamma,
                           p->sigma_r_um, p->sigma_z_um, p->div_mrad, p->window_fwhm,
                           p->kernel_sigma_bins, p->c_theta, p->e_lo, p->e_hi,
                           p->th_lo_mrad, p->th_hi_mrad};
    for (double v : vals) if (!std::isfinite(v)) return -1;
    if (!(p->a0 >= 0) || !(p->lambda_um > 0) || !(p->w0_um >= 0) || !(p->tau_fs > 0)) return -1;
    if (!(p->gamma0 > 1) || !finite_nonneg(p->sigma_gamma) || !finite_nonneg(p->sigma_r_um) ||
        !finite_nonneg(p->sigma_z_um) || !finite_nonneg(p->div_mrad)) return -1;
    if (!(p->window_fwhm > 0) || !(p->kernel_sigma_bins >= 0) || !(p->c_theta >= 0)) return -1;
    if (p->n_samples < 0 || p->n_steps < 1) return -1;
    if (p->n_e < 1 || p->n_th < 1 || p->n_a < 1) return -1;
    if (!(p->e_hi > p->e_lo) || !(p->th_hi_mrad > p->th_lo_mrad)) return -1;
    if (p->envelope != QSO_ENV_GAUSS && p->envelope != QSO_ENV_SIN2) return -1;
    if ((p->transverse != QSO_PROFILE_GAUSS && p->transverse != QSO_PROFILE_FLAT) ||
        (p->longitudinal != QSO_PROFILE_GAUSS && p->longitudinal != QSO_PROFILE_FLAT))
        return -1;
    if (p->mode != QSO_MODE_GAUSS && p->mode != QSO_MODE_HG && p->mode != QSO_MODE_LG) return -1;
    if (p->mode != QSO_MODE_GAUSS &&
        (p->mode_m < 0 || p->mode_m > 8 || std::abs(p->mode_n) > 8 ||
         (p->mode == QSO_MODE_HG && p->mode_n < 0)))
        return -1;
    if (p->rr_model != QSO_RR_CLASSICAL && p->rr_model != QSO_RR_QUANTUM) return -1;
    if (p->amp_mode != QSO_AMP_A0EFF && p->amp_mode != QSO_AMP_LOCAL) return -1;
    if (p->deposit < QSO_DEP_POINT || p->deposit > QSO_DEP_GAUSS) return -1;
    return 0;
}

Derived derive(const qso_problem *p) {
    Derived d;
    d.omega0 = 2.0 * kPi * kC_um_per_fs / p->lambda_um;
    /* a_S = e E_S / (m c w0) = m c^2 / (hbar w0) = lambda / (2 pi lambdabar_C)  */
    d.aS = p->lambda_um / (2.0 * kPi * kLambdaBarC_um);
    /* eq. dpdtRR with chi = 2 gamma a / a_S, p = gamma m c and dpsi = 2 w0 dt
     * (head-on: the phase advances at twice the laser frequency):
     *   dgamma/dpsi = -g (2 alpha / 3) (c / (lambdabar_C w0)) chi^2 / 2
     *               = -(4 alpha / (3 a_S)) a^2 gamma^2 g.                    */
    d.K = 4.0 * kAlpha / (3.0 * d.aS);
    /* Second moment of the LCFA photon spectrum in the classical limit:
     *   d<dgamma^2>/dt = (55 / (24 sqrt3)) (alpha c / lambdabar_C) gamma chi^3,
     * converted to phase units the same way (h(chi) -> 1 as chi -> 0).       */
    d.CD = 55.0 / (6.0 * std::sqrt(3.0)) * kAlpha / (d.aS * d.aS);
    d.zR = kPi * p->w0_um * p->w0_um / p->lambda_um;
    if (p->envelope == QSO_ENV_GAUSS)
        d.psi_max = p->window_fwhm * d.omega0 * p->tau_fs;
    else
        d.psi_max = d.omega0 * p->tau_fs;
    d.h = 2.0 * d.psi_max / (double)p->n_steps;
    return d;
}

/* Temporal envelope of the vector potential as a function of the phase
 * psi = w0 (t - z/c) relative to the pulse peak.  GAUSS: intensity FWHM tau,
 * i.e. the amplitude falls as exp(-2 ln2 (psi / (w0 tau))^2).  SIN2: the
 * amplitude ramps from zero to peak over the rise time (the PIC set-ups of
 * Appendix A use this shape). */
double envelope(const qso_problem *p, const Derived &d, double psi) {
    if (p->envelope == QSO_ENV_GAUSS) {
        const double u = psi / (d.omega0 * p->tau_fs);
        return std::exp(-2.0 * std::log(2.0) * u * u);
    }
    const double pr = d.omega0 * p->tau_fs;
    if (std::fabs(psi) > pr) return 0.0;
    const double s = std::sin(kPi * (psi + pr) / (2.0 * pr));
    return s * s;
}

/* Linear polarisation along x with the carrier resolved (CEP 0). */
double envelope_carrier(const qso_problem *p, const Derived &d, double psi) {
    return envelope(p, d, psi) * std::cos(psi);
}

/* eq. a0eff: the focused Gaussian spatial factor a/a0 at (rho, z); the laser
 * phase and wavefront curvature are neglected as in Sec. 2.  w0 = 0 selects a
 * plane wave. */
/* ---- transverse laser modes (conclusions) ------------------------------- */
/* Hermite and generalised Laguerre polynomials by their three-term
 * recurrences. */
template <class T>
T hermite_poly(int m, const T &s) {
    T h0(1.0), h1 = 2.0 * s;
    if (m == 0) return h0;
    for (int k = 1; k < m; ++k) {
        const T h2 = 2.0 * s * h1 - (2.0 * k) * h0;
        h0 = h1;
        h1 = h2;
    }
    return h1;
}

template <class T>
T laguerre_poly(int p, int l, const T &t) {
    if (p < 0) return T(0.0);
    T L0(1.0), L1 = (1.0 + l) - t;
    if (p == 0) return L0;
    for (int k = 1; k < p; ++k) {
        const T L2 = ((2.0 * k + 1.0 + l - t) * L1 - (double)(k + l) * L0) / (double)(k + 1);
        L0 = L1;
        L1 = L2;
    }
    return L1;
}

/* Focal-plane peak of a mode's amplitude.  HG m: the extrema of |H_m(s)|
 * e^(-s^2/2) are where s H_m(s) = H_(m+1)(s) (the derivative with H_m' =
 * 2m H_(m-1)); LG p, l: those of t^(l/2) |L_p^l(t)| e^(-t/2) where
 * (l - t) L_p^l(t) = 2t L_(p-1)^(l+1)(t) (with dL_p^l/dt = -L_(p-1)^(l+1)).
 * Sign changes on a fine grid, bisection, the largest value. */
double extremum_max(const std::function<double(double)> &cond,
                    const std::function<double(double)> &val, double hi) {
    double best = std::fmax(val(0.0), val(hi));
    const int n = 20000;
    double a = 0.0, fa = cond(0.0);
    for (int k = 1; k <= n; ++k) {
        const double b = hi * k / n, fb = cond(b);
        if ((fa < 0.0) != (fb < 0.0)) {
            double lo = a, up = b, flo = fa;
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (lo + up), fm = cond(mid);
                if ((fm < 0.0) == (flo < 0.0)) lo = mid, flo = fm;
                else up = mid;
            }
            best = std::fmax(best, val(0.5 * (lo + up)));
        }
        a = b;
        fa = fb;
    }
    return best;
}

double mode_peak(int mode, int m, int n) {
    if (mode == QSO_MODE_HG) {
        auto one = [](int k) {
            return extremum_max(
                [k](double s) { return s * hermite_poly<double>(k, s) - hermite_poly<double>(k + 1, s); },
                [k](double s) { return std::fabs(hermite_poly<double>(k, s)) * std::exp(-0.5 * s * s); },
                std::sqrt(2.0 * k + 1.0) + 5.0);
        };
        return one(m) * one(n);
    }
    if (mode == QSO_MODE_LG) {
        const int l = std::abs(n), p = m;
        return extremum_max(
            [p, l](double t) {
                return (l - t) * laguerre_poly<double>(p, l, t) -
                       2.0 * t * laguerre_poly<double>(p - 1, l + 1, t);
            },
            [p, l](double t) {
                return std::pow(t, 0.5 * l) * std::fabs(laguerre_poly<double>(p, l, t)) *
                       std::exp(-0.5 * t);
            },
            4.0 * p + 2.0 * l + 40.0);
    }
    return 1.0;
}

double mode_inv_peak(const qso_problem *p) {
    thread_local int key[3] = {-1, -1, -1};
    thread_local double v = 1.0;
    if (key[0] != p->mode || key[1] != p->mode_m || key[2] != p->mode_n) {
        v = 1.0 / mode_peak(p->mode, p->mode_m, p->mode_n);
        key[0] = p->mode;
        key[1] = p->mode_m;
        key[2] = p->mode_n;
    }
    return v;
}

/* eq. a0eff: the focused Gaussian spatial factor a/a0 at (rho, z); a higher
 * mode (the conclusions' Laguerre- or Hermite-Gauss extension) replaces the
 * transverse profile, amplitude only, scaled to a focal-plane peak of 1:
 *   HG: |H_m(sqrt2 x/W) H_n(sqrt2 y/W)| e^(-rho^2/W^2) (W0/W) / C,
 *   LG: (2 rho^2/W^2)^(|l|/2) |L_p^|l|(2 rho^2/W^2)| e^(-rho^2/W^2) (W0/W) / C. */
template <class T>
T spatial(const qso_problem *p, const T &w0, const T &zR, const T &x, const T &y, const T &z) {
    if (val(w0) == 0.0) return T(1.0);
    const T zz = z / zR;
    const T q = 1.0 + zz * zz;
    const T r2 = (x * x + y * y) / (w0 * w0);
    const T g = exp(-r2 / q) / sqrt(q);
    if (p->mode == QSO_MODE_HG) {
        const T sc = sqrt(2.0 / q) / w0;
        return fabs(hermite_poly<T>(p->mode_m, x * sc) * hermite_poly<T>(p->mode_n, y * sc)) * g *
               mode_inv_peak(p);
    }
    if (p->mode == QSO_MODE_LG) {
        const int l = std::abs(p->mode_n);
        const T t = 2.0 * r2 / q;
        T tp(1.0);
        for (int k = 0; k < l / 2; ++k) tp = tp * t;
        if (l & 1) tp = tp * sqrt(t);
        return tp * fabs(laguerre_poly<T>(p->mode_m, l, t)) * g * mode_inv_peak(p);
    }
    return g;
}

/* ---- radiation functions g(chi), h(chi) -------------------------------- */
/* The quantum-synchrotron (LCFA) emission rate per unit photon energy
 * fraction xi, with y = 2 xi / (3 chi (1 - xi)), is proportional to
 *   (1 - xi + 1/(1 - xi)) K_{2/3}(y) - Int_y^inf K_{1/3}.
 * The Gaunt factor g (eq. dpdtRR) is its first xi-moment over the classical
 * power, and h its second moment over the classical second moment:
 *   g = sqrt3/(2 pi chi^2) Int_0^1 xi [..] dxi,
 *   h = 24/(55 pi chi^3)   Int_0^1 xi^2 [..] dxi.
 * The Int K_{1/3} term is integrated by parts in xi (d/dy of it is -K_{1/3},
 * the boundary terms vanish), and xi is traded for y, which gives
 *   Int_0^1 xi^n [..] dxi = Int_0^inf [xi^n w xi_y K_{2/3}(y)
 *                                       - xi^{n+1}/(n+1) K_{1/3}(y)] dy
 * with xi = 3 chi y / (2 + 3 chi y), xi_y = dxi/dy, w = 1 - xi + 1/(1 - xi).
 * The y integral uses the exp-sinh rule y = exp(pi/2 sinh t). */
void gh_integrals(double chi, double step, double *Ig, double *Ih) {
    double sg = 0.0, sh = 0.0;
    const double t_lo = std::asinh(2.0 / kPi * std::log(1e-22));
    const double t_hi = std::asinh(2.0 / kPi * std::log(70.0));
    const long k_lo = (long)std::floor(t_lo / step), k_hi = (long)std::ceil(t_hi / step);
    for (long k = k_lo; k <= k_hi; ++k) {
        const double t = k * step;
        const double y = std::exp(0.5 * kPi * std::sinh(t));
        const double dydt = y * 0.5 * kPi * std::cosh(t);
        const double q = 2.0 + 3.0 * chi * y;
        const double xi = 3.0 * chi * y / q;
        const double one_m_xi = 2.0 / q;
        const double w = one_m_xi + q / 2.0;
        const double xi_y = 6.0 * chi / (q * q);
        const double k23 = std::cyl_bessel_k(2.0 / 3.0, y);
        const double k13 = std::cyl_bessel_k(1.0 / 3.0, y);
        sg += (xi * w * xi_y * k23 - 0.5 * xi * xi * k13) * dydt;
        sh += (xi * xi * w * xi_y * k23 - xi * xi * xi / 3.0 * k13) * dydt;
    }
    *Ig = sg * step;
    *Ih = sh * step;
}

const double kQuadStep = 1.0 / 48.0;

void gh_exact(double chi, double *g, double *h) {
    double Ig, Ih;
    gh_integrals(chi, kQuadStep, &Ig, &Ih);
    *g = std::sqrt(3.0) / (2.0 * kPi * chi * chi) * Ig;
    *h = 24.0 / (55.0 * kPi * chi * chi * chi) * Ih;
}

/* Table in u = ln chi.  Derivatives from sixth-order central differences of
 * the quadrature values: G1 = chi g' = dg/du, G2 = chi^2 g'' = d2g/du2 - dg/du.
 * Below chi_min the small-chi expansions hold (g: the Sokolov-Ternov series;
 * h: its first-order term from the same Mellin moments that fix h(0) = 1). */
struct RadTable {
    double u0, du;
    int n;  /* node count including padding */
    std::vector<double> g, G1, G2, h;
};

const double kChiMin = 1e-6, kChiMax = 1e3;
const int kPad = 6;
const double kG1 = -55.0 * 1.7320508075688772 / 16.0;   /* -55 sqrt3 / 16  */
const double kG2 = 48.0;
const double kH1 = -1344.0 / (55.0 * 1.7320508075688772); /* -1344/(55 sqrt3) */

RadTable *g_table = nullptr;
std::once_flag g_table_once;

void build_table() {
    RadTable *t = new RadTable;
    t->du = 1.0 / 256.0;
    const double u_min = std::log(kChiMin), u_max = std::log(kChiMax);
    const int core = (int)std::ceil((u_max - u_min) / t->du) + 1;
    t->n = core + 2 * kPad;
    t->u0 = u_min - kPad * t->du;
    std::vector<double> gv(t->n), hv(t->n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < t->n; ++k) {
        const double chi = std::exp(t->u0 + k * t->du);
        gh_exact(chi, &gv[k], &hv[k]);
    }
    t->g = gv; t->h = hv;
    t->G1.assign(t->n, 0.0);
    t->G2.assign(t->n, 0.0);
    for (int k = 3; k < t->n - 3; ++k) {
        const double *f = &gv[k];
        const double d1 = (-f[-3] + 9 * f[-2] - 45 * f[-1] + 45 * f[1] - 9 * f[2] + f[3]) /
                          (60.0 * t->du);
        const double d2 = (2 * f[-3] - 27 * f[-2] + 270 * f[-1] - 490 * f[0] + 270 * f[1] -
                           27 * f[2] + 2 * f[3]) / (180.0 * t->du * t->du);
        t->G1[k] = d1;
        t->G2[k] = d2 - d1;
    }
    g_table = t;
}

const RadTable &table() {
    std::call_once(g_table_once, build_table);
    return *g_table;
}

/* g, chi g', chi^2 g'', h at chi >= 0 (4-point Lagrange in u). */
template <class T>
void radiation(const T &chi, T out[4]) {
    if (!(val(chi) >= 0.0)) {  /* a negative energy or amplitude: no physical chi */
        out[0] = out[1] = out[2] = out[3] = T(NAN);
        return;
    }
    if (val(chi) < kChiMin) {
        out[0] = 1.0 + kG1 * chi + kG2 * chi * chi;
        out[1] = kG1 * chi + 2.0 * kG2 * chi * chi;
        out[2] = 2.0 * kG2 * chi * chi;
        out[3] = 1.0 + kH1 * chi;
        return;
    }
    if (!(val(chi) <= kChiMax)) {
        out[0] = out[1] = out[2] = out[3] = T(NAN);
        return;
    }
    const RadTable &t = table();
    const T s = (log(chi) - t.u0) / t.du;
    const int i = (int)std::floor(val(s));
    const T x = s - (double)i;
    const T w[4] = {-x * (x - 1.0) * (x - 2.0) / 6.0, (x + 1.0) * (x - 1.0) * (x - 2.0) / 2.0,
                    -(x + 1.0) * x * (x - 2.0) / 2.0, (x + 1.0) * x * (x - 1.0) / 6.0};
    const std::vector<double> *cols[4] = {&t.g, &t.G1, &t.G2, &t.h};
    for (int c = 0; c < 4; ++c) {
        T acc(0.0);
        for (int m = 0; m < 4; ++m) acc += w[m] * (*cols[c])[i - 1 + m];
        out[c] = acc;
    }
}

/* ---- the moment system ------------------------------------------------- */
/* Drift A(mu) from eq. dpdtRR in phase units; the mean and variance of the
 * energy distribution of a beamlet obey, at second order about the mean
 * (Fokker-Planck regime of Sec. 1):
 *   dmu/dpsi   = A(mu) + A''(mu) sig2 / 2,
 *   dsig2/dpsi = 2 A'(mu) sig2 + D(mu),
 * with chi = 2 mu |a| / a_S.  The classical model is g = 1, D = 0.          */
template <class T>
struct Rhs { T A, A1, A2, D, dmu, dsig2; };

template <class T>
Rhs<T> rhs(const qso_problem *p, const Derived &d, const T &mu, const T &sig2, const T &a) {
    T g(1.0), G1(0.0), G2(0.0), hq(0.0);
    const T abs_a = fabs(a);
    if (p->rr_model == QSO_RR_QUANTUM) {
        T rf[4];
        radiation<T>(2.0 * mu * abs_a / d.aS, rf);
        g = rf[0]; G1 = rf[1]; G2 = rf[2]; hq = rf[3];
    }
    Rhs<T> r;
    const T a2 = a * a;
    r.A = -d.K * a2 * mu * mu * g;
    r.A1 = -d.K * a2 * mu * (2.0 * g + G1);
    r.A2 = -d.K * a2 * (2.0 * g + 4.0 * G1 + G2);
    r.D = (p->rr_model == QSO_RR_QUANTUM) ? d.CD * a2 * abs_a * mu * mu * mu * mu * hq : T(0.0);
    r.dmu = r.A + 0.5 * r.A2 * sig2;
    r.dsig2 = 2.0 * r.A1 * sig2 + r.D;
    return r;
}

/* ---- one sample -------------------------------------------------------- */
/* The eight parameters a derivative can be taken with respect to. */
template <class T>
struct Params {
    T a0, w0, x_off, y_off, delay, gamma0, sigma_gamma, div_mrad;
    T zR;  /* Rayleigh length pi w0^2 / lambda */
};

template <class T>
Params<T> params(const qso_problem *p) {
    Params<T> P;
    P.a0 = p->a0; P.w0 = p->w0_um; P.x_off = p->x_off_um; P.y_off = p->y_off_um;
    P.delay = p->delay_fs; P.gamma0 = p->gamma0; P.sigma_gamma = p->sigma_gamma;
    P.div_mrad = p->div_mrad;
    return P;
}

template <class T>
void finish_params(const qso_problem *p, Params<T> &P) {
    P.zR = kPi * P.w0 * P.w0 / p->lambda_um;
}

template <class T>
struct SampleIn {
    T x, y, z, gamma0, thx, thy;  /* um, um, um, -, rad, rad */
};

/* The six 24-bit uniforms in (0, 1) of sample i: counter (i, shot, k, 0),
 * key = seed. */
void uniforms(uint64_t seed, int32_t shot, int64_t i, double u[6]) {
    uint32_t r[8];
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t k = 0; k < 2; ++k) {
        const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)shot, k, 0u};
        qso_philox4x32_10(ctr, key, &r[4 * k]);
    }
    for (int m = 0; m < 6; ++m) u[m] = ((double)(r[m] >> 8) + 0.5) * (1.0 / 16777216.0);
}

void normals(uint64_t seed, int32_t shot, int64_t i, double n[6]) {
    double u[6];
    uniforms(seed, shot, i, u);
    /* Box-Muller on consecutive pairs */
    for (int m = 0; m < 3; ++m) {
        const double R = std::sqrt(-2.0 * std::log(u[2 * m]));
        n[2 * m] = R * std::cos(2.0 * kPi * u[2 * m + 1]);
        n[2 * m + 1] = R * std::sin(2.0 * kPi * u[2 * m + 1]);
    }
}

/* A sample of the beam (Sec. 2 volume element).  Gaussian profiles use the
 * Box-Muller normals; the flat-top beams of Table 1 (Wide, Thin) use the
 * same uniforms directly: a uniform disk of radius sigma_r, r = sigma_r
 * sqrt(u0) at the Box-Muller angle 2 pi u1, and a uniform length sigma_z,
 * z = sigma_z (u2 - 1/2). */
template <class T>
SampleIn<T> make_sample(const qso_problem *p, const Params<T> &P, int64_t i) {
    double n[6], u[6];
    normals(p->seed, p->shot, i, n);
    uniforms(p->seed, p->shot, i, u);
    SampleIn<T> s;
    if (p->transverse == QSO_PROFILE_FLAT) {
        const double r = p->sigma_r_um * std::sqrt(u[0]);
        s.x = P.x_off + r * std::cos(2.0 * kPi * u[1]);
        s.y = P.y_off + r * std::sin(2.0 * kPi * u[1]);
    } else {
        s.x = P.x_off + p->sigma_r_um * n[0];
        s.y = P.y_off + p->sigma_r_um * n[1];
    }
    s.z = T(p->longitudinal == QSO_PROFILE_FLAT ? p->sigma_z_um * (u[2] - 0.5)
                                                : p->sigma_z_um * n[2]);
    s.gamma0 = P.gamma0 + P.sigma_gamma * n[3];
    s.thx = 1e-3 * P.div_mrad * n[4];
    s.thy = 1e-3 * P.div_mrad * n[5];
    return s;
}

/* Ballistic geometry (probe particles on ballistic trajectories, as the
 * conclusions restate).  The laser moves along +z with its peak at z = c t
 * and focus at z = 0; the beam moves along -z and its centroid meets the
 * peak at t = delay/2, at z = c delay / 2.  Sample coordinates (x, y) are
 * taken at that instant.  A sample at longitudinal offset z meets the peak at
 * z* = (z + c delay)/2; at phase psi it has travelled l = c psi / (2 w0) =
 * psi lambda / (4 pi) past that point.                                     */
template <class T>
struct Geometry {
    T zstar;  /* collision point on the axis [um]                            */
    T S0;     /* spatial factor at the collision point                        */
};

template <class T>
Geometry<T> geometry(const qso_problem *p, const Params<T> &P, const SampleIn<T> &s) {
    Geometry<T> gmt;
    gmt.zstar = 0.5 * (s.z + kC_um_per_fs * P.delay);
    const T xc = s.x + s.thx * 0.5 * s.z;
    const T yc = s.y + s.thy * 0.5 * s.z;
    gmt.S0 = spatial<T>(p, P.w0, P.zR, xc, yc, gmt.zstar);
    (void)p;
    return gmt;
}

template <class T>
T amplitude(const qso_problem *p, const Derived &d, const Params<T> &P, const SampleIn<T> &s,
            const Geometry<T> &gmt, double psi) {
    T S;
    if (p->amp_mode == QSO_AMP_A0EFF) {
        /* Sec. 2: the sample is assigned the peak amplitude it meets, a0,eff */
        S = gmt.S0;
    } else {
        const double l = psi * p->lambda_um / (4.0 * kPi);
        S = spatial<T>(p, P.w0, P.zR, s.x + s.thx * (0.5 * s.z + l),
                       s.y + s.thy * (0.5 * s.z + l), gmt.zstar - l);
    }
    return P.a0 * S * envelope_carrier(p, d, psi);
}

template <class T>
struct SampleOut {
    T mu, sig2, thx, thy, sigth, aeff_ratio;
    double chimax;
    T gamma0, x, y, z;
};

/* No-op stage visitor (see run_sample). */
struct NoVisit {
    template <class T>
    void operator()(double, const T &, const T &, const Rhs<T> &) const {}
};

/* The trajectory of a sample with initial state s and geometry gmt.
 * visit(w, mu_s, a_s, k_s) is called at every RK4 stage with its quadrature
 * weight w (h/6, h/3, h/3, h/6), the stage state and amplitude, and the
 * stage's right-hand side. */
template <class T, class Visit>
SampleOut<T> evolve(const qso_problem *p, const Derived &d, const Params<T> &P,
                    const SampleIn<T> &s, const Geometry<T> &gmt, Visit &visit) {
    T mu = s.gamma0, sig2(0.0);
    double chimax = 0.0;
    const double h = d.h;
    for (int j = 0; j < p->n_steps; ++j) {
        /* classical fourth-order Runge-Kutta in psi on (mu, sig2) */
        const double psi = -d.psi_max + j * h;
        const T a1 = amplitude<T>(p, d, P, s, gmt, psi);
        const T ah = amplitude<T>(p, d, P, s, gmt, psi + 0.5 * h);
        const T a4 = amplitude<T>(p, d, P, s, gmt, psi + h);
        chimax = std::fmax(chimax, 2.0 * val(mu) * std::fabs(val(a1)) / d.aS);
        const Rhs<T> k1 = rhs<T>(p, d, mu, sig2, a1);
        const T m2 = mu + 0.5 * h * k1.dmu;
        const Rhs<T> k2 = rhs<T>(p, d, m2, sig2 + 0.5 * h * k1.dsig2, ah);
        const T m3 = mu + 0.5 * h * k2.dmu;
        const Rhs<T> k3 = rhs<T>(p, d, m3, sig2 + 0.5 * h * k2.dsig2, ah);
        const T m4 = mu + h * k3.dmu;
        const Rhs<T> k4 = rhs<T>(p, d, m4, sig2 + h * k3.dsig2, a4);
        visit(h / 6.0, mu, a1, k1);
        visit(h / 3.0, m2, ah, k2);
        visit(h / 3.0, m3, ah, k3);
        visit(h / 6.0, m4, a4, k4);
        mu += h / 6.0 * (k1.dmu + 2.0 * k2.dmu + 2.0 * k3.dmu + k4.dmu);
        sig2 += h / 6.0 * (k1.dsig2 + 2.0 * k2.dsig2 + 2.0 * k3.dsig2 + k4.dsig2);
    }
    {
        const T aN = amplitude<T>(p, d, P, s, gmt, d.psi_max);
        chimax = std::fmax(chimax, 2.0 * val(mu) * std::fabs(val(aN)) / d.aS);
    }
    SampleOut<T> o;
    o.mu = mu;
    o.sig2 = sig2;
    /* The photon recoil of an ultra-relativistic emitter is along its
     * momentum (emission within 1/gamma of it, Sec. 5.1), so the direction
     * is kept; the stochastic broadening of Sec. 5.2 is applied in the
     * polarisation plane x: sigma_theta = c_theta sqrt(2/pi) a0eff sigma_f /
     * gamma_f^2.                                                           */
    o.thx = 1e3 * s.thx;
    o.thy = 1e3 * s.thy;
    const T sigf = sqrt(fmax(sig2, T(0.0)));
    const T aeff = P.a0 * gmt.S0;
    o.sigth = 1e3 * p->c_theta * std::sqrt(2.0 / kPi) * aeff * sigf / (mu * mu);
    o.aeff_ratio = gmt.S0;
    o.chimax = chimax;
    o.gamma0 = s.gamma0;
    o.x = s.x; o.y = s.y; o.z = s.z;
    return o;
}

/* One sample's trajectory (its draw, its geometry, its evolution). */
template <class T, class Visit>
SampleOut<T> run_sample(const qso_problem *p, const Derived &d, const Params<T> &P, int64_t i,
                        Visit &visit) {
    const SampleIn<T> s = make_sample<T>(p, P, i);
    const Geometry<T> gmt = geometry<T>(p, P, s);
    return evolve<T>(p, d, P, s, gmt, visit);
}

template <class T>
SampleOut<T> run_sample(const qso_problem *p, const Derived &d, const Params<T> &P, int64_t i) {
    NoVisit none;
    return run_sample<T>(p, d, P, i, none);
}

SampleOut<double> run_sample(const qso_problem *p, const Derived &d, int64_t i) {
    Params<double> P = params<double>(p);
    finish_params(p, P);
    return run_sample<double>(p, d, P, i);
}

/* ---- deposit ------------------------------------------------------------ */
template <class T> T Phi(const T &t) { return 0.5 * erfc(-t / std::sqrt(2.0)); }
template <class T> T PhiC(const T &t) { return 0.5 * erfc(t / std::sqrt(2.0)); }
template <class T> T phi(const T &t) { return exp(-0.5 * t * t) / std::sqrt(2.0 * kPi); }

/* The law deposited by one sample is its own energy (or angle) law -- a point
 * at v when s = 0, else N(v, s^2) -- convolved with the deposit kernel
 * (POINT: none, CIC: a box one bin wide, GAUSS: N(0, (k bins)^2)); each bin
 * gets that law's mass over it, so a sample always adds exactly one unit.
 * cdf(x) returns P(X <= x), ccdf(x) returns P(X > x).                       */
template <class T>
struct Law {
    int mode;  /* 0 step, 1 box, 2 gauss, 3 box (x) gauss */
    T v, s;
    double half;
};

template <class T>
Law<T> make_law(const T &v, const T &s, int32_t deposit, double ksig_bins, double width) {
    Law<T> L;
    L.v = v;
    L.half = 0.5 * width;
    if (deposit == QSO_DEP_GAUSS) {
        const double ks = ksig_bins * width;
        L.s = sqrt(s * s + ks * ks);
        L.mode = val(L.s) > 0 ? 2 : 0;
    } else if (deposit == QSO_DEP_CIC) {
        L.s = s;
        L.mode = val(s) > 0 ? 3 : 1;
    } else {
        L.s = s;
        L.mode = val(s) > 0 ? 2 : 0;
    }
    return L;
}

/* Psi(t) = Int_-inf^t Phi(u/s) du = t Phi(t/s) + s phi(t/s);
 * PsiC(t) = Psi(t) - t = -t PhiC(t/s) + s phi(t/s).                        */
template <class T> T Psi(const T &t, const T &s) { return t * Phi<T>(t / s) + s * phi<T>(t / s); }
template <class T> T PsiC(const T &t, const T &s) {
    return -t * PhiC<T>(t / s) + s * phi<T>(t / s);
}

template <class T>
T law_cdf(const Law<T> &L, double x) {
    const T t = x - L.v;
    switch (L.mode) {
        case 0: return T(val(t) > 0 ? 1.0 : 0.0);  /* NGP: floor((v - lo) / width) */
        case 1: return fmin(T(1.0), fmax(T(0.0), t / (2 * L.half) + 0.5));
        case 2: return Phi<T>(t / L.s);
        default: return (Psi<T>(t + L.half, L.s) - Psi<T>(t - L.half, L.s)) / (2 * L.half);
    }
}

template <class T>
T law_ccdf(const Law<T> &L, double x) {
    const T t = x - L.v;
    switch (L.mode) {
        case 0: return T(val(t) > 0 ? 0.0 : 1.0);
        case 1: return fmin(T(1.0), fmax(T(0.0), 0.5 - t / (2 * L.half)));
        case 2: return PhiC<T>(t / L.s);
        default: return (PsiC<T>(t - L.half, L.s) - PsiC<T>(t + L.half, L.s)) / (2 * L.half);
    }
}

template <class T>
void deposit(const T &v, const T &s, int32_t dep, double ksig, double lo, double hi, int32_t n,
             T *hist) {
    const double width = (hi - lo) / n;
    const Law<T> L = make_law<T>(v, s, dep, ksig, width);
    hist[n] += law_cdf<T>(L, lo);
    hist[n + 1] += law_ccdf<T>(L, hi);
    for (int k = 0; k < n; ++k) {
        const double e0 = lo + k * width, e1 = lo + (k + 1) * width;
        /* difference of whichever tail is smaller, for relative accuracy */
        const T m = (0.5 * (e0 + e1) <= val(v)) ? law_cdf<T>(L, e1) - law_cdf<T>(L, e0)
                                                 : law_ccdf<T>(L, e0) - law_ccdf<T>(L, e1);
        hist[k] += m;
    }
}

/* ---- photon emission (Sec. 4) ------------------------------------------- */
/* The approximate photon spectrum of Sec. 4: at each phase the electron of
 * mean energy gamma meets the instantaneous amplitude a and emits the LCFA
 * quantum-synchrotron spectrum of chi = 2 gamma |a| / a_S; the spectra are
 * integrated over the phase.  Per unit phase (dpsi = 2 omega0 dt) and unit
 * photon energy fraction xi the expected photon number is
 *   d2N / (dpsi dxi) = C_ph F(xi, chi) / gamma,   C_ph = alpha a_S / (2 sqrt3 pi),
 *   F = (1 - xi + 1/(1 - xi)) K_{2/3}(y) - Int_y^inf K_{1/3},  y = 2 xi / (3 chi (1 - xi)),
 * the emission rate of the radiation functions above over dpsi/dt; its first
 * xi-moment is (2 pi chi^2 / sqrt3) g, i.e. the drift of eq. dpdtRR.
 * Reading: the phase integral uses the RK4 stages of each step with their
 * weights (h/6, h/3, h/3, h/6) at the stage states, so that in the classical
 * model the emitted photon energy equals the electron's energy loss exactly.
 *
 * The number CDF Phi(xi; chi) = Int_0^xi F dxi' is tabulated over
 * u = ln chi and z = y^(1/3), as Phi / (chi z): Phi grows like z near 0 and
 * in the classical limit Phi = chi H(y).  Per row the Int K_{1/3} term is
 * integrated by parts:
 *   Phi = Int_0^y [w K_{2/3}(y') xi_y(y') - xi(y') K_{1/3}(y')] dy' - xi Int_y^inf K_{1/3},
 * with 5-point Gauss-Legendre on every z interval, and Int_y^inf K_{1/3}
 * accumulated downwards from y_max = 80 (both tails there are below 1e-34). */
struct PhotonTable {
    double u0, du, dz;
    int nu, nz;
    std::vector<double> v;  /* [nu][nz + 1]: Phi / (chi z) at z_j = j dz */
};

const double kPhotonYMax = 80.0;
PhotonTable *g_photon = nullptr;
std::once_flag g_photon_once;

void build_photon_table() {
    PhotonTable *T = new PhotonTable;
    T->du = 1.0 / 32.0;
    T->u0 = std::log(1e-6);
    T->nu = (int)std::ceil((std::log(1e3) - T->u0) / T->du) + 1;
    T->nz = 2048;
    T->dz = std::cbrt(kPhotonYMax) / T->nz;
    T->v.assign((size_t)T->nu * (T->nz + 1), 0.0);
    const double gx[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831,
                          0.9061798459386640};
    const double gw[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                          0.4786286704993665, 0.2369268850561891};
#pragma omp parallel for schedule(dynamic, 4)
    for (int r = 0; r < T->nu; ++r) {
        const double chi = std::exp(T->u0 + r * T->du);
        const int nz = T->nz;
        const double dz = T->dz;
        std::vector<double> I13(nz + 1, 0.0), A(nz + 1, 0.0);
        for (int j = nz - 1; j >= 0; --j) {  /* Int_y^inf K_{1/3}, downwards */
            double s = 0.0;
            for (int g = 0; g < 5; ++g) {
                const double z = dz * (j + 0.5 + 0.5 * gx[g]);
                const double y = z * z * z;
                s += gw[g] * std::cyl_bessel_k(1.0 / 3.0, y) * 3.0 * z * z;
            }
            I13[j] = I13[j + 1] + 0.5 * dz * s;
        }
        for (int j = 0; j < nz; ++j) {  /* the other two terms, upwards */
            double s = 0.0;
            for (int g = 0; g < 5; ++g) {
                const double z = dz * (j + 0.5 + 0.5 * gx[g]);
                const double y = z * z * z;
                const double q = 2.0 + 3.0 * chi * y;
                const double xi = 3.0 * chi * y / q;
                const double w = 2.0 / q + 0.5 * q;  /* 1 - xi + 1/(1 - xi) */
                const double xi_y = 6.0 * chi / (q * q);
                const double f = w * std::cyl_bessel_k(2.0 / 3.0, y) * xi_y -
                                 xi * std::cyl_bessel_k(1.0 / 3.0, y);
                s += gw[g] * f * 3.0 * z * z;
            }
            A[j + 1] = A[j] + 0.5 * dz * s;
        }
        double *row = &T->v[(size_t)r * (nz + 1)];
        /* stored: Phi / (chi z), smooth at z = 0, where it tends to
         * 9 2^(-1/3) Gamma(2/3) (from K_{2/3}(y) ~ Gamma(2/3)/2 (y/2)^(-2/3)) */
        row[0] = 9.0 * std::pow(2.0, -1.0 / 3.0) * std::tgamma(2.0 / 3.0);
        for (int j = 1; j <= nz; ++j) {
            const double z = dz * j, y = z * z * z;
            const double xi = 3.0 * chi * y / (2.0 + 3.0 * chi * y);
            row[j] = (A[j] - xi * I13[j]) / (chi * z);
        }
    }
    g_photon = T;
}

const PhotonTable &photon_table() {
    std::call_once(g_photon_once, build_photon_table);
    return *g_photon;
}

/* 4-point Lagrange weights at x in [0, 3] for nodes 0..3. */
void lagrange4(double x, double w[4]) {
    w[0] = -(x - 1.0) * (x - 2.0) * (x - 3.0) / 6.0;
    w[1] = x * (x - 2.0) * (x - 3.0) / 2.0;
    w[2] = -x * (x - 1.0) * (x - 3.0) / 2.0;
    w[3] = x * (x - 1.0) * (x - 2.0) / 6.0;
}

/* Interpolation in u fixed for one chi: Phi(xi; chi) at many xi.  Below the
 * table's first row the classical scaling Phi = chi H(y) is used (row 0 at the
 * sample's own y); above its last row the value is NaN. */
struct PhotonRow {
    const PhotonTable *T;
    double chi, wu[4];
    int r0;
    bool ok;
    explicit PhotonRow(double chi_) : T(&photon_table()), chi(chi_) {
        const double s = (std::log(chi) - T->u0) / T->du;
        ok = chi > 0.0 && s <= T->nu - 1;
        if (s < 0.0) {
            r0 = 0;
            wu[0] = 1.0; wu[1] = wu[2] = wu[3] = 0.0;
            return;
        }
        int i = (int)std::floor(s) - 1;
        if (i < 0) i = 0;
        if (i > T->nu - 4) i = T->nu - 4;
        r0 = i;
        lagrange4(s - i, wu);
    }
    double at_z(double z) const {  /* Phi / chi at z (clamped to the table) */
        if (z > T->nz * T->dz) z = T->nz * T->dz;
        double t = z / T->dz;
        int j = (int)std::floor(t) - 1;
        if (j < 0) j = 0;
        if (j > T->nz - 3) j = T->nz - 3;
        double wz[4];
        lagrange4(t - j, wz);
        double acc = 0.0;
        for (int a = 0; a < 4; ++a) {
            const double *row = &T->v[(size_t)(r0 + a) * (T->nz + 1) + j];
            acc += wu[a] * (wz[0] * row[0] + wz[1] * row[1] + wz[2] * row[2] + wz[3] * row[3]);
        }
        return acc * z;
    }
    double total() const { return ok ? chi * at_z(T->nz * T->dz) : NAN; }
    double cdf(double xi) const {
        if (!ok) return NAN;
        if (!(xi > 0.0)) return 0.0;
        if (xi >= 1.0) return total();
        const double y = 2.0 * xi / (3.0 * chi * (1.0 - xi));
        return chi * at_z(std::cbrt(y));
    }
};

/* Photon bins of one emission: weight C_ph w / gamma times the CDF
 * differences at the bin edges (underflow [n], overflow [n + 1]). */
void photon_deposit(double weight, double gamma, const PhotonRow &R, int32_t n, double lo,
                    double width, double *hist) {
    const double N = R.total();
    double prev = R.cdf(lo / gamma);
    hist[n] += weight * prev;
    for (int k = 0; k < n; ++k) {
        const double next = R.cdf((lo + (k + 1) * width) / gamma);
        hist[k] += weight * (next - prev);
        prev = next;
    }
    hist[n + 1] += weight * (N - prev);
}

/* Neumaier-compensated running sum. */
struct KSum {
    double s = 0.0, c = 0.0;
    void add(double x) {
        const double t = s + x;
        if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
        s = t;
    }
    double value() const { return s + c; }
};

}  // namespace

/* ======================================================================== */
extern "C" {

void qso_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

void qso_normals(uint64_t seed, int32_t shot, int64_t i, double out[6]) {
    normals(seed, shot, i, out);
}

void qso_gh_quadrature(double chi, double *g, double *h) { gh_exact(chi, g, h); }

void qso_radiation(double chi, double out[4]) { radiation(chi, out); }

int qso_derived(const qso_problem *p, double out[7]) {
    if (validate(p)) return -1;
    const Derived d = derive(p);
    out[0] = d.omega0; out[1] = d.aS; out[2] = d.K; out[3] = d.CD;
    out[4] = d.zR; out[5] = d.psi_max; out[6] = d.h;
    return 0;
}

double qso_envelope_carrier(const qso_problem *p, double psi) {
    const Derived d = derive(p);
    return envelope_carrier(p, d, psi);
}

int qso_rhs(const qso_problem *p, double mu, double sig2, double a, double out[6]) {
    if (validate(p)) return -1;
    const Derived d = derive(p);
    const Rhs r = rhs(p, d, mu, sig2, a);
    out[0] = r.A; out[1] = r.A1; out[2] = r.A2; out[3] = r.D; out[4] = r.dmu; out[5] = r.dsig2;
    return 0;
}

int qso_sample(const qso_problem *p, int64_t i, double *rec) {
    if (validate(p)) return -1;
    const Derived d = derive(p);
    const SampleOut<double> o = run_sample(p, d, i);
    rec[QSO_S_MU] = o.mu; rec[QSO_S_SIG2] = o.sig2; rec[QSO_S_THX] = o.thx;
    rec[QSO_S_THY] = o.thy; rec[QSO_S_SIGTH] = o.sigth; rec[QSO_S_AEFF] = p->a0 * o.aeff_ratio;
    rec[QSO_S_CHIMAX] = o.chimax; rec[QSO_S_GAMMA0] = o.gamma0;
    rec[QSO_S_X] = o.x; rec[QSO_S_Y] = o.y; rec[QSO_S_Z] = o.z;
    return std::isfinite(o.mu) && std::isfinite(o.sig2) ? 0 : -2;
}

int qso_deposit(double v, double s, int32_t dep, double ksig, double lo, double hi, int32_t n,
                double *hist) {
    if (!(hi > lo) || n < 1 || !std::isfinite(v) || !(s >= 0)) return -1;
    deposit<double>(v, s, dep, ksig, lo, hi, n, hist);
    return 0;
}

int qso_forward(const qso_problem *p, int64_t i_begin, int64_t i_end, int nthreads,
                double *energy_hist, double *angle_hist, double *a0eff_hist, double *moments) {
    if (validate(p) || i_begin < 0 || i_end < i_begin || i_end > p->n_samples) return -1;
    const Derived d = derive(p);
    if (p->rr_model == QSO_RR_QUANTUM) table();
    if (nthreads < 1) nthreads = omp_get_max_threads();
    const int ne = p->n_e, nt = p->n_th, na = p->n_a;
    const int64_t total = i_end - i_begin;
    enum { S1E, S2E, S1X, S2X, S1Y, S2Y, SAEFF, SRAD, SSIGF, NSUM };
    std::vector<std::vector<double>> he(nthreads, std::vector<double>(ne + 2, 0.0));
    std::vector<std::vector<double>> ht(nthreads, std::vector<double>(nt + 2, 0.0));
    std::vector<std::vector<double>> ha(nthreads, std::vector<double>(na, 0.0));
    std::vector<std::vector<KSum>> sums(nthreads, std::vector<KSum>(NSUM));
    std::vector<double> chimax(nthreads, 0.0);
    std::vector<int> bad(nthreads, 0);
#pragma omp parallel num_threads(nthreads)
    {
        const int t = omp_get_thread_num();
        const int nth = omp_get_num_threads();
        /* fixed contiguous range per thread, merged in thread order below */
        const int64_t b = i_begin + total * t / nth, e = i_begin + total * (t + 1) / nth;
        for (int64_t i = b; i < e; ++i) {
            const SampleOut<double> o = run_sample(p, d, i);
            if (!std::isfinite(o.mu) || !std::isfinite(o.sig2)) { bad[t] = 1; continue; }
            const double sigf = std::sqrt(std::fmax(o.sig2, 0.0));
            deposit<double>(o.mu, sigf, p->deposit, p->kernel_sigma_bins, p->e_lo, p->e_hi, ne,
                            he[t].data());
            deposit<double>(o.thx, o.sigth, p->deposit, p->kernel_sigma_bins, p->th_lo_mrad,
                            p->th_hi_mrad, nt, ht[t].data());
            /* a0,eff histogram: NGP over a0,eff / a0 in [0, 1], top edge closed */
            int ka = (int)std::floor(o.aeff_ratio * na);
            if (ka > na - 1) ka = na - 1;
            if (ka < 0) ka = 0;
            ha[t][ka] += 1.0;
            const double de = o.mu - p->gamma0;
            sums[t][S1E].add(de);
            sums[t][S2E].add(de * de + std::fmax(o.sig2, 0.0));
            sums[t][S1X].add(o.thx);
            sums[t][S2X].add(o.thx * o.thx + o.sigth * o.sigth);
            sums[t][S1Y].add(o.thy);
            sums[t][S2Y].add(o.thy * o.thy);
            sums[t][SAEFF].add(p->a0 * o.aeff_ratio);
            sums[t][SRAD].add(1.0 - o.mu / o.gamma0);
            sums[t][SSIGF].add(sigf);
            chimax[t] = std::fmax(chimax[t], o.chimax);
        }
    }
    for (int t = 1; t < nthreads; ++t) {
        for (int k = 0; k < ne + 2; ++k) he[0][k] += he[t][k];
        for (int k = 0; k < nt + 2; ++k) ht[0][k] += ht[t][k];
        for (int k = 0; k < na; ++k) ha[0][k] += ha[t][k];
        for (int m = 0; m < NSUM; ++m) {
            sums[0][m].add(sums[t][m].s);
            sums[0][m].add(sums[t][m].c);
        }
        chimax[0] = std::fmax(chimax[0], chimax[t]);
    }
    for (int t = 0; t < nthreads; ++t) if (bad[t]) return -2;
    if (energy_hist) std::memcpy(energy_hist, he[0].data(), sizeof(double) * (ne + 2));
    if (angle_hist) std::memcpy(angle_hist, ht[0].data(), sizeof(double) * (nt + 2));
    if (a0eff_hist) std::memcpy(a0eff_hist, ha[0].data(), sizeof(double) * na);
    if (moments) {
        for (int m = 0; m < QSO_M_N; ++m) moments[m] = 0.0;
        const double W = (double)total;
        moments[QSO_M_WEIGHT] = W;
        if (total > 0) {
            const double m1 = sums[0][S1E].value() / W;
            moments[QSO_M_MEAN_G] = p->gamma0 + m1;
            moments[QSO_M_STD_G] = std::sqrt(std::fmax(sums[0][S2E].value() / W - m1 * m1, 0.0));
            moments[QSO_M_MEAN_THX] = sums[0][S1X].value() / W;
            moments[QSO_M_RMS_THX] = std::sqrt(sums[0][S2X].value() / W);
            moments[QSO_M_MEAN_THY] = sums[0][S1Y].value() / W;
            moments[QSO_M_RMS_THY] = std::sqrt(sums[0][S2Y].value() / W);
            moments[QSO_M_MEAN_AEFF] = sums[0][SAEFF].value() / W;
            moments[QSO_M_MAX_CHI] = chimax[0];
            moments[QSO_M_RAD_FRAC] = sums[0][SRAD].value() / W;
            moments[QSO_M_MEAN_SIGF] = sums[0][SSIGF].value() / W;
        }
    }
    return 0;
}

/* ---- plane-wave reconstruction (Sec. 3.2, Sec. 3.3) --------------------- */
/* The paper rebuilds the 3D spectrum from plane-wave runs over a uniform
 * discrete set of a0,eff values weighted by dN_b/da0,eff: every volume element
 * takes the plane-wave result at its a0,eff.  In A0EFF mode a sample's
 * trajectory depends only on its a0,eff and its initial Lorentz factor, so the
 * plane-wave runs are made on the nodes
 *   a_k     = a0 k / (K - 1),                          k = 0 .. K-1,
 *   gamma_m = gamma0 + 6 sigma_gamma (2 m / (M - 1) - 1), m = 0 .. M-1
 * (M = 1, gamma_0 = gamma0, when sigma_gamma = 0; six standard deviations
 * hold every Box-Muller normal drawn from 24-bit uniforms, |n| <= 5.89).
 * Steps:
 *   1. the plane-wave runs: the moment system at every node (a_k, gamma_m);
 *   2. each sample takes the bilinear interpolant, at (a0,eff, gamma0_i), of
 *      the nodes' final mean, variance and largest chi; the bilinear weights
 *      summed over the samples are the node weights H_n (the discrete joint
 *      distribution of a0,eff and gamma0);
 *   3. the sample is deposited as in the direct pass, with its own direction
 *      and a0,eff (Sec. 5.2 width from its interpolated state).
 * (Reading: the weighted sum of the paper is taken with the weights carried
 * by the samples rather than by bins of a0,eff, so that node laws narrower
 * than the node spacing are not mixed into a comb.)                        */
/* The node grid, its plane-wave runs, and the interpolated state of a sample. */
struct NodeGrid {
    int K = 0, M = 0;
    double g_lo = 0.0, g_step = 0.0;
    std::vector<SampleOut<double>> node;  /* node n = k M + m */

    /* 1. the plane-wave runs; returns -2 on a non-finite node state */
    int run(const qso_problem *p, const Derived &d, const Params<double> &P, int K_, int M_,
            int nthreads) {
        K = K_;
        M = M_;
        g_lo = p->gamma0 - 6.0 * p->sigma_gamma;
        g_step = M > 1 ? 12.0 * p->sigma_gamma / (M - 1) : 0.0;
        node.assign((size_t)K * M, SampleOut<double>{});
        int bad = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) reduction(| : bad)
        for (int n = 0; n < K * M; ++n) {
            const int k = n / M, m = n % M;
            SampleIn<double> s{};
            s.gamma0 = M > 1 ? g_lo + m * g_step : p->gamma0;
            Geometry<double> gmt{};
            gmt.S0 = (double)k / (K - 1);
            NoVisit none;
            node[n] = evolve<double>(p, d, P, s, gmt, none);
            if (!std::isfinite(node[n].mu) || !std::isfinite(node[n].sig2)) bad = 1;
        }
        return bad ? -2 : 0;
    }

    /* 2. bilinear weights w[4] on nodes idx[4] at (S0 = a0,eff / a0, gamma0) */
    void weights(double S0, double gamma0, double w[4], int idx[4]) const {
        const double ta = S0 * (K - 1);
        int k = (int)std::floor(ta);
        if (k > K - 2) k = K - 2;
        if (k < 0) k = 0;
        const double fa = ta - k;
        int m = 0;
        double fg = 0.0;
        if (M > 1) {
            double tg = (gamma0 - g_lo) / g_step;
            if (tg < 0.0) tg = 0.0;
            if (tg > M - 1) tg = M - 1;
            m = (int)std::floor(tg);
            if (m > M - 2) m = M - 2;
            fg = tg - m;
        }
        const int n00 = k * M + m, n10 = n00 + M;
        w[0] = (1.0 - fa) * (1.0 - fg);
        w[1] = fa * (1.0 - fg);
        w[2] = M > 1 ? (1.0 - fa) * fg : 0.0;
        w[3] = M > 1 ? fa * fg : 0.0;
        idx[0] = n00;
        idx[1] = n10;
        idx[2] = M > 1 ? n00 + 1 : n00;
        idx[3] = M > 1 ? n10 + 1 : n10;
    }

    /* the sample's interpolated final state and observables (its own draw,
     * direction and a0,eff) */
    SampleOut<double> sample(const qso_problem *p, const Params<double> &P, int64_t i, double w[4],
                             int idx[4]) const {
        const SampleIn<double> s = make_sample<double>(p, P, i);
        const Geometry<double> gmt = geometry<double>(p, P, s);
        weights(gmt.S0, s.gamma0, w, idx);
        SampleOut<double> o{};
        o.mu = 0.0;
        o.sig2 = 0.0;
        o.chimax = 0.0;
        for (int q = 0; q < 4; ++q) {
            o.mu += w[q] * node[idx[q]].mu;
            o.sig2 += w[q] * node[idx[q]].sig2;
            o.chimax += w[q] * node[idx[q]].chimax;
        }
        const double sigf = std::sqrt(std::fmax(o.sig2, 0.0));
        const double aeff = P.a0 * gmt.S0;
        o.thx = 1e3 * s.thx;
        o.thy = 1e3 * s.thy;
        o.sigth = 1e3 * p->c_theta * std::sqrt(2.0 / kPi) * aeff * sigf / (o.mu * o.mu);
        o.aeff_ratio = gmt.S0;
        o.gamma0 = s.gamma0;
        o.x = s.x; o.y = s.y; o.z = s.z;
        return o;
    }
};

bool valid_grid(const qso_problem *p, int32_t n_anodes, int32_t n_gnodes) {
    if (p->amp_mode != QSO_AMP_A0EFF || n_anodes < 2) return false;
    return p->sigma_gamma > 0.0 ? n_gnodes >= 2 : n_gnodes == 1;
}

int qso_factorised(const qso_problem *p, int32_t n_anodes, int32_t n_gnodes, int64_t i_begin,
                   int64_t i_end, int nthreads, double *energy_hist, double *angle_hist,
                   double *a0eff_hist, double *moments, double *node_states,
                   double *node_weights) {
    if (validate(p) || i_begin < 0 || i_end < i_begin || i_end > p->n_samples) return -1;
    if (!valid_grid(p, n_anodes, n_gnodes)) return -1;
    const Derived d = derive(p);
    if (p->rr_model == QSO_RR_QUANTUM) table();
    if (nthreads < 1) nthreads = omp_get_max_threads();
    Params<double> P = params<double>(p);
    finish_params(p, P);
    NodeGrid grid;
    if (grid.run(p, d, P, n_anodes, n_gnodes, nthreads)) return -2;
    const int NN = n_anodes * n_gnodes;

    /* 2-3. samples: interpolated plane-wave state, deposit, node weights */
    const int ne = p->n_e, nt = p->n_th, na = p->n_a;
    const int64_t total = i_end - i_begin;
    enum { S1E, S2E, S1X, S2X, S1Y, S2Y, SAEFF, SRAD, SSIGF, NSUM };
    std::vector<std::vector<double>> hw(nthreads, std::vector<double>(NN, 0.0));
    std::vector<std::vector<double>> he(nthreads, std::vector<double>(ne + 2, 0.0));
    std::vector<std::vector<double>> ht(nthreads, std::vector<double>(nt + 2, 0.0));
    std::vector<std::vector<double>> ha(nthreads, std::vector<double>(na, 0.0));
    std::vector<std::vector<KSum>> sums(nthreads, std::vector<KSum>(NSUM));
    std::vector<double> chimax(nthreads, 0.0);
#pragma omp parallel num_threads(nthreads)
    {
        const int t = omp_get_thread_num();
        const int nth = omp_get_num_threads();
        const int64_t b = i_begin + total * t / nth, e = i_begin + total * (t + 1) / nth;
        for (int64_t i = b; i < e; ++i) {
            double w[4];
            int idx[4];
            const SampleOut<double> o = grid.sample(p, P, i, w, idx);
            for (int q = 0; q < 4; ++q) hw[t][idx[q]] += w[q];
            const double sigf = std::sqrt(std::fmax(o.sig2, 0.0));
            deposit<double>(o.mu, sigf, p->deposit, p->kernel_sigma_bins, p->e_lo, p->e_hi, ne,
                            he[t].data());
            deposit<double>(o.thx, o.sigth, p->deposit, p->kernel_sigma_bins, p->th_lo_mrad,
                            p->th_hi_mrad, nt, ht[t].data());
            int ka = (int)std::floor(o.aeff_ratio * na);
            if (ka > na - 1) ka = na - 1;
            if (ka < 0) ka = 0;
            ha[t][ka] += 1.0;
            const double de = o.mu - p->gamma0;
            sums[t][S1E].add(de);
            sums[t][S2E].add(de * de + std::fmax(o.sig2, 0.0));
            sums[t][S1X].add(o.thx);
            sums[t][S2X].add(o.thx * o.thx + o.sigth * o.sigth);
            sums[t][S1Y].add(o.thy);
            sums[t][S2Y].add(o.thy * o.thy);
            sums[t][SAEFF].add(p->a0 * o.aeff_ratio);
            sums[t][SRAD].add(1.0 - o.mu / o.gamma0);
            sums[t][SSIGF].add(sigf);
            chimax[t] = std::fmax(chimax[t], o.chimax);
        }
    }
    for (int t = 1; t < nthreads; ++t) {
        for (int n = 0; n < NN; ++n) hw[0][n] += hw[t][n];
        for (int k = 0; k < ne + 2; ++k) he[0][k] += he[t][k];
        for (int k = 0; k < nt + 2; ++k) ht[0][k] += ht[t][k];
        for (int k = 0; k < na; ++k) ha[0][k] += ha[t][k];
        for (int q = 0; q < NSUM; ++q) {
            sums[0][q].add(sums[t][q].s);
            sums[0][q].add(sums[t][q].c);
        }
        chimax[0] = std::fmax(chimax[0], chimax[t]);
    }
    if (energy_hist) std::memcpy(energy_hist, he[0].data(), sizeof(double) * (ne + 2));
    if (angle_hist) std::memcpy(angle_hist, ht[0].data(), sizeof(double) * (nt + 2));
    if (a0eff_hist) std::memcpy(a0eff_hist, ha[0].data(), sizeof(double) * na);
    if (node_weights) std::memcpy(node_weights, hw[0].data(), sizeof(double) * NN);
    if (node_states) {
        for (int n = 0; n < NN; ++n) {
            double *r = node_states + (size_t)n * QSO_N_N;
            r[QSO_N_A] = p->a0 * ((double)(n / n_gnodes) / (n_anodes - 1));
            r[QSO_N_GAMMA0] = grid.node[n].gamma0;
            r[QSO_N_MU] = grid.node[n].mu;
            r[QSO_N_SIG2] = grid.node[n].sig2;
            r[QSO_N_CHIMAX] = grid.node[n].chimax;
        }
    }
    if (moments) {
        for (int q = 0; q < QSO_M_N; ++q) moments[q] = 0.0;
        const double W = (double)total;
        moments[QSO_M_WEIGHT] = W;
        if (total > 0) {
            const double m1 = sums[0][S1E].value() / W;
            moments[QSO_M_MEAN_G] = p->gamma0 + m1;
            moments[QSO_M_STD_G] = std::sqrt(std::fmax(sums[0][S2E].value() / W - m1 * m1, 0.0));
            moments[QSO_M_MEAN_THX] = sums[0][S1X].value() / W;
            moments[QSO_M_RMS_THX] = std::sqrt(sums[0][S2X].value() / W);
            moments[QSO_M_MEAN_THY] = sums[0][S1Y].value() / W;
            moments[QSO_M_RMS_THY] = std::sqrt(sums[0][S2Y].value() / W);
            moments[QSO_M_MEAN_AEFF] = sums[0][SAEFF].value() / W;
            moments[QSO_M_MAX_CHI] = chimax[0];
            moments[QSO_M_RAD_FRAC] = sums[0][SRAD].value() / W;
            moments[QSO_M_MEAN_SIGF] = sums[0][SSIGF].value() / W;
        }
    }
    return 0;
}

int qso_factorised_samples(const qso_problem *p, int32_t n_anodes, int32_t n_gnodes,
                           int64_t n_idx, const int64_t *idx, int nthreads, double *recs) {
    if (validate(p) || !valid_grid(p, n_anodes, n_gnodes) || n_idx < 0) return -1;
    for (int64_t r = 0; r < n_idx; ++r)
        if (idx[r] < 0 || idx[r] >= p->n_samples) return -1;
    const Derived d = derive(p);
    if (p->rr_model == QSO_RR_QUANTUM) table();
    if (nthreads < 1) nthreads = omp_get_max_threads();
    Params<double> P = params<double>(p);
    finish_params(p, P);
    NodeGrid grid;
    if (grid.run(p, d, P, n_anodes, n_gnodes, nthreads)) return -2;
    for (int64_t r = 0; r < n_idx; ++r) {
        double w[4];
        int ix[4];
        const SampleOut<double> o = grid.sample(p, P, idx[r], w, ix);
        double *rec = recs + (size_t)r * QSO_S_N;
        rec[QSO_S_MU] = o.mu; rec[QSO_S_SIG2] = o.sig2; rec[QSO_S_THX] = o.thx;
        rec[QSO_S_THY] = o.thy; rec[QSO_S_SIGTH] = o.sigth; rec[QSO_S_AEFF] = p->a0 * o.aeff_ratio;
        rec[QSO_S_CHIMAX] = o.chimax; rec[QSO_S_GAMMA0] = o.gamma0;
        rec[QSO_S_X] = o.x; rec[QSO_S_Y] = o.y; rec[QSO_S_Z] = o.z;
    }
    return 0;
}

/* ---- photon angular distribution (Sec. 5.1) --------------------------------- */
/* Photons leave along the electron's direction within a cone of about 1/gamma.
 * In a linearly polarised plane wave the transverse momentum in the
 * polarisation plane is the vector potential, so at a stage with amplitude a
 * and mean energy mu the emission angle in x is theta_x + a / mu (theta_x the
 * sample's own direction) and in y is theta_y; the cone adds 1 / mu^2 to the
 * mean square in each plane (reading: rms 1/gamma per plane).  The paper's
 * photon-number weighting (theta^2 averaged with N_gamma / N_e over the
 * a0,eff distribution) is taken per stage: each RK4 stage emits
 *   dN = C_ph (w / mu) Phi(1; chi)   photons (the LCFA number over all
 *                                     photon energies, Sec. 4),
 *   dE = -w A                         in photon energy (the drift),
 * with the stage weights w of the phase quadrature.  out[6] = {total number,
 * rms theta_x and theta_y weighted by number [mrad], emitted energy, rms
 * theta_x and theta_y weighted by energy [mrad]}. */
int qso_photon_angles(const qso_problem *p, int64_t i_begin, int64_t i_end, int nthreads,
                      double *out) {
    if (validate(p) || i_begin < 0 || i_end < i_begin || i_end > p->n_samples || !out) return -1;
    const Derived d = derive(p);
    if (p->rr_model == QSO_RR_QUANTUM) table();
    photon_table();
    if (nthreads < 1) nthreads = omp_get_max_threads();
    const int64_t total = i_end - i_begin;
    const double c_ph = kAlpha * d.aS / (2.0 * std::sqrt(3.0) * kPi);
    enum { N, NX, NY, E, EX, EY, NS };
    std::vector<std::vector<KSum>> S(nthreads, std::vector<KSum>(NS));
    std::vector<int> bad(nthreads, 0);
    Params<double> P = params<double>(p);
    finish_params(p, P);
#pragma omp parallel num_threads(nthreads)
    {
        const int t = omp_get_thread_num();
        const int nth = omp_get_num_threads();
        const int64_t b = i_begin + total * t / nth, e = i_begin + total * (t + 1) / nth;
        std::vector<KSum> &acc = S[t];
        double thx = 0.0, thy = 0.0;
        auto visit = [&](double w, const double &mu, const double &a, const Rhs<double> &k) {
            const double chi = 2.0 * mu * std::fabs(a) / d.aS;
            if (!(chi > 0.0)) return;
            const double dN = c_ph * w / mu * PhotonRow(chi).total();
            const double dE = -w * k.A;
            const double tx = thx + a / mu, cone = 1.0 / (mu * mu);
            const double x2 = tx * tx + cone, y2 = thy * thy + cone;
            acc[N].add(dN);
            acc[NX].add(dN * x2);
            acc[NY].add(dN * y2);
            acc[E].add(dE);
            acc[EX].add(dE * x2);
            acc[EY].add(dE * y2);
        };
        for (int64_t i = b; i < e; ++i) {
            const SampleIn<double> s = make_sample<double>(p, P, i);
            thx = s.thx;
            thy = s.thy;
            const SampleOut<double> o = run_sample<double>(p, d, P, i, visit);
            if (!std::isfinite(o.mu) || !std::isfinite(o.sig2)) bad[t] = 1;
        }
    }
    for (int t = 1; t < nthreads; ++t)
        for (int m = 0; m < NS; ++m) {
            S[0][m].add(S[t][m].s);
            S[0][m].add(S[t][m].c);
        }
    for (int t = 0; t < nthreads; ++t) if (bad[t]) return -2;
    const double n = S[0][N].value(), en = S[0][E].value();
    out[0] = n;
    out[1] = n > 0.0 ? 1e3 * std::sqrt(S[0][NX].value() / n) : 0.0;
    out[2] = n > 0.0 ? 1e3 * std::sqrt(S[0][NY].value() / n) : 0.0;
    out[3] = en;
    out[4] = en > 0.0 ? 1e3 * std::sqrt(S[0][EX].value() / en) : 0.0;
    out[5] = en > 0.0 ? 1e3 * std::sqrt(S[0][EY].value() / en) : 0.0;
    return 0;
}

/* ---- derivatives ---------------------------------------------------------- */
static Params<Dual> seeded_params(const qso_problem *p) {
    Params<Dual> P = params<Dual>(p);
    P.a0.d[0] = 1.0;
    P.w0.d[1] = 1.0;
    P.x_off.d[2] = 1.0;
    P.y_off.d[3] = 1.0;
    P.delay.d[4] = 1.0;
    P.gamma0.d[5] = 1.0;
    P.sigma_gamma.d[6] = 1.0;
    P.div_mrad.d[7] = 1.0;
    finish_params(p, P);
    return P;
}

int qso_flop_tally(const qso_problem *p, int64_t i_begin, int64_t i_end, int32_t n_steps_b,
                   double *out) {
    if (validate(p) || i_begin < 0 || i_end <= i_begin || i_end > p->n_samples ||
        n_steps_b <= p->n_steps)
        return -1;
    if (p->rr_model == QSO_RR_QUANTUM) table();
    qso_problem pb = *p;
    pb.n_steps = n_steps_b;
    const Derived da = derive(p), db = derive(&pb);
    Params<Counted> P = params<Counted>(p);
    finish_params(p, P);
    OpCount tot = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = i_begin; i < i_end; ++i) {
        /* the same sample at two step counts: the difference is the work of
         * n_steps_b - n_steps phase steps (set-up and deposit cancel) */
        g_ops = OpCount{0.0, 0.0, 0.0, 0.0};
        (void)run_sample<Counted>(p, da, P, i);
        const OpCount a = g_ops;
        g_ops = OpCount{0.0, 0.0, 0.0, 0.0};
        (void)run_sample<Counted>(&pb, db, P, i);
        const OpCount b = g_ops;
        tot.add += b.add - a.add;
        tot.mul += b.mul - a.mul;
        tot.div += b.div - a.div;
        tot.trans += b.trans - a.trans;
    }
    const double steps = (double)(i_end - i_begin) * (double)(n_steps_b - p->n_steps);
    out[0] = tot.add / steps;
    out[1] = tot.mul / steps;
    out[2] = tot.div / steps;
    out[3] = tot.trans / steps;
    out[4] = (tot.add + tot.mul + tot.div + tot.trans) / steps;
    /* one amplitude evaluation (spatial factor along the path, times a0 and
     * the envelope), on the first sample at the window centre */
    {
        const SampleIn<Counted> smp = make_sample<Counted>(p, P, i_begin);
        const Geometry<Counted> gmt = geometry<Counted>(p, P, smp);
        g_ops = OpCount{0.0, 0.0, 0.0, 0.0};
        (void)amplitude<Counted>(p, da, P, smp, gmt, 0.0);
        out[5] = g_ops.add + g_ops.mul + g_ops.div + g_ops.trans;
    }
    return 0;
}

int qso_sample_grad(const qso_problem *p, int64_t i, double *out) {
    if (validate(p)) return -1;
    const Derived d = derive(p);
    const Params<Dual> P = seeded_params(p);
    const SampleOut<Dual> o = run_sample<Dual>(p, d, P, i);
    out[0] = o.mu.v;
    out[9] = o.sig2.v;
    for (int k = 0; k < kNP; ++k) {
        out[1 + k] = o.mu.d[k];
        out[10 + k] = o.sig2.d[k];
    }
    return std::isfinite(o.mu.v) && std::isfinite(o.sig2.v) ? 0 : -2;
}

int qso_grad(const qso_problem *p, int64_t i_begin, int64_t i_end, int nthreads, double *hist,
             double *jac) {
    if (validate(p) || i_begin < 0 || i_end < i_begin || i_end > p->n_samples) return -1;
    const Derived d = derive(p);
    if (p->rr_model == QSO_RR_QUANTUM) table();
    if (nthreads < 1) nthreads = omp_get_max_threads();
    const int ne = p->n_e;
    const int64_t total = i_end - i_begin;
    const Params<Dual> P = seeded_params(p);
    std::vector<std::vector<Dual>> he(nthreads, std::vector<Dual>(ne + 2, Dual(0.0)));
    std::vector<int> bad(nthreads, 0);
#pragma omp parallel num_threads(nthreads)
    {
        const int t = omp_get_thread_num();
        const int nth = omp_get_num_threads();
        const int64_t b = i_begin + total * t / nth, e = i_begin + total * (t + 1) / nth;
        for (int64_t i = b; i < e; ++i) {
            const SampleOut<Dual> o = run_sample<Dual>(p, d, P, i);
            if (!std::isfinite(o.mu.v) || !std::isfinite(o.sig2.v)) { bad[t] = 1; continue; }
            const Dual sigf = sqrt(fmax(o.sig2, Dual(0.0)));
            deposit<Dual>(o.mu, sigf, p->deposit, p->kernel_sigma_bins, p->e_lo, p->e_hi, ne,
                          he[t].data());
        }
    }
    for (int t = 1; t < nthreads; ++t)
        for (int k = 0; k < ne + 2; ++k) he[0][k] += he[t][k];
    for (int t = 0; t < nthreads; ++t) if (bad[t]) return -2;
    for (int k = 0; k < ne + 2; ++k) {
        if (hist) hist[k] = he[0][k].v;
        if (jac)
            for (int m = 0; m < kNP; ++m) jac[k * kNP + m] = he[0][k].d[m];
    }
    return 0;
}

int qso_grad_outputs(const qso_problem *p, int64_t i_begin, int64_t i_end, int nthreads,
                     double *angle_hist, double *jac_angle, double *moments, double *jac_moments) {
    if (validate(p) || i_begin < 0 || i_end < i_begin || i_end > p->n_samples) return -1;
    const Derived d = derive(p);
    if (p->rr_model == QSO_RR_QUANTUM) table();
    if (nthreads < 1) nthreads = omp_get_max_threads();
    const int nt = p->n_th;
    const int64_t total = i_end - i_begin;
    const Params<Dual> P = seeded_params(p);
    /* the sums of qso_forward, as dual numbers */
    enum { S1E, S2E, S1X, S2X, S1Y, S2Y, SAEFF, SRAD, SSIGF, NSUM };
    std::vector<std::vector<Dual>> ht(nthreads, std::vector<Dual>(nt + 2, Dual(0.0)));
    std::vector<std::vector<Dual>> sums(nthreads, std::vector<Dual>(NSUM, Dual(0.0)));
    std::vector<double> chimax(nthreads, 0.0);
    std::vector<int> bad(nthreads, 0);
#pragma omp parallel num_threads(nthreads)
    {
        const int t = omp_get_thread_num();
        const int nth = omp_get_num_threads();
        const int64_t b = i_begin + total * t / nth, e = i_begin + total * (t + 1) / nth;
        std::vector<Dual> &S = sums[t];
        for (int64_t i = b; i < e; ++i) {
            const SampleOut<Dual> o = run_sample<Dual>(p, d, P, i);
            if (!std::isfinite(o.mu.v) || !std::isfinite(o.sig2.v)) { bad[t] = 1; continue; }
            deposit<Dual>(o.thx, o.sigth, p->deposit, p->kernel_sigma_bins, p->th_lo_mrad,
                          p->th_hi_mrad, nt, ht[t].data());
            const Dual sigf = sqrt(fmax(o.sig2, Dual(0.0)));
            const Dual de = o.mu - P.gamma0;
            S[S1E] += de;
            S[S2E] += de * de + fmax(o.sig2, Dual(0.0));
            S[S1X] += o.thx;
            S[S2X] += o.thx * o.thx + o.sigth * o.sigth;
            S[S1Y] += o.thy;
            S[S2Y] += o.thy * o.thy;
            S[SAEFF] += P.a0 * o.aeff_ratio;
            S[SRAD] += 1.0 - o.mu / o.gamma0;
            S[SSIGF] += sigf;
            chimax[t] = std::fmax(chimax[t], o.chimax);
        }
    }
    for (int t = 1; t < nthreads; ++t) {
        for (int k = 0; k < nt + 2; ++k) ht[0][k] += ht[t][k];
        for (int m = 0; m < NSUM; ++m) sums[0][m] += sums[t][m];
        chimax[0] = std::fmax(chimax[0], chimax[t]);
    }
    for (int t = 0; t < nthreads; ++t) if (bad[t]) return -2;
    for (int k = 0; k < nt + 2; ++k) {
        if (angle_hist) angle_hist[k] = ht[0][k].v;
        if (jac_angle)
            for (int m = 0; m < kNP; ++m) jac_angle[k * kNP + m] = ht[0][k].d[m];
    }
    std::vector<Dual> M(QSO_M_N, Dual(0.0));
    const double W = (double)total;
    M[QSO_M_WEIGHT] = Dual(W);
    if (total > 0) {
        const std::vector<Dual> &S = sums[0];
        const Dual m1 = S[S1E] / W;
        M[QSO_M_MEAN_G] = P.gamma0 + m1;
        M[QSO_M_STD_G] = sqrt(fmax(S[S2E] / W - m1 * m1, Dual(0.0)));
        M[QSO_M_MEAN_THX] = S[S1X] / W;
        M[QSO_M_RMS_THX] = sqrt(S[S2X] / W);
        M[QSO_M_MEAN_THY] = S[S1Y] / W;
        M[QSO_M_RMS_THY] = sqrt(S[S2Y] / W);
        M[QSO_M_MEAN_AEFF] = S[SAEFF] / W;
        M[QSO_M_MAX_CHI] = Dual(chimax[0]);
        M[QSO_M_RAD_FRAC] = S[SRAD] / W;
        M[QSO_M_MEAN_SIGF] = S[SSIGF] / W;
    }
    for (int k = 0; k < QSO_M_N; ++k) {
        if (moments) moments[k] = M[k].v;
        if (jac_moments)
            for (int m = 0; m < kNP; ++m) jac_moments[k * kNP + m] = M[k].d[m];
    }
    return 0;
}

int qso_photon_cdf(double xi, double chi, double *phi, double *total) {
    if (!(chi > 0.0) || !(chi <= 1e3)) return -1;
    const PhotonRow R(chi);
    if (phi) *phi = R.cdf(xi);
    if (total) *total = R.total();
    return 0;
}

int qso_photons(const qso_problem *p, int64_t i_begin, int64_t i_end, int nthreads, int32_t n_ph,
                double ph_lo, double ph_hi, double *hist, double *energy) {
    if (validate(p) || i_begin < 0 || i_end < i_begin || i_end > p->n_samples) return -1;
    if (n_ph < 1 || !(ph_lo >= 0.0) || !(ph_hi > ph_lo) || !std::isfinite(ph_hi)) return -1;
    const Derived d = derive(p);
    if (p->rr_model == QSO_RR_QUANTUM) table();
    photon_table();
    if (nthreads < 1) nthreads = omp_get_max_threads();
    const int64_t total = i_end - i_begin;
    const double width = (ph_hi - ph_lo) / n_ph;
    const double c_ph = kAlpha * d.aS / (2.0 * std::sqrt(3.0) * kPi);
    std::vector<std::vector<double>> H(nthreads, std::vector<double>(n_ph + 2, 0.0));
    std::vector<KSum> eph(nthreads), eel(nthreads);
    std::vector<int> bad(nthreads, 0);
    Params<double> P = params<double>(p);
    finish_params(p, P);
#pragma omp parallel num_threads(nthreads)
    {
        const int t = omp_get_thread_num();
        const int nth = omp_get_num_threads();
        const int64_t b = i_begin + total * t / nth, e = i_begin + total * (t + 1) / nth;
        double *h = H[t].data();
        KSum &ep = eph[t];
        auto visit = [&](double w, const double &mu, const double &a, const Rhs<double> &k) {
            const double chi = 2.0 * mu * std::fabs(a) / d.aS;
            if (!(chi > 0.0)) return;
            ep.add(-w * k.A);  /* photon energy = the drift's energy loss */
            const PhotonRow R(chi);
            photon_deposit(c_ph * w / mu, mu, R, n_ph, ph_lo, width, h);
        };
        for (int64_t i = b; i < e; ++i) {
            const SampleOut<double> o = run_sample<double>(p, d, P, i, visit);
            if (!std::isfinite(o.mu) || !std::isfinite(o.sig2)) { bad[t] = 1; continue; }
            eel[t].add(o.gamma0 - o.mu);
        }
    }
    for (int t = 1; t < nthreads; ++t) {
        for (int k = 0; k < n_ph + 2; ++k) H[0][k] += H[t][k];
        eph[0].add(eph[t].s); eph[0].add(eph[t].c);
        eel[0].add(eel[t].s); eel[0].add(eel[t].c);
    }
    for (int t = 0; t < nthreads; ++t) if (bad[t]) return -2;
    if (hist) std::memcpy(hist, H[0].data(), sizeof(double) * (n_ph + 2));
    if (energy) {
        energy[0] = eph[0].value();
        energy[1] = eel[0].value();
    }
    return 0;
}

}  // extern "C"

