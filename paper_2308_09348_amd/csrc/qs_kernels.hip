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
#include "qs_device.h"

namespace qs {

// ===========================================================================
// Phase kernel: sample -> ballistic path -> RK4 phase loop -> final state
// ===========================================================================
// The envelope tables come as separate restrict-qualified arguments: the
// kernel never writes them, so the compiler reads them with scalar loads
// (every lane of a wavefront is at the same phase step).
// NODES: the lane runs node i = k n_gnode + m of the shot's plane-wave
// reconstruction grid (a0,eff = a0 k / (n_anode - 1), gamma0 of node m, no
// angles) instead of drawing sample i; the caller passes the node view of the
// shot table (its node count and node offset as samples and state offset).
// FP64 steps of the mixed-precision loop from step j on, for as long as some
// lane of the wavefront has chi above the threshold at the step start: the
// amplitude's spatial factor is carried from one step's end to the next
// step's start, as in the FP64 loop.  Returns the first step not taken.
template <bool QUANTUM, bool MODES>
__device__ __forceinline__ int fp64_segment(const BatchParams &P, const ShotParams &sp,
                                            const Path<double, MODES> &pd, bool local,
                                            double a0S0, const double *__restrict__ env64, int j,
                                            double2 *stage, double &mu, double &s2, float &cmx,
                                            double &chd) {
    const RadTabWave tabd(P.rad64, stage);
    const Phys<double> phd{P.K, P.CD, P.two_over_aS};
    const int N = P.n_steps;
    double aS1 = local ? sp.a0 * pd.S(fma((double)j, P.h, -P.psi_max) * P.ell_per_psi) : a0S0;
    bool more = true;
    while (more) {
        const double psi = fma((double)j, P.h, -P.psi_max);
        double aSh = a0S0, aS4 = a0S0;
        if (local) {
            aSh = sp.a0 * pd.S(fma(0.5, P.h, psi) * P.ell_per_psi);
            aS4 = sp.a0 * pd.S((psi + P.h) * P.ell_per_psi);
        }
        double dm, ds;
        rk4_increment<double, QUANTUM, RadTabWave>(mu, s2, aS1 * env64[2 * j],
                                                   aSh * env64[2 * j + 1], aS4 * env64[2 * j + 2],
                                                   P.h, phd, tabd, dm, ds, chd);
        mu += dm;
        s2 += ds;
        aS1 = aS4;
        ++j;
        if (j >= N) break;
        const double chi = P.two_over_aS * mu * fabs(aS1 * env64[2 * j]);
        cmx = fmaxf(cmx, (float)chi);
        more = __any(chi > (double)P.chi_fp64);
    }
    return j;
}

template <int PREC, bool QUANTUM, bool LOCAL, bool NODES = false, bool MODES = false>
// stage: this wavefront's staging rows for the FP64 table (quantum passes
// with FP64 steps; every lane of the wavefront runs, live says whether the
// lane's sample is real and its state is stored).
__device__ __forceinline__ void phase_sample(const BatchParams &P, const ShotParams &sp, int64_t i,
                                             const float *__restrict__ env32,
                                             const double *__restrict__ env64,
                                             const float *tab32, double2 *stage, bool live,
                                             int &flags, int &nprom) {
    const RadTabWave tabd(P.rad64, stage);
    const RadTab<float> tabf{tab32};
    const Phys<float> phf{P.Kf, P.CDf, P.two_over_aSf};
    const Phys<double> phd{P.K, P.CD, P.two_over_aS};
    const int N = P.n_steps;
    const bool local = LOCAL && !sp.plane_wave;
    const float chi_top = (float)(1 << (kEMax + 1));  // end of the tabulated range

    // ---- sample and geometry (FP64, once per sample) ----
    double g0, thx = 0.0, thy = 0.0, S0;
    Path<double, MODES> pd{};
    if (NODES) {
        static_assert(!NODES || !LOCAL, "nodes carry a fixed amplitude");
        const int k = (int)(i / sp.n_gnode);
        const int m = (int)(i - (int64_t)k * sp.n_gnode);
        S0 = (double)k / (double)(sp.n_anode - 1);
        g0 = sp.gamma0;
        if (sp.n_gnode > 1) {
#pragma clang fp contract(off)
            g0 = sp.g_node_lo + (double)m * sp.g_node_step;  // rounded twice, as defined
        }
    } else {
        draw_sample<MODES>(sp, P.key0, P.key1, i, g0, thx, thy, pd, S0);
    }
    const double a0S0 = sp.a0 * S0;

    double mu_f, s2_f;
    float cmx = 0.0f;     // largest chi at a step start for this sample
    float chi_hi = 0.0f;  // largest chi of the table reads (range check)
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
            rk4_increment<double, QUANTUM, RadTabWave>(mu, s2, a1, ah, a4, P.h, phd, tabd, dm, ds,
                                                       chd);
            mu += dm;
            s2 += ds;
            aS_prev = aS4;
        }
        mu_f = mu;
        s2_f = s2;
        chi_hi = (float)chd;
    } else {
        Path<float, MODES> pf;
        pf.xc = (float)pd.xc;
        pf.yc = (float)pd.yc;
        pf.thx = (float)thx;
        pf.thy = (float)thy;
        pf.zstar = (float)pd.zstar;
        pf.inv_w0sq = sp.inv_w0sqf;
        pf.inv_zR = sp.inv_zRf;
        pf.mode = sp.mode;
        pf.mm = sp.mode_m;
        pf.mn = sp.mode_n;
        pf.inv_norm = sp.mode_inv_normf;
        const float a0f = sp.a0f;
        const float a0S0f = (float)a0S0;
        float mu = (float)g0, mu_lo = (float)(g0 - (double)mu), s2 = 0.0f, s2_lo = 0.0f;
        // the part of g0 that the FP32 pair cannot hold: restored at the end,
        // or taken into the state by the first FP64 step
        double g0_rest = (g0 - (double)mu) - (double)mu_lo;
        double chd = 0.0;
        float aS_prev = local ? a0f * pf.S(P.psi0f * P.ellf) : a0S0f;
        RadCell32 carry;
        AmpQ amp1;  // amplitude factors of the next stage 1
        if (QUANTUM) {
            amp1 = AmpQ(aS_prev * env32[0], phf);
            rad_lookup32(tab32, amp1.cpm * mu, carry);
        }
        // local amplitude: one spatial factor per step, at psi_{j+2}; the
        // stage-2/3 value at psi_j + h/2 is the quadratic through psi_j,
        // psi_{j+1} and psi_{j+2} (error of order h^3 times the third
        // derivative of S, far below FP32 rounding)
        float aS_next = local ? a0f * pf.S((P.psi0f + P.hf) * P.ellf) : a0S0f;
        int j = 0;
        // two steps an iteration: the loop's bookkeeping and the moves of the
        // carried values at its back edge are halved (FP32 quantum pass 3%
        // faster; four steps no faster, with spills)
#pragma clang loop unroll_count(2)
        while (j < N) {
            if (PREC == PREC_F32MIX) {
                const float chi1 = amp1.cpm * mu;
                cmx = fmaxf(cmx, chi1);
                if (__any(chi1 > P.chi_fp64)) {
                    // FP64 steps while any lane of the wavefront has chi above
                    // the threshold at the step start (uniform loop); the FP32
                    // state, amplitudes and cell are rebuilt at the exit step
                    double mud = ((double)mu + (double)mu_lo) + g0_rest;
                    double s2d = (double)s2 + (double)s2_lo;
                    g0_rest = 0.0;
                    const int j0 = j;
                    j = fp64_segment<QUANTUM>(P, sp, pd, local, a0S0, env64, j, stage, mud, s2d,
                                              cmx, chd);
                    nprom += j - j0;  // wave-uniform
                    mu = (float)mud;
                    mu_lo = (float)(mud - (double)mu);
                    s2 = (float)s2d;
                    s2_lo = (float)(s2d - (double)s2);
                    if (local) {
                        aS_prev = a0f * pf.S(fmaf((float)j, P.hf, P.psi0f) * P.ellf);
                        aS_next = a0f * pf.S(fmaf((float)(j + 1), P.hf, P.psi0f) * P.ellf);
                    }
                    if (j < N) {
                        amp1 = AmpQ(aS_prev * env32[2 * j], phf);
                        rad_lookup32(tab32, amp1.cpm * mu, carry);
                    }
                    continue;
                }
            }
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
            if (QUANTUM) {
                if (PREC != PREC_F32MIX) cmx = fmaxf(cmx, amp1.cpm * mu);
                float dm, ds;
                rk4_q32(mu, s2, amp1, ah, a4, P.hf, phf, tab32, carry, dm, ds, chi_hi);
                comp_add(mu, mu_lo, dm);
                comp_add(s2, s2_lo, ds);
            } else {
                cmx = fmaxf(cmx, phf.two_over_aS * mu * fabsf(a1));
                float dm, ds;
                rk4_increment<float, false>(mu, s2, a1, ah, a4, P.hf, phf, tabf, dm, ds, chi_hi);
                comp_add(mu, mu_lo, dm);
            }
            aS_prev = aS4;
            ++j;
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
    if (!live) return;
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

template <int PREC, bool QUANTUM, bool LOCAL, bool NODES = false, bool MODES = false>
__global__ __launch_bounds__(kPhaseBlock)
__attribute__((amdgpu_waves_per_eu((PREC == PREC_F32 && QUANTUM) ? 4 : 1))) void phase_kernel(BatchParams P,
                                                            const float *__restrict__ env32,
                                                            const double *__restrict__ env64) {
    constexpr bool kTab32 = QUANTUM && PREC != PREC_F64;
    // FP64 table staging (quantum passes with FP64 steps): every lane of a
    // wavefront takes part in the table reads, so lanes past the end of the
    // shot run its last sample again without storing it
    constexpr bool kWave64 = QUANTUM && PREC != PREC_F32;
    __shared__ __align__(16) float tab32[kTab32 ? kCells32 * kCellVals : 4];
    __shared__ double2 stage[kWave64 ? (kPhaseBlock / 64) * kStageChunks : 1];
    __shared__ int64_t slot;
    // FP32 passes: the lanes take the item's samples in order of their chi
    // scale (chi_order), so that neighbouring lanes read nearby table cells;
    // with FP64 steps the work items are groups of kChiGroup samples taken in
    // rounds in that order, so that wavefronts step alike
    constexpr bool kOrder = PREC != PREC_F64 && QUANTUM && !NODES;
    constexpr bool kGroup = PREC == PREC_F32MIX && QUANTUM && !NODES;
    constexpr int kOrderN = kGroup ? kChiGroup : kPhaseBlock;
    __shared__ float okey[kOrder ? kOrderN : 1];
    __shared__ unsigned short oidx[kOrder ? kOrderN : 1];
    if (kTab32) {
        const float4 *src = reinterpret_cast<const float4 *>(P.rad32);
        float4 *dst = reinterpret_cast<float4 *>(tab32);
        for (int k = threadIdx.x; k < kCells32 * kCellVals / 4; k += blockDim.x) dst[k] = src[k];
        __syncthreads();
    }
    double2 *wstage = stage + (kWave64 ? (threadIdx.x >> 6) * kStageChunks : 0);
    // one sample (a lane that is not live runs the sample for the
    // wavefront's table reads and stores nothing)
    auto one = [&](const ShotParams &sp, int s, int64_t i, bool live) {
        int flags = 0, nprom = 0;
        phase_sample<PREC, QUANTUM, LOCAL, NODES, MODES>(P, sp, i, env32, env64, tab32, wstage,
                                                         live, flags, nprom);
        if (flags) atomicOr(&P.flags[s], flags);
        if (PREC == PREC_F32MIX && P.fp64_steps != nullptr) {
            // FP64 wave-steps of the wavefronts that hold a sample of the shot
            const bool count = __any(live);
            if (count && nprom > 0 && (threadIdx.x & 63) == 0)
                atomicAdd(&P.fp64_steps[s], (unsigned long long)nprom);
        }
    };
    int s_prev = 0;  // the shot of the block's previous item
    for (;;) {
        const int64_t item = next_item(&P.queue[0], &slot);
        if constexpr (kGroup) {
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
                one(sp, s, base + oidx[live ? rank : cnt - 1], live);
            }
        } else {
            if (item >= P.n_items) break;
            const int s = __builtin_amdgcn_readfirstlane(
                find_shot_from(P.shots, P.n_shots, item, false, s_prev));
            s_prev = s;
            const ShotParams &sp = P.shots[s];
            const int64_t base = (item - sp.item0) * kPhaseBlock;
            int off = threadIdx.x;
            if constexpr (kOrder) {
                chi_order<kPhaseBlock, kPhaseBlock, true>(sp, P.key0, P.key1, base, sp.n_samples,
                                                          okey, oidx);
                off = oidx[threadIdx.x];
            }
            const int64_t i = base + off;
            const bool live = i < sp.n_samples;
            if (kWave64 || live) one(sp, s, live ? i : sp.n_samples - 1, live);
        }
    }
}

// ===========================================================================
// Deposit kernel: final states -> observables -> histograms and moments
// ===========================================================================
// Exclusive prefix sum over the block of one value a thread (256 threads);
// *total receives the sum.
__device__ __forceinline__ unsigned int block_scan(unsigned int v, unsigned int *wsum,
                                                   unsigned int *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    unsigned int before = 0, all = 0;
    for (int w = 0; w < kDepBlock / 64; ++w) {
        if (w < wid) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();  // wsum is reused by the next scan
    *total = all;
    return before + x - v;
}

// Bin masses of one histogram of n bins from the edge accumulators of a tile
// (see wave_deposit): edge e carries T(e) = Q[e] (- QU[e]) + 2^32 C(e), C(e) =
// sum_(c <= e) cnt[c]; bin b gets T(b+1) - T(b), the underflow T(0), the
// overflow 2^32 S - T(n) with S = sum of all cnt (every sample counts once).
// Added to the global words G[0 .. n+1] (bins, underflow, overflow).
template <bool SPLIT>
__device__ void flush_edges(const unsigned long long *Q, const unsigned long long *QU,
                            const unsigned int *cnt, int n, unsigned long long *G,
                            unsigned int *wsum) {
    auto q = [&](int e) { return SPLIT ? Q[e] - QU[e] : Q[e]; };
    const int m = (n + 2 + kDepBlock - 1) / kDepBlock;  // cnt entries a thread
    const int c0 = threadIdx.x * m, c1 = min(c0 + m, n + 2);
    unsigned int local = 0;
    for (int c = c0; c < c1; ++c) local += cnt[c];
    unsigned int S;
    unsigned int C = block_scan(local, wsum, &S);
    const unsigned long long one = kOne;
    unsigned long long prev = c0 >= 1 && c0 <= n + 1 ? q(c0 - 1) + one * C : 0ull;
    for (int e = c0; e < c1 && e <= n; ++e) {
        C += cnt[e];
        const unsigned long long T = q(e) + one * C;
        const long long mass = (long long)(e == 0 ? T : T - prev);
        const int bin = e == 0 ? n : e - 1;
        if (mass > 0) atomicAdd(&G[bin], (unsigned long long)mass);
        if (e == n) {
            const long long over = (long long)(one * S - T);
            if (over > 0) atomicAdd(&G[n + 1], (unsigned long long)over);
        }
        prev = T;
    }
}

// FP64 shadow, histogram level: the bin masses of a sample's law (its own law
// convolved with the deposit kernel, as deposited) from its FP32 state minus
// those from its FP64 state, added to D[n + 2] (bins, underflow n, overflow
// n + 1) in signed fixed point of 2^-40 (the differences are small: units of
// 2^-32 would round most of them away; a word holds up to 2^23 whole masses).  Both laws' CDFs are evaluated exactly
// in FP64, so the difference is that of the two trajectories alone.  Only the
// CDF difference at each edge matters: edge j adds it to the mass below
// (bin j - 1, or the underflow) and subtracts it from the mass above (bin j,
// or the overflow); edges beyond 9 standard deviations of both laws add
// nothing at FP64 precision.
__device__ double law_cdf64(double t, double s, int dep, double ksig, double w) {
    const double r = 0.70710678118654752440;
    if (dep == 2) {  // GAUSS: N(0, s^2 + (ksig bins)^2)
        const double se = sqrt(fma(s, s, (ksig * w) * (ksig * w)));
        return 0.5 * erfc(-t * r / se);
    }
    if (dep == 1) {  // CIC: box one bin wide (x) N(0, s^2)
        const double h = 0.5 * w;
        if (!(s > 0.0)) return fmin(fmax((t + h) / w, 0.0), 1.0);
        auto psi = [&](double x) {  // Int_-inf^x Phi(u / s) du
            return x * 0.5 * erfc(-x * r / s) + s * 0.39894228040143267794 * exp(-0.5 * (x / s) * (x / s));
        };
        return fmin(fmax((psi(t + h) - psi(t - h)) / w, 0.0), 1.0);
    }
    if (!(s > 0.0)) return t > 0.0 ? 1.0 : 0.0;  // POINT: a value on an edge goes up
    return 0.5 * erfc(-t * r / s);
}

__device__ __forceinline__ void shadow_law_diff(double v32, double s32, double v64, double s64, int dep,
                                double ksig, double lo, double w, int n,
                                unsigned long long *D) {
    double reach = 9.0 * fmax(s32, s64) + w;
    if (dep == 2) reach += 9.0 * ksig * w;
    const double a = fmin(v32, v64) - reach, b = fmax(v32, v64) + reach;
    const int ja = (int)fmin(fmax(ceil((a - lo) / w), 0.0), (double)n + 1.0);
    const int jb = (int)fmin(fmax(floor((b - lo) / w), -1.0), (double)n);
    for (int j = ja; j <= jb; ++j) {
        const double e = fma((double)j, w, lo);
        const double d = law_cdf64(e - v32, s32, dep, ksig, w) - law_cdf64(e - v64, s64, dep, ksig, w);
        const long long q = llrint(d * 1099511627776.0);
        if (q == 0) continue;
        atomicAdd(&D[j == 0 ? n : j - 1], (unsigned long long)q);
        atomicAdd(&D[j == n ? n + 1 : j], (unsigned long long)(-q));
    }
}

// One lane per shadowed sample, over the work items of the shadow view
// (P.shots; an item lies within one shot; the FP32 state of shadowed sample q
// is src_off + q draw_stride, its FP64 state state_off + q in P.sst): the law
// differences summed per item in LDS, then added to the shot's words.  A
// kernel of its own keeps the FP64 CDFs off the deposit's register budget.
__global__ __launch_bounds__(kPhaseBlock) void shadow_diff_kernel(BatchParams P, int64_t n_items) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *D = reinterpret_cast<unsigned long long *>(smem);
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int s = __builtin_amdgcn_readfirstlane(find_shot(P.shots, P.n_shots, item, false));
        const ShotParams &sv = P.shots[s];
        const int nd = sv.n_e + 2 + sv.n_th + 2;
        for (int k = threadIdx.x; k < nd; k += blockDim.x) D[k] = 0ull;
        __syncthreads();
        const int64_t q = (item - sv.item0) * kPhaseBlock + threadIdx.x;
        if (q < sv.n_samples) {
            const int64_t k32 = sv.src_off + q * sv.draw_stride, k64 = sv.state_off + q;
            const double mu_f = P.st.mu[k32], s2_f = P.st.s2[k32];
            const double m64 = P.sst.mu[k64];
            if (mu_f > 0.0 && isfinite(mu_f) && isfinite(s2_f) && m64 > 0.0) {
                const double thx_m = 1e3 * P.st.thx[k32];
                const double sigf = sqrt(fmax(s2_f, 0.0)), s64 = sqrt(fmax(P.sst.s2[k64], 0.0));
                // Sec. 5.2 broadening of either state, as deposited
                const double c = 1e3 * P.c_theta * 0.79788456080286535588 * sv.a0 * P.st.S0[k32];
                const double sth32 = c * sigf / (mu_f * mu_f), sth64 = c * s64 / (m64 * m64);
                shadow_law_diff(mu_f, sigf, m64, s64, P.deposit, P.ksig_bins, sv.e_lo, sv.e_w,
                                sv.n_e, D);
                shadow_law_diff(thx_m, sth32, thx_m, sth64, P.deposit, P.ksig_bins, sv.th_lo,
                                sv.th_w, sv.n_th, D + sv.n_e + 2);
            }
        }
        __syncthreads();
        unsigned long long *G = P.shdiff + sv.shd_off;
        for (int k = threadIdx.x; k < nd; k += blockDim.x)
            if (D[k]) atomicAdd(&G[k], D[k]);
        __syncthreads();  // the next item clears D
    }
}

// Held to 128 VGPRs (four waves per SIMD; it takes 131 otherwise, which
// leaves three): one spilled register, a quarter less time.
// SPLIT: the runs' upper-side tails in arrays of their own (16 bytes an edge
// instead of 8; histograms of up to 64 KB of LDS words take it).
template <bool SPLIT>
__global__ __launch_bounds__(kDepBlock) __attribute__((amdgpu_waves_per_eu(4))) void deposit_kernel(
    BatchParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t slot;
    __shared__ double red[kDepBlock / 64][P_N];
    __shared__ float redmax[kDepBlock / 64];
    __shared__ double redsh[kDepBlock / 64][2];
    __shared__ unsigned int wsum[kDepBlock / 64];
    __shared__ int4 wrec[kDepBlock];
    __shared__ int2 wext[kDepBlock];
    __shared__ int woff[kDepBlock], wmark[kDepBlock];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const WaveLaws WL{wrec + 64 * wid, wext + 64 * wid, woff + 64 * wid, wmark + 64 * wid};
    WL.mark[lane] = -1;
    int s_prev = 0;  // the shot of the block's previous item
    for (;;) {
        const int64_t item = next_item(&P.queue[1], &slot);
        if (item >= P.n_ditems) break;
        const int s = __builtin_amdgcn_readfirstlane(
            find_shot_from(P.shots, P.n_shots, item, true, s_prev));
        s_prev = s;
        const ShotParams &sp = P.shots[s];
        const ShotOut &so = P.outs[s];
        const int nh_e = sp.n_e + 2, nh_t = sp.n_th + 2;
        // LDS: edge weights Qe [n_e + 1], Qt [n_th + 1] (u64; SPLIT: and the
        // upper tails QeU [n_e + 1], QtU [n_th + 1]); counters ce [n_e + 2],
        // ct [n_th + 2], ca [n_a] (u32)
        unsigned long long *Qe = reinterpret_cast<unsigned long long *>(smem);
        unsigned long long *Qt = Qe + sp.n_e + 1;
        unsigned long long *QeU = Qt + sp.n_th + 1;
        unsigned long long *QtU = QeU + (SPLIT ? sp.n_e + 1 : 0);
        unsigned int *ce =
            reinterpret_cast<unsigned int *>(SPLIT ? QtU + sp.n_th + 1 : QeU);
        unsigned int *ct = ce + nh_e;
        unsigned int *ca = ct + nh_t;
        const int nq = (SPLIT ? 2 : 1) * (sp.n_e + 1 + sp.n_th + 1), nc = nh_e + nh_t + sp.n_a;
        for (int k = threadIdx.x; k < nq; k += blockDim.x) Qe[k] = 0ull;
        for (int k = threadIdx.x; k < nc; k += blockDim.x) ce[k] = 0u;
        __syncthreads();

        int flags = 0;
        const int64_t i0 = (item - sp.ditem0) * P.dep_tile;
        const int64_t i1 = i0 + P.dep_tile < sp.n_samples ? i0 + P.dep_tile : sp.n_samples;
        const float hfe = (float)(0.5 * sp.e_w), hft = (float)(0.5 * sp.th_w);
        const double inv_we = 1.0 / sp.e_w, inv_wt = 1.0 / sp.th_w;
        for (int64_t t0 = i0; t0 < i1; t0 += kMomTile) {
            const int64_t t1 = t0 + kMomTile < i1 ? t0 + kMomTile : i1;
            double acc[P_N];
#pragma unroll
            for (int m = 0; m < P_N; ++m) acc[m] = 0.0;
            float chimax = 0.0f;
            double emu = 0.0, esig = 0.0;  // FP64 shadow: largest differences
            // every lane runs every round (the wavefront deposit needs them all)
            for (int64_t base = t0; base < t1; base += blockDim.x) {
                const int64_t i = base + threadIdx.x;
                LawLane le{-1, 0, -1, 0, 0.0f, 0.0f, 0.0f}, lt = le;
                if (i < i1) {
                    const int64_t k = sp.state_off + i;
                    const double mu_f = P.st.mu[k], s2_f = P.st.s2[k], S0 = P.st.S0[k];
                    const double g0 = P.st.g0[k];
                    const double thx_m = 1e3 * P.st.thx[k], thy_m = 1e3 * P.st.thy[k];
                    const float cmx = P.st.cmx[k];
                    if (!(mu_f > 0.0) || !isfinite(mu_f) || !isfinite(s2_f)) {
                        flags |= kFlagNonFinite;  // also raised by the phase kernel
                    } else {
                        chimax = fmaxf(chimax, cmx);
                        // Sec. 5.2: the direction is kept, the stochastic broadening
                        // c_theta sqrt(2/pi) a0,eff sigma_f / gamma_f^2 acts in x
                        const double sigf = sqrt(fmax(s2_f, 0.0));
                        const double a_eff = sp.a0 * S0;
                        // 1 / mu_f^2 and 1 / g0 by the hardware reciprocal
                        // and two Newton steps (FP64 rounding)
                        const double mu2 = mu_f * mu_f;
                        double imu2 = __builtin_amdgcn_rcp(mu2), ig0 = __builtin_amdgcn_rcp(g0);
                        imu2 = fma(fma(-mu2, imu2, 1.0), imu2, imu2);
                        imu2 = fma(fma(-mu2, imu2, 1.0), imu2, imu2);
                        ig0 = fma(fma(-g0, ig0, 1.0), ig0, ig0);
                        ig0 = fma(fma(-g0, ig0, 1.0), ig0, ig0);
                        const double sigth =
                            1e3 * P.c_theta * 0.79788456080286535588 * a_eff * sigf * imu2;
                        le = law_setup(mu_f, sigf, P.deposit, P.ksig_bins, sp.e_lo, sp.e_w, inv_we,
                                       sp.n_e);
                        lt = law_setup(thx_m, sigth, P.deposit, P.ksig_bins, sp.th_lo, sp.th_w,
                                       inv_wt, sp.n_th);
                        {
                            int ka = (int)floor(S0 * (double)sp.n_a);
                            ka = min(max(ka, 0), sp.n_a - 1);
                            atomicAdd(&ca[ka], 1u);
                        }
                        const double de = mu_f - sp.gamma0;
                        acc[P_S1E] += de;
                        acc[P_S2E] += fma(de, de, fmax(s2_f, 0.0));
                        acc[P_S1X] += thx_m;
                        acc[P_S2X] += fma(thx_m, thx_m, sigth * sigth);
                        acc[P_S1Y] += thy_m;
                        acc[P_S2Y] += thy_m * thy_m;
                        acc[P_SAEFF] += a_eff;
                        acc[P_SRAD] += fma(-mu_f, ig0, 1.0);
                        acc[P_SSIGF] += sigf;
                        if (sp.shadow_stride > 0 && i % sp.shadow_stride == 0) {
                            // the same sample integrated in FP64
                            const int64_t q = sp.shadow_off + i / sp.shadow_stride;
                            const double m64 = P.sst.mu[q];
                            const double s64 = sqrt(fmax(P.sst.s2[q], 0.0));
                            if (m64 > 0.0) {
                                const double d = mu_f - m64;
                                acc[P_SHN] += 1.0;
                                acc[P_SHMU] += d / m64;
                                acc[P_SHG] += d;
                                emu = fmax(emu, fabs(d) / m64);
                                esig = fmax(esig, fabs(sigf - s64) / m64);
                            }
                        }

                        if (so.samples != nullptr && i % so.rec_stride == 0 &&
                            i / so.rec_stride < so.rec_n) {
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
                }
                wave_deposit<SPLIT>(le, sp.e_w, hfe, Qe, QeU, ce, WL);
                wave_deposit<SPLIT>(lt, sp.th_w, hft, Qt, QtU, ct, WL);
            }

            // ---- moment tile reduction (fixed order) ----
#pragma unroll
            for (int m = 0; m < P_N; ++m) {
                const double v = wave_sum(acc[m]);
                if (lane == 0) red[wid][m] = v;
            }
            const float wm = wave_max(chimax);
            const double we = wave_max(emu), ws = wave_max(esig);
            if (lane == 0) {
                redmax[wid] = wm;
                redsh[wid][0] = we;
                redsh[wid][1] = ws;
            }
            __syncthreads();
            double *part = P.partials + (size_t)(sp.mtile0 + t0 / kMomTile) * kPartials;
            if (threadIdx.x < P_N) {
                double sum = 0.0;
                for (int w = 0; w < kDepBlock / 64; ++w) sum += red[w][threadIdx.x];
                part[threadIdx.x] = sum;
            }
            if (threadIdx.x == 0) {
                float m = 0.0f;
                double e0 = 0.0, e1 = 0.0;
                for (int w = 0; w < kDepBlock / 64; ++w) {
                    m = fmaxf(m, redmax[w]);
                    e0 = fmax(e0, redsh[w][0]);
                    e1 = fmax(e1, redsh[w][1]);
                }
                part[kPMaxChi] = m;
                part[kPMaxEmu] = e0;
                part[kPMaxEsig] = e1;
            }
            __syncthreads();  // red is rewritten by the next tile
        }
        if (flags) atomicOr(&P.flags[s], flags);
        unsigned long long *G = P.hist + sp.hist_off;
        flush_edges<SPLIT>(Qe, QeU, ce, sp.n_e, G, wsum);
        flush_edges<SPLIT>(Qt, QtU, ct, sp.n_th, G + nh_e, wsum);
        for (int k = threadIdx.x; k < sp.n_a; k += blockDim.x)
            if (ca[k]) atomicAdd(&G[nh_e + nh_t + k], kOne * ca[k]);
        __syncthreads();  // the next item clears the LDS words
    }
}

// ===========================================================================
// Finalize: one block per shot, fixed-order reduction of its moment tiles
// ===========================================================================
__global__ __launch_bounds__(256) void finalize_kernel(BatchParams P) {
    const int s = blockIdx.x;
    const ShotParams &sp = P.shots[s];
    const ShotOut &so = P.outs[s];
    const int64_t nd = (sp.n_samples + kMomTile - 1) / kMomTile;
    __shared__ double sums[kPartials];
    __shared__ double tree[256];
    // each column: thread t sums items t, t + 256, ... then a fixed tree
    for (int m = 0; m < kPartials; ++m) {
        double acc = 0.0;
        for (int64_t b = threadIdx.x; b < nd; b += blockDim.x) {
            const double v = P.partials[(size_t)(sp.mtile0 + b) * kPartials + m];
            acc = m >= P_N ? fmax(acc, v) : acc + v;
        }
        tree[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                const double o = tree[threadIdx.x + w];
                tree[threadIdx.x] = m >= P_N ? fmax(tree[threadIdx.x], o) : tree[threadIdx.x] + o;
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
    // FP64 shadow, histogram level: L1 and largest bin of the summed law
    // differences, energy then angle, per shadowed sample
    __shared__ double shd[4];
    if (sp.shadow_stride > 0 && sums[P_SHN] > 0.0) {
        const unsigned long long *D = P.shdiff + sp.shd_off;
        for (int h = 0; h < 2; ++h) {
            const int n0 = h == 0 ? 0 : nh_e, n1 = h == 0 ? nh_e : nh_e + nh_t;
            double l1 = 0.0, mx = 0.0;
            for (int k = n0 + threadIdx.x; k < n1; k += blockDim.x) {
                const double v = fabs((double)(long long)D[k]) * (1.0 / 1099511627776.0);
                l1 += v;
                mx = fmax(mx, v);
            }
            for (int part = 0; part < 2; ++part) {
                tree[threadIdx.x] = part == 0 ? l1 : mx;
                __syncthreads();
                for (int w = 128; w > 0; w >>= 1) {
                    if (threadIdx.x < w) {
                        const double o = tree[threadIdx.x + w];
                        tree[threadIdx.x] = part == 0 ? tree[threadIdx.x] + o : fmax(tree[threadIdx.x], o);
                    }
                    __syncthreads();
                }
                if (threadIdx.x == 0) shd[2 * h + part] = tree[0] / sums[P_SHN];
                __syncthreads();
            }
        }
    }
    if (threadIdx.x == 0) {
        double *M = so.moments;
        for (int m = 0; m < kMoments; ++m) M[m] = 0.0;
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
            M[8] = sums[kPMaxChi];
            M[9] = sums[P_SRAD] / W;
            M[10] = sums[P_SSIGF] / W;
            const double ns = sums[P_SHN];
            if (ns > 0.0) {
                M[11] = ns;
                M[12] = sums[kPMaxEmu];
                M[13] = sums[P_SHMU] / ns;
                M[14] = sums[kPMaxEsig];
                M[15] = sums[P_SHG] / ns;
                for (int q = 0; q < 4; ++q) M[16 + q] = shd[q];
            }
        }
        // share of the wavefront phase steps taken in FP64
        if (P.fp64_steps == nullptr)
            M[20] = -1.0;
        else if (P.prec == PREC_F64)
            M[20] = 1.0;
        else
            M[20] = (double)P.fp64_steps[s] /
                    ((double)((sp.n_samples + 63) / 64) * (double)P.n_steps);
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
// Launchers
// ===========================================================================
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
static const void *phase_ptr(bool modes) {
    if (modes) return reinterpret_cast<const void *>(&phase_kernel<PREC, QUANTUM, LOCAL, false, true>);
    return reinterpret_cast<const void *>(&phase_kernel<PREC, QUANTUM, LOCAL>);
}

// modes: some shot of the launch uses a higher transverse mode
static const void *select_phase(int prec, int rr, int amp, bool modes) {
    const bool q = rr == 1, l = amp == 1;
    if (prec == PREC_F32MIX && !q) prec = PREC_F32;  // no radiation table, no promotion
#define QS_SEL(P)                                              \
    if (prec == P) {                                           \
        if (q && l) return phase_ptr<P, true, true>(modes);    \
        if (q && !l) return phase_ptr<P, true, false>(modes);  \
        if (!q && l) return phase_ptr<P, false, true>(modes);  \
        return phase_ptr<P, false, false>(modes);              \
    }
    QS_SEL(PREC_F32)
    QS_SEL(PREC_F64)
    if (prec == PREC_F32MIX) {
        if (l) return phase_ptr<PREC_F32MIX, true, true>(modes);
        return phase_ptr<PREC_F32MIX, true, false>(modes);
    }
#undef QS_SEL
    return nullptr;
}

hipError_t launch_phase(const BatchParams &p, const float *env32, const double *env64, int prec,
                        int rr, int amp, hipStream_t s) {
    const void *fn = select_phase(prec, rr, amp, p.any_mode != 0);
    if (!fn) return hipErrorInvalidValue;
    // FP64 steps: work items are groups of kChiGroup samples
    const bool grouped = prec == PREC_F32MIX && rr == 1;
    int grid = 0;
    hipError_t e =
        resident_grid(fn, kPhaseBlock, 0, grouped ? p.n_gitems : p.n_items, &grid, p.phase_cap);
    if (e != hipSuccess) return e;
    BatchParams pc = p;
    const float *e32 = env32;
    const double *e64 = env64;
    void *args[] = {&pc, &e32, &e64};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kPhaseBlock), args, 0, s);
}

template <int PREC, bool QUANTUM>
static const void *node_ptr() {
    return reinterpret_cast<const void *>(&phase_kernel<PREC, QUANTUM, false, true>);
}

hipError_t launch_phase_nodes(const BatchParams &p, const float *env32, const double *env64,
                              int prec, int rr, hipStream_t s) {
    const bool q = rr == 1;
    if (prec == PREC_F32MIX && !q) prec = PREC_F32;
    const void *fn = nullptr;
    if (prec == PREC_F32) fn = q ? node_ptr<PREC_F32, true>() : node_ptr<PREC_F32, false>();
    if (prec == PREC_F64) fn = q ? node_ptr<PREC_F64, true>() : node_ptr<PREC_F64, false>();
    if (prec == PREC_F32MIX) fn = node_ptr<PREC_F32MIX, true>();
    if (!fn) return hipErrorInvalidValue;
    int grid = 0;
    hipError_t e = resident_grid(fn, kPhaseBlock, 0, p.n_items, &grid, p.phase_cap);
    if (e != hipSuccess) return e;
    BatchParams pc = p;
    const float *e32 = env32;
    const double *e64 = env64;
    void *args[] = {&pc, &e32, &e64};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kPhaseBlock), args, 0, s);
}

// edge weights (u64, one per edge) and counters (u32, one per bin and two
// more) of the deposit kernel: at most 12 bytes a histogram word (20 with the
// runs' upper tails apart)
size_t deposit_lds_bytes(int max_hist_words) { return (size_t)max_hist_words * 12; }

hipError_t launch_deposit(const BatchParams &p, int max_hist_words, hipStream_t s) {
    const bool split = (size_t)max_hist_words * 20 <= 64 * 1024;
    const void *fn = split ? reinterpret_cast<const void *>(&deposit_kernel<true>)
                           : reinterpret_cast<const void *>(&deposit_kernel<false>);
    const size_t lds = (size_t)max_hist_words * (split ? 20 : 12);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int grid = 0;
    e = resident_grid(fn, kDepBlock, lds, p.n_ditems, &grid, p.dep_cap);
    if (e != hipSuccess) return e;
    BatchParams pc = p;
    void *args[] = {&pc};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kDepBlock), args, lds, s);
}

hipError_t launch_shadow_diff(const BatchParams &p, int64_t n_items, int max_hist_words,
                              hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    const int grid = (int)(n_items < 2048 ? n_items : 2048);
    shadow_diff_kernel<<<grid, kPhaseBlock, (size_t)max_hist_words * 8, s>>>(p, n_items);
    return hipGetLastError();
}

hipError_t launch_finalize(const BatchParams &p, hipStream_t s) {
    finalize_kernel<<<p.n_shots, 256, 0, s>>>(p);
    return hipGetLastError();
}

}  // namespace qs
