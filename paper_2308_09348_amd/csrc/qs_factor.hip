// qs_factor.hip -- plane-wave reconstruction of the A0EFF forward pass.
//
// Sec. 3.2 rebuilds the 3D spectrum from plane-wave runs over a uniform set
// of a0,eff values weighted by dN_b/da0,eff, and Sec. 3.3 applies it to the
// quantum case.  With the amplitude frozen at a0,eff, a sample's trajectory
// depends only on (a0,eff, gamma0_i), so the plane-wave runs are made once per
// node of an (a0,eff, gamma0) grid and every sample takes their result at its
// own coordinates:
//
//   node pass      (qs_kernels.hip, phase kernel in node mode): the moment
//                  system at every node a_k = a0 k / (K - 1), gamma_m;
//   interpolation  (here): each sample draws its coordinates as in the direct
//                  pass and takes the bilinear interpolant of the nodes' final
//                  mean, variance and largest chi; the bilinear weights summed
//                  over the samples (32.32 fixed point, in LDS) are the node
//                  weights, the discrete joint distribution of (a0,eff,
//                  gamma0);
//   deposit, finalize (qs_kernels.hip): unchanged from the direct pass.
//
// Only the node pass has a phase loop: K M trajectories instead of one per
// sample.  The interpolation pass is one Philox draw, one spatial factor and
// four node reads (L2-resident) per sample.
#include "qs_device.h"

namespace qs {

// One block per deposit tile (dep_tile samples of one shot).  Dynamic LDS:
// the node weights of the tile's shot, when that shot asks for them.
__global__ __launch_bounds__(kDepBlock) void interp_kernel(BatchParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *Hn = reinterpret_cast<unsigned long long *>(smem);
    const int64_t item = blockIdx.x;
    const int s = __builtin_amdgcn_readfirstlane(find_shot(P.shots, P.n_shots, item, true));
    const ShotParams &sp = P.shots[s];
    const int K = sp.n_anode, M = sp.n_gnode;
    const bool weights = P.outs[s].node_weights != nullptr;
    if (weights) {
        for (int k = threadIdx.x; k < K * M; k += blockDim.x) Hn[k] = 0ull;
        __syncthreads();
    }
    const SampleState &nd = P.nst;
    const int64_t i0 = (item - sp.ditem0) * P.dep_tile;
    const int64_t i1 = i0 + P.dep_tile < sp.n_samples ? i0 + P.dep_tile : sp.n_samples;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        double g0, thx, thy, S0;
        Path<double> pd;
        draw_sample(sp, P.key0, P.key1, i, g0, thx, thy, pd, S0);

        // bilinear weights on the node grid (a0,eff / a0 = S0 in [0, 1])
        const double ta = S0 * (double)(K - 1);
        const int k = min((int)ta, K - 2);
        const double fa = ta - (double)k;
        int m = 0;
        double fg = 0.0;
        if (M > 1) {
            const double tg =
                fmin(fmax((g0 - sp.g_node_lo) / sp.g_node_step, 0.0), (double)(M - 1));
            m = min((int)tg, M - 2);
            fg = tg - (double)m;
        }
        const int n00 = k * M + m, n10 = n00 + M;
        const double w[4] = {(1.0 - fa) * (1.0 - fg), fa * (1.0 - fg), (1.0 - fa) * fg, fa * fg};
        const int nn[4] = {n00, n10, M > 1 ? n00 + 1 : n00, M > 1 ? n10 + 1 : n10};
        double mu = 0.0, s2 = 0.0, cmx = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t g = sp.node_off + nn[j];
            mu += w[j] * nd.mu[g];
            s2 += w[j] * nd.s2[g];
            cmx += w[j] * (double)nd.cmx[g];
        }
        const int64_t o = sp.state_off + i;
        P.st.mu[o] = mu;
        P.st.s2[o] = s2;
        P.st.S0[o] = S0;
        P.st.g0[o] = g0;
        P.st.thx[o] = thx;
        P.st.thy[o] = thy;
        P.st.cmx[o] = (float)cmx;

        if (weights) {
            // the four weights rounded to 2^-32 so that they add up to exactly
            // one sample; the rounding remainder (at most two units) goes to
            // the largest
            unsigned long long q[4];
            long long rest = (long long)kOne;
            int big = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                q[j] = (unsigned long long)llrint(w[j] * 4294967296.0);
                rest -= (long long)q[j];
                if (w[j] > w[big]) big = j;
            }
            q[big] = (unsigned long long)((long long)q[big] + rest);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (q[j]) atomicAdd(&Hn[nn[j]], q[j]);
        }
    }
    if (weights) {
        __syncthreads();
        unsigned long long *G = P.hist + sp.hist_off + sp.n_e + 2 + sp.n_th + 2 + sp.n_a;
        for (int k = threadIdx.x; k < K * M; k += blockDim.x) {
            const unsigned long long v = Hn[k];
            if (v) atomicAdd(&G[k], v);
        }
    }
}

// Node records and weights of the shots that ask for them (one block a shot).
__global__ __launch_bounds__(256) void node_outputs_kernel(BatchParams P) {
    const int s = blockIdx.x;
    const ShotParams &sp = P.shots[s];
    const ShotOut &so = P.outs[s];
    const int K = sp.n_anode, M = sp.n_gnode;
    if (so.node_weights) {
        const unsigned long long *H = P.hist + sp.hist_off + sp.n_e + 2 + sp.n_th + 2 + sp.n_a;
        for (int n = threadIdx.x; n < K * M; n += blockDim.x)
            so.node_weights[n] = (double)H[n] * (1.0 / 4294967296.0);
    }
    if (so.node_states) {
        for (int n = threadIdx.x; n < K * M; n += blockDim.x) {
            const int64_t g = sp.node_off + n;
            double *r = so.node_states + (size_t)n * kNodeFields;
            r[0] = sp.a0 * ((double)(n / M) / (double)(K - 1));
            r[1] = P.nst.g0[g];
            r[2] = P.nst.mu[g];
            r[3] = P.nst.s2[g];
            r[4] = (double)P.nst.cmx[g];
        }
    }
}

hipError_t launch_interp(const BatchParams &p, int weight_words, hipStream_t s) {
    const void *fn = reinterpret_cast<const void *>(&interp_kernel);
    const size_t lds = (size_t)weight_words * 8;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (p.n_ditems < 1) return hipSuccess;
    interp_kernel<<<(unsigned)p.n_ditems, kDepBlock, lds, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_node_outputs(const BatchParams &p, hipStream_t s) {
    node_outputs_kernel<<<p.n_shots, 256, 0, s>>>(p);
    return hipGetLastError();
}

}  // namespace qs
