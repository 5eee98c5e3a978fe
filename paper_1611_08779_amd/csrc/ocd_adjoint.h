// ocd_adjoint.h -- device pieces of the adjoint of Algorithm 1 plus the soft
// output, shared by the adjoint kernel and the fused training-step kernel: the
// loss gradient of the mean binary cross-entropy, the soft-output adjoint of one
// user, one reverse coordinate update, and the deterministic hand-off of the
// per-workgroup partial sums to the last workgroup.
#pragma once

#include "ocd_stage.h"

namespace ocd {

// dLoss/dLLR of the mean binary cross-entropy softplus(L) - bit L over n bits
// (P(bit = 1) = sigmoid(L)): (sigmoid(L) - bit) / n, for bit 1 as -sigmoid(-L) / n,
// so that a confidently right bit keeps its small gradient instead of 1 - 1 = 0.
__device__ __forceinline__ float bce_grad(float L, unsigned char bit, float inv_n)
{
    return (bit ? -1.0f / (1.0f + expf(L)) : 1.0f / (1.0f + expf(-L))) * inv_n;
}

// dLoss/dz of one user from dLoss/dLLR through L_b = rho * D_b(x), x = z/(mu sqrt(Es)),
// and the contribution of mu(lambda_K), rho(lambda_K) to dLoss/dlambda_K.  dLoss/dLLR
// is read from Lbar, or (Lbar null) formed from the user's bits for the mean BCE of
// the LLRs, L_b recomputed here.
template <int HALF>
__device__ __forceinline__ void user_llr_adjoint(const float *Lbar, const unsigned char *bits,
                                                 float inv_n, float xr, float xi, float s,
                                                 float mu, float rho, float scale, float2 *zbar,
                                                 float *dmu, float *drho)
{
    float Dr[HALF], Di[HALF];
    axis_llr<HALF>(xr, scale, 1.0f, Dr);
    axis_llr<HALF>(xi, scale, 1.0f, Di);
    float xbr = 0.f, xbi = 0.f, gm = 0.f, gr = 0.f;
#pragma unroll
    for (int bb = 0; bb < HALF; ++bb) {
        const float sr = axis_llr_slope<HALF>(xr, scale, bb);
        const float si = axis_llr_slope<HALF>(xi, scale, bb);
        const float lr = Lbar ? Lbar[bb] : bce_grad(rho * Dr[bb], bits[bb], inv_n);
        const float li = Lbar ? Lbar[HALF + bb] : bce_grad(rho * Di[bb], bits[HALF + bb], inv_n);
        xbr = fmaf(lr * rho, sr, xbr);
        xbi = fmaf(li * rho, si, xbi);
        gr = fmaf(lr, Dr[bb], fmaf(li, Di[bb], gr));
        // dx/dmu = -x/mu
        gm = fmaf(lr * rho * sr, -xr / mu, gm);
        gm = fmaf(li * rho * si, -xi / mu, gm);
    }
    *zbar = make_float2(xbr * s, xbi * s);
    *dmu = gm;
    *drho = gr;
}

// Cross-workgroup hand-off of the partial sums.  The L2 caches of the XCDs are not
// coherent with each other, and a device-scope release fence would write back a
// whole L2 (every dirty line, the adjoint's dy included) once per workgroup.  Only
// the K + 1 partials need to travel, so they bypass the caches instead: they are
// written with device-scope atomic stores (through to the device's coherence
// point), the store is waited for (vmcnt 0) before the ticket is taken, and the last
// workgroup reads them with device-scope atomic loads (through the caches) after
// its ticket returned.
constexpr int WAIT_VMEM_ONLY = 0x0F70;   // s_waitcnt vmcnt(0), expcnt and lgkmcnt not waited

__device__ __forceinline__ void store_partial(float *p, float v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float load_partial(const float *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The last workgroup to take the completion ticket sums every workgroup's E
// partials in workgroup order (thread t adds workgroups t, t + blockDim, ...;
// the waves' lanes by a fixed DPP tree; the waves in order), writes dlambda
// (entries 0 .. K-1), dbeta (entry K) and, with E = K + 2, the mean loss (entry
// K + 1, scaled by 1 / bits), and resets the ticket.  Every thread of the
// workgroup must call it after storing its share of the workgroup's partials with
// store_partial.
__device__ inline void finish_partials(const Params &P, int E)
{
    const int K = P.K;
    __shared__ int last;
    __shared__ float red[8][8];   // [entry of the batch][wave], at most 8 waves
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(WAIT_VMEM_ONLY);   // this thread's partial stores performed
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = __hip_atomic_fetch_add(P.ticket, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        last = t == gridDim.x - 1u;
    }
    __syncthreads();
    if (!last) return;
    __builtin_amdgcn_s_waitcnt(WAIT_VMEM_ONLY);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int nb = gridDim.x;
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    for (int e0 = 0; e0 < E; e0 += 8) {
        float acc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = 0.f;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            const float *pb = P.partials + (size_t)b * E + e0;
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (e0 + i < E) acc[i] += load_partial(pb + i);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = wave_sum(acc[i]);
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int i = 0; i < 8; ++i) red[i][wave] = acc[i];
        __syncthreads();
        const int e = e0 + (int)threadIdx.x;
        if (threadIdx.x < 8 && e < E) {
            float t = 0.f;
            for (int w = 0; w < nwaves; ++w) t += red[threadIdx.x][w];
            if (e < K) P.dlambda[e] = t;
            else if (e == K) *P.dbeta = P.box ? t : 0.f;
            else *P.loss = t * P.inv_nbits;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) __hip_atomic_store(P.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One adjoint coordinate update (the reverse of update (k, u)): returns the new
// z_bar_u, accumulates lambda_bar_k and beta_bar, and adds h d^-1 c_bar to r_bar.
// h: this lane's part of column u; dp = (d_u^-1, p_u); zn = z_u after the update;
// zbu = z_bar_u before.
template <int L, int NPL, bool BOX>
__device__ __forceinline__ float2 adjoint_update(const float2 *h, float2 dp, float2 zn, float2 zbu,
                                                 float beta, float2 *rb, float &lam_bar,
                                                 float &beta_bar)
{
    const float2 hb = group_sum2<L>(partial_inner<NPL, 2>(h, rb));   // h^H r_bar
    const float tr = zbu.x - hb.x, ti = zbu.y - hb.y;                // z_bar + Delta_bar
    float cbr = tr, cbi = ti;
    if constexpr (BOX) {
        if (!(fabsf(zn.x) < beta)) { beta_bar += zn.x > 0.f ? tr : -tr; cbr = 0.f; }
        if (!(fabsf(zn.y) < beta)) { beta_bar += zn.y > 0.f ? ti : -ti; cbi = 0.f; }
    }
    lam_bar = fmaf(-dp.x, fmaf(zn.x, cbr, zn.y * cbi), lam_bar);
    axpy_add<NPL>(h, make_float2(dp.x * cbr, dp.x * cbi), rb);
    return make_float2(hb.x + dp.y * cbr, hb.y + dp.y * cbi);       // -Delta_bar + p c_bar
}


}  // namespace ocd
