// ocd_forward.hip -- the one-problem detection kernel (Algorithm 1 plus the soft
// output, one tile of `vpb` vectors per workgroup) and the standalone
// preprocessing kernel.
#include "ocd_tile.h"

namespace ocd {

template <int L, int NPL, bool F16, bool BOX, int UC, bool PREFETCH = false, bool CHUNKED = false>
__global__ __launch_bounds__(512) void k_forward(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Smem sm = carve(smem, P, blockDim.x / L, false);
    const int bid = P.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    stagger_loads(P);
    forward_tile<L, NPL, F16, BOX, UC, true, PREFETCH, CHUNKED>(P, sm, tile_of(P, bid));
}

// Standalone preprocessing: a 16-lane group per (subcarrier, user) column, lane l
// summing entries l, l + 16, ... and the same DPP tree as the fused staging, so
// both paths give bit-identical g, d^-1 and p.
template <bool F16>
__global__ __launch_bounds__(256) void k_preprocess(Params P, float *g, float *dinv, float *pp)
{
    const int Kt = P.per_sweep ? P.K : 1;
    const long col = (long)blockIdx.x * (blockDim.x >> 4) + (threadIdx.x >> 4);
    const int l16 = threadIdx.x & 15;
    const bool live = col < (long)P.W * P.U;
    float acc = 0.f;
    if (live) {
        for (int b = l16; b < P.B; b += 16) {
            float2 v;
            load_chunk<F16, 1>(P.H, col * P.B + b, b, P.B, false, &v);
            acc = fmaf(v.x, v.x, fmaf(v.y, v.y, acc));
        }
    }
    acc = group_sum<16>(acc);
    if (!live) return;
    const long w = col / P.U;
    const int u = (int)(col - w * P.U);
    if (l16 == 0) g[col] = acc;
    for (int kt = l16; kt < Kt; kt += 16) {
        const float lam = P.lambda ? P.lambda[kt] : P.lam_default;
        const float den = acc + lam;
        const float di = den > 0.f ? 1.0f / den : 0.f;
        const long o = (w * Kt + kt) * P.U + u;
        dinv[o] = di;
        pp[o] = di * acc;
    }
}

template <int L, int NPL, bool F16, bool BOX, int UC, bool PREFETCH = false, bool CHUNKED = false>
static hipError_t launch_fwd_u(const Params &p, int threads, size_t lds, hipStream_t s)
{
    auto fn = k_forward<L, NPL, F16, BOX, UC, PREFETCH, CHUNKED>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    Params q = p;
    if (q.stagger > 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(fn), threads, lds);
        if (e != hipSuccess) return e;
        q.stagger_cap = per_cu * device_cu_count();
    }
    hipLaunchKernelGGL(fn, dim3(q.nblocks), dim3(threads), lds, s, q);
    return hipGetLastError();
}

// Exactly 8 or 16 users with at most 8 entries per lane take the unrolled user loop,
// other multiples of 8 users its chunked form.
template <int L, int NPL, bool F16, bool BOX>
static hipError_t launch_fwd_t(const Params &p, int threads, size_t lds, hipStream_t s)
{
    if constexpr (NPL <= 8) {
        const bool few = latency_bound(p, threads);
        if (p.U == 8)
            return few ? launch_fwd_u<L, NPL, F16, BOX, 8, true>(p, threads, lds, s)
                       : launch_fwd_u<L, NPL, F16, BOX, 8>(p, threads, lds, s);
        if (p.U == 16)
            return few ? launch_fwd_u<L, NPL, F16, BOX, 16, true>(p, threads, lds, s)
                       : launch_fwd_u<L, NPL, F16, BOX, 16>(p, threads, lds, s);
        if (p.U % 8 == 0)
            return launch_fwd_u<L, NPL, F16, BOX, 8, false, true>(p, threads, lds, s);
    }
    return launch_fwd_u<L, NPL, F16, BOX, 0>(p, threads, lds, s);
}

template <int L, int NPL>
static hipError_t launch_fwd_ln(bool f16, const Params &p, int threads, size_t lds, hipStream_t s)
{
    if (f16) return p.box ? launch_fwd_t<L, NPL, true, true>(p, threads, lds, s)
                          : launch_fwd_t<L, NPL, true, false>(p, threads, lds, s);
    return p.box ? launch_fwd_t<L, NPL, false, true>(p, threads, lds, s)
                 : launch_fwd_t<L, NPL, false, false>(p, threads, lds, s);
}

template <int L>
static hipError_t launch_fwd_l(int NPL, bool f16, const Params &p, int threads, size_t lds,
                               hipStream_t s)
{
    switch (NPL) {
    case 2: return launch_fwd_ln<L, 2>(f16, p, threads, lds, s);
    case 4: return launch_fwd_ln<L, 4>(f16, p, threads, lds, s);
    case 8: return launch_fwd_ln<L, 8>(f16, p, threads, lds, s);
    case 16: return launch_fwd_ln<L, 16>(f16, p, threads, lds, s);
    case 32: return launch_fwd_ln<L, 32>(f16, p, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward(int L, int NPL, bool f16, const Params &p, int threads, size_t lds,
                          hipStream_t s)
{
    switch (L) {
    case 4: return launch_fwd_l<4>(NPL, f16, p, threads, lds, s);
    case 8: return launch_fwd_l<8>(NPL, f16, p, threads, lds, s);
    case 16: return launch_fwd_l<16>(NPL, f16, p, threads, lds, s);
    case 32: return launch_fwd_l<32>(NPL, f16, p, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_preprocess(bool f16, const Params &p, float *g, float *dinv, float *pp,
                             hipStream_t s)
{
    const long cols = (long)p.W * p.U;
    if (cols == 0) return hipSuccess;
    const int per_block = 16;   // 16-lane groups of a 256-thread block
    const dim3 grid((unsigned)((cols + per_block - 1) / per_block));
    if (f16) hipLaunchKernelGGL(k_preprocess<true>, grid, dim3(256), 0, s, p, g, dinv, pp);
    else hipLaunchKernelGGL(k_preprocess<false>, grid, dim3(256), 0, s, p, g, dinv, pp);
    return hipGetLastError();
}

}  // namespace ocd
