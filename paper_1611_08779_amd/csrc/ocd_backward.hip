// ocd_backward.hip -- adjoint of Algorithm 1 plus the soft output.
//
// The forward update (k, u) computes c = d^-1 (h^H r + g z_old) with
// d^-1 = (g + lambda_k)^-1, so dc/dlambda_k = -d^-1 c, and z_new = proj(c).
// Where a component of c is not clipped it equals that component of z_new, and
// where it is clipped its adjoint is zero; so the adjoint of the update needs
// only z_new (stored per sweep in z_hist), never the residual r:
//   Delta_bar = -h^H r_bar,  t = z_bar + Delta_bar
//   c_bar = t on unclipped parts, 0 on clipped ones (those add sign(z_new) t to beta_bar)
//   lambda_bar_k += -d^-1 Re(conj(z_new) c_bar)
//   z_bar = -Delta_bar + p c_bar,  r_bar += h d^-1 c_bar
// walked backwards over k = K..1, u = U..1, after seeding z_bar from dLoss/dLLR
// through the max-log LLR (and lambda_bar_K through mu and rho).  dLoss/dLLR is
// given, or formed here from the transmitted bits for the mean BCE of the LLRs.  y_bar is r_bar
// at the end; y itself is not read.  Each update costs one lane-local inner
// product, one 2-float all-reduce and one axpy: the work of a forward update.
// A component of z_new equal to +-beta counts as clipped (c exactly at +-beta,
// where the projection's derivative is one-sided, has measure zero).
// Per-sweep and box partial sums go to a per-workgroup slot of the workspace.
// The last workgroup to finish (a completion ticket taken with one device-scope
// atomic from a vector lane) sums them in workgroup order and writes dlambda and
// dbeta: a fixed order, so the gradients are bitwise reproducible, and no second
// launch (finish_partials in ocd_adjoint.h: the partials travel through the
// caches, not the L2s).  The ticket counts to the number of workgroups and is set
// back to zero by that last workgroup, so it is zero again after every launch.
#include "ocd_adjoint.h"

namespace ocd {

// UC > 0: U == UC and the user loop is unrolled: every LDS address of an update is
// a compile-time offset from one base, and the straight-line sweep lets the
// compiler read the next column while the current update computes.  PREFETCH
// (UC > 0, launches with few waves per SIMD): that read is issued one update ahead
// into a second register buffer (same arithmetic).
template <int L, int NPL, bool F16, bool BOX, int UC, bool PREFETCH = false>
__global__ __launch_bounds__(512) void k_backward(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int U = P.U, K = P.K, Bpad = P.Bpad;
    const int Kt = P.per_sweep ? K : 1;
    const int vpb_cap = blockDim.x / L;
    const Smem sm = carve(smem, P, vpb_cap, true);
    const int bid = P.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const Tile t = tile_of(P, bid);
    stagger_loads(P);

    const int grp = threadIdx.x / L, j = threadIdx.x % L;
    const bool active = grp < t.nvb;
    const int v = t.vbase + (active ? grp : 0);
    const int slot = slot_of_group(P, t, active ? grp : 0);

    // H_w staged as in forward_tile (the adjoint never needs the receive vector)
    const int chunks = t.nslots * U * (Bpad >> 1);
    float4 hbuf[STAGE_CHUNKS];
    stage_h_load<F16>(P, t.w_first, t.nslots, chunks, 0, hbuf);
    stage_h_store(P, sm, t.nslots, chunks, 0, hbuf);
    stage_h_copy<F16>(P, sm, t.w_first, t.nslots, chunks, STAGE_CHUNKS * (int)blockDim.x);
    stage_preprocess<L * NPL>(P, sm, t.w_first, t.nslots);
    const float2 *Hs = sm.H + (size_t)slot * P.slot_stride;
    const float2 *dps = sm.dp + (size_t)slot * Kt * U;
    const float *gs = sm.g + (size_t)slot * U;
    const int zr = zrow_of(P, grp);
    float2 *zv = sm.z + (size_t)zr * U;      // z^(k) of the sweep being reversed
    float2 *zb = sm.zbar + (size_t)zr * U;   // dLoss/dz
    const float2 *zh = P.zh_in + (long)v * K * U;

    for (int u = 0; u < U; ++u)
        zv[u] = active ? zh[(size_t)(K - 1) * U + u] : make_float2(0.f, 0.f);

    // soft-output adjoint, one owner lane per user
    const float lamK = P.lambda ? P.lambda[K - 1] : P.lam_default;
    const float2 *dpK = dps + (P.per_sweep ? K - 1 : 0) * U;
    const float sqEs = P.sqEs, scale = P.qscale;
    float lamK_bar = 0.f;
    for (int u = j; u < U; u += L) {
        float2 zbar = make_float2(0.f, 0.f);
        const float gu = gs[u];
        float mu, rho;
        gain_sinr(P, lamK, gu, dpK[u].y, &mu, &rho);
        if (active && rho > 0.f && mu > 0.f) {
            const float s = 1.0f / (mu * sqEs);
            const float2 zu = zv[u];
            const long o = ((long)v * U + u) * P.Q;
            const float *Lbar = P.dllr ? P.dllr + o : nullptr;
            const unsigned char *bt = P.dllr ? nullptr : P.bits + o;
            const float in = P.inv_nbits;
            float dmu = 0.f, drho = 0.f;
            if (P.Q == 2) user_llr_adjoint<1>(Lbar, bt, in, zu.x * s, zu.y * s, s, mu, rho, scale, &zbar, &dmu, &drho);
            else if (P.Q == 4) user_llr_adjoint<2>(Lbar, bt, in, zu.x * s, zu.y * s, s, mu, rho, scale, &zbar, &dmu, &drho);
            else user_llr_adjoint<3>(Lbar, bt, in, zu.x * s, zu.y * s, s, mu, rho, scale, &zbar, &dmu, &drho);
            if (lamK > 0.f) {
                const float dK = dpK[u].x;   // (g + lambda_K)^-1
                lamK_bar = fmaf(drho, -gu / (lamK * lamK), lamK_bar);
                lamK_bar = fmaf(dmu, -gu * dK * dK, lamK_bar);
            }
        }
        zb[u] = zbar;
    }
    lamK_bar = group_sum<L>(lamK_bar);

    float2 rb[NPL];
#pragma unroll
    for (int i = 0; i < NPL; ++i) rb[i] = make_float2(0.f, 0.f);
    const float beta = P.beta;
    float beta_bar = 0.f;
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    // per-wave partial of sweep k, parked in LDS until the end
    auto park_sweep = [&](int k, float lam_bar) {
        const float ws = wave_sum(active && j == 0 ? lam_bar : 0.f);
        if ((threadIdx.x & 63) == 0) sm.part[k * nwaves + wave] = ws;
    };

    // z^(k) rows: lane j owns users j, j + L, ...; with U <= ZPL * L the row of the
    // next sweep is loaded into registers while the current sweep computes
    constexpr int ZPL = 4;
    const bool zpre = U <= ZPL * L;
    float2 znext[ZPL];
    auto fetch_row = [&](int k) {
#pragma unroll
        for (int i = 0; i < ZPL; ++i) {
            const int u = j + i * L;
            const bool ok = active && u < U;
            znext[i] = zh[ok ? (size_t)k * U + u : 0];   // a valid address either way
            if (!ok) znext[i] = make_float2(0.f, 0.f);
        }
    };
    if (zpre && K >= 2) fetch_row(K - 2);
    __syncthreads();   // z_bar rows of every group written (groups never span waves,
                       // so later row updates need only the wave's own LDS order)
    float2 hn[NPL];    // PREFETCH: the next update's column (users run backwards)
    if constexpr (PREFETCH && UC > 0) load_column<L, NPL>(Hs + (UC - 1) * L * NPL, j, hn);
    for (int k = K - 1; k >= 0; --k) {
        if (k < K - 1) {
            if (zpre) {
#pragma unroll
                for (int i = 0; i < ZPL; ++i)
                    if (j + i * L < U) zv[j + i * L] = znext[i];
                if (k >= 1) fetch_row(k - 1);
            } else {
                for (int u = j; u < U; u += L)
                    zv[u] = active ? zh[(size_t)k * U + u] : make_float2(0.f, 0.f);
            }
        }
        __builtin_amdgcn_wave_barrier();   // z^(k) row written by its owner lanes
        const float2 *dpk = dps + (P.per_sweep ? k : 0) * U;
        float lam_bar = (k == K - 1) ? lamK_bar : 0.f;
        if constexpr (UC > 0) {
            constexpr int BP = L * NPL;   // = Bpad: the columns are BP apart
#pragma unroll
            for (int u = UC - 1; u >= 0; --u) {
                float2 h[NPL];
                if constexpr (PREFETCH) {
#pragma unroll
                    for (int i = 0; i < NPL; ++i) h[i] = hn[i];
                    load_column<L, NPL>(Hs + (u > 0 ? u - 1 : UC - 1) * BP, j, hn);
                } else {
                    load_column<L, NPL>(Hs + u * BP, j, h);
                }
                zb[u] = adjoint_update<L, NPL, BOX>(h, dpk[u], zv[u], zb[u], beta, rb, lam_bar,
                                                    beta_bar);
            }
        } else {
            for (int u = U - 1; u >= 0; --u) {
                float2 h[NPL];
                load_column<L, NPL>(Hs + (size_t)u * Bpad, j, h);
                zb[u] = adjoint_update<L, NPL, BOX>(h, dpk[u], zv[u], zb[u], beta, rb, lam_bar,
                                                    beta_bar);
            }
        }
        park_sweep(k, lam_bar);
        __builtin_amdgcn_wave_barrier();
    }
    {
        const float ws = wave_sum(active && j == 0 ? beta_bar : 0.f);
        if ((threadIdx.x & 63) == 0) sm.part[K * nwaves + wave] = ws;
    }
    if (active && P.dy) {
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            const int b = lane_antenna(j, i, L, 2);
            if (b < P.B) P.dy[(long)v * P.B + b] = rb[i];
        }
    }
    __syncthreads();
    // the workgroup's partials: waves summed in order (fixed order, reproducible)
    float *part_out = P.partials + (size_t)bid * (K + 1);
    for (int e = threadIdx.x; e <= K; e += blockDim.x) {
        float sum = 0.f;
        for (int w = 0; w < nwaves; ++w) sum += sm.part[e * nwaves + w];
        store_partial(part_out + e, sum);
    }
    finish_partials(P, K + 1);
}

// Writes dlambda and dbeta (and, with loss, the mean loss) from nblocks
// per-workgroup partials of E entries in a fixed order (thread t adds workgroups
// t, t + 256, ...; fixed cross-lane tree; waves in order).  The adjoint and
// training-step kernels reduce their own partials; this kernel writes the zero
// gradients and loss of an empty problem (nblocks = 0).
__global__ __launch_bounds__(256) void k_reduce_partials(const float *partials, int nblocks, int K,
                                                         int E, int box, float inv_nbits,
                                                         float *dlambda, float *dbeta, float *loss)
{
    __shared__ float red[4];
    const int e = blockIdx.x;   // 0..K-1: dlambda, K: dbeta, K + 1: loss
    float s = 0.f;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partials[(size_t)b * E + e];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float t = (red[0] + red[1]) + (red[2] + red[3]);
        if (e < K) dlambda[e] = t;
        else if (e == K) *dbeta = box ? t : 0.f;
        else *loss = t * inv_nbits;
    }
}

template <int L, int NPL, bool F16, bool BOX, int UC, bool PREFETCH = false>
static hipError_t launch_bwd_u(const Params &p, int threads, size_t lds, hipStream_t s)
{
    auto fn = k_backward<L, NPL, F16, BOX, UC, PREFETCH>;
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

// Exactly 8 or 16 users with at most 8 entries per lane take the unrolled user loop.
template <int L, int NPL, bool F16, bool BOX>
static hipError_t launch_bwd_t(const Params &p, int threads, size_t lds, hipStream_t s)
{
    if constexpr (NPL <= 8) {
        const bool few = latency_bound(p, threads);
        if (p.U == 8)
            return few ? launch_bwd_u<L, NPL, F16, BOX, 8, true>(p, threads, lds, s)
                       : launch_bwd_u<L, NPL, F16, BOX, 8>(p, threads, lds, s);
        if (p.U == 16)
            return few ? launch_bwd_u<L, NPL, F16, BOX, 16, true>(p, threads, lds, s)
                       : launch_bwd_u<L, NPL, F16, BOX, 16>(p, threads, lds, s);
    }
    return launch_bwd_u<L, NPL, F16, BOX, 0>(p, threads, lds, s);
}

template <int L, int NPL>
static hipError_t launch_bwd_ln(bool f16, const Params &p, int threads, size_t lds, hipStream_t s)
{
    if (f16) return p.box ? launch_bwd_t<L, NPL, true, true>(p, threads, lds, s)
                          : launch_bwd_t<L, NPL, true, false>(p, threads, lds, s);
    return p.box ? launch_bwd_t<L, NPL, false, true>(p, threads, lds, s)
                 : launch_bwd_t<L, NPL, false, false>(p, threads, lds, s);
}

template <int L>
static hipError_t launch_bwd_l(int NPL, bool f16, const Params &p, int threads, size_t lds,
                               hipStream_t s)
{
    switch (NPL) {
    case 2: return launch_bwd_ln<L, 2>(f16, p, threads, lds, s);
    case 4: return launch_bwd_ln<L, 4>(f16, p, threads, lds, s);
    case 8: return launch_bwd_ln<L, 8>(f16, p, threads, lds, s);
    case 16: return launch_bwd_ln<L, 16>(f16, p, threads, lds, s);
    case 32: return launch_bwd_ln<L, 32>(f16, p, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_backward(int L, int NPL, bool f16, const Params &p, int threads, size_t lds,
                           hipStream_t s)
{
    switch (L) {
    case 4: return launch_bwd_l<4>(NPL, f16, p, threads, lds, s);
    case 8: return launch_bwd_l<8>(NPL, f16, p, threads, lds, s);
    case 16: return launch_bwd_l<16>(NPL, f16, p, threads, lds, s);
    case 32: return launch_bwd_l<32>(NPL, f16, p, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce_partials(const Params &p, float *dlambda, float *dbeta, float *loss,
                                  hipStream_t s)
{
    const int E = p.K + (loss ? 2 : 1);
    hipLaunchKernelGGL(k_reduce_partials, dim3(E), dim3(256), 0, s, p.partials, p.nblocks, p.K, E,
                       p.box, p.inv_nbits, dlambda, dbeta, loss);
    return hipGetLastError();
}

}  // namespace ocd
