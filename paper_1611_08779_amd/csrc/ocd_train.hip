// ocd_train.hip -- one training step of the differentiable detector in one launch:
// Algorithm 1 and the soft output of Section III-C (forward), the mean binary
// cross-entropy of the LLRs against the transmitted bits, and the adjoint of both
// (the reverse sweeps of ocd_backward.hip), for the vectors of one tile.
//
// The two-launch form (ocd_detect with z_hist, then ocd_detect_backward_bce)
// stages every H_w and runs the preprocessing twice and sends the per-sweep
// history of z through HBM.  Here a workgroup stages H_w once, keeps z after every
// sweep in LDS ([vpb + 1][K][U]), writes the LLRs it computes (if asked), seeds
// dLoss/dz from them, and reverses the sweeps on the same staged columns.  The
// forward, the soft output and the reverse updates are the same device code as the
// one-problem kernels (ocd_tile.h, ocd_adjoint.h), so z, the LLRs and dy are those
// of the two-launch form bit for bit; dlambda, dbeta and the loss are reduced in a
// fixed order across workgroups (the last one to finish sums them).
#include "ocd_adjoint.h"

namespace ocd {

// softplus(L) - bit L, the cross-entropy of one bit with P(bit = 1) = sigmoid(L),
// written as max(t, 0) + log(1 + e^-|L|) with t = L for bit 0 and -L for bit 1: a
// bit that is confidently right costs the small second term alone, which the
// subtraction softplus(L) - L would round away in FP32
__device__ __forceinline__ float bce_term(float L, unsigned char bit)
{
    const float t = bit ? -L : L;
    return fmaxf(t, 0.f) + log1pf(expf(-fabsf(L)));
}

template <int L, int NPL, bool F16, bool BOX, int UC>
__global__ __launch_bounds__(512) void k_train(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int U = P.U, K = P.K, Bpad = P.Bpad;
    const int Kt = P.per_sweep ? K : 1;
    const Smem sm = carve(smem, P, blockDim.x / L, true, true);
    const int bid = P.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const Tile t = tile_of(P, bid);
    stagger_loads(P);

    const int grp = threadIdx.x / L, j = threadIdx.x % L;
    const bool active = grp < t.nvb;
    const int v = t.vbase + (active ? grp : 0);
    const int slot = slot_of_group(P, t, active ? grp : 0);

    // staging and preprocessing as in forward_tile (the receive vector's loads in
    // flight with the channel's)
    const int chunks = t.nslots * U * (Bpad >> 1);
    float4 hbuf[STAGE_CHUNKS];
    stage_h_load<F16>(P, t.w_first, t.nslots, chunks, 0, hbuf);
    float2 r[NPL];
    load_vector<L, NPL, F16>(P, P.y, t, grp, j, active, r);
    stage_h_store(P, sm, t.nslots, chunks, 0, hbuf);
    stage_h_copy<F16>(P, sm, t.w_first, t.nslots, chunks, STAGE_CHUNKS * (int)blockDim.x);
    stage_preprocess<L * NPL>(P, sm, t.w_first, t.nslots);
    clear_padding<L, NPL>(P, j, active, r);

    const float2 *Hs = sm.H + (size_t)slot * P.slot_stride;
    const float2 *dps = sm.dp + (size_t)slot * Kt * U;
    const float *gs = sm.g + (size_t)slot * U;
    const int zr = zrow_of(P, grp);
    float2 *zh = sm.zh + (size_t)zr * K * U;   // z^(k) of this vector, [K][U]
    float2 *zb = sm.zbar + (size_t)zr * U;     // dLoss/dz
    const float beta = P.beta;

    // ---- forward: K sweeps over the users in order (Alg. 1), z^(k) into LDS
    if constexpr (UC > 0) {
        constexpr int BP = L * NPL;
        float2 zv[UC];
#pragma unroll
        for (int u = 0; u < UC; ++u) zv[u] = make_float2(0.f, 0.f);
        for (int k = 0; k < K; ++k) {
            const float2 *dpk = dps + (P.per_sweep ? k : 0) * U;
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                float2 h[NPL];
                load_column<L, NPL>(Hs + u * BP, j, h);
                if (u == UC - 1 && k == K - 1)   // r is not read after the last update
                    zv[u] = coordinate_update<L, NPL, BOX, 1, false>(h, dpk[u], zv[u], beta, r);
                else
                    zv[u] = coordinate_update<L, NPL, BOX>(h, dpk[u], zv[u], beta, r);
            }
            // every lane holds the row; lane j stores users j, j + L, ...
#pragma unroll
            for (int u = 0; u < UC; ++u)
                if (u % L == j) zh[k * U + u] = zv[u];
        }
    } else {
        float2 *zcur = sm.z + (size_t)zr * U;
        for (int u = 0; u < U; ++u) zcur[u] = make_float2(0.f, 0.f);   // z^(0) = 0
        for (int k = 0; k < K; ++k) {
            const float2 *dpk = dps + (P.per_sweep ? k : 0) * U;
            for (int u = 0; u < U; ++u) {
                UpdateOperands<NPL> a;
                fetch_operands<L, NPL>(Hs, Bpad, dpk, zcur, u, j, a);
                zcur[u] = coordinate_update<L, NPL, BOX>(a.h, a.dp, a.zo, beta, r);
            }
            for (int u = j; u < U; u += L) zh[k * U + u] = zcur[u];
        }
    }
    __builtin_amdgcn_wave_barrier();   // the rows are complete (groups never span waves)
    const float2 *zK = zh + (size_t)(K - 1) * U;

    // ---- soft output (as forward_tile), its z and LLR outputs, and the loss terms
    float loss_acc = 0.f;
    if (active) {
        if (P.z) {
            float2 *zt = P.z + (size_t)t.vbase * U;
            for (int u = j; u < U; u += L) zt[grp * U + u] = zK[u];
        }
        const int Q = P.Q, half = Q >> 1;
        const float2 *lcs = sm.lc + (size_t)slot * U;
        const unsigned char *bt = P.bits + (size_t)v * U * Q;
        for (int idx = j; idx < 2 * U; idx += L) {
            const int u = idx >> 1, ax = idx & 1;
            const float2 zu = zK[u], co = lcs[u];
            const float tt = (ax ? zu.y : zu.x) * co.x;
            float Lv[3];
            if (half == 3) axis_llrs<3>(tt, co.y, Lv);
            else if (half == 2) axis_llrs<2>(tt, co.y, Lv);
            else axis_llrs<1>(tt, co.y, Lv);
            const int o = u * Q + ax * half;
            for (int b = 0; b < half; ++b) {
                if (P.llr) P.llr[(size_t)v * U * Q + o + b] = Lv[b];
                loss_acc += bce_term(Lv[b], bt[o + b]);
            }
        }
    }

    // ---- adjoint of the soft output and of the loss: dLoss/dz, one owner lane per user
    const float lamK = P.lambda ? P.lambda[K - 1] : P.lam_default;
    const float2 *dpK = dps + (P.per_sweep ? K - 1 : 0) * U;
    float lamK_bar = 0.f;
    for (int u = j; u < U; u += L) {
        float2 zbar = make_float2(0.f, 0.f);
        const float gu = gs[u];
        float mu, rho;
        gain_sinr(P, lamK, gu, dpK[u].y, &mu, &rho);
        if (active && rho > 0.f && mu > 0.f) {
            const float s = 1.0f / (mu * P.sqEs);
            const float2 zu = zK[u];
            const unsigned char *bt = P.bits + ((size_t)v * U + u) * P.Q;
            float dmu = 0.f, drho = 0.f;
            const float in = P.inv_nbits, sc = P.qscale;
            if (P.Q == 2) user_llr_adjoint<1>(nullptr, bt, in, zu.x * s, zu.y * s, s, mu, rho, sc, &zbar, &dmu, &drho);
            else if (P.Q == 4) user_llr_adjoint<2>(nullptr, bt, in, zu.x * s, zu.y * s, s, mu, rho, sc, &zbar, &dmu, &drho);
            else user_llr_adjoint<3>(nullptr, bt, in, zu.x * s, zu.y * s, s, mu, rho, sc, &zbar, &dmu, &drho);
            if (lamK > 0.f) {
                const float dK = dpK[u].x;   // (g + lambda_K)^-1
                lamK_bar = fmaf(drho, -gu / (lamK * lamK), lamK_bar);
                lamK_bar = fmaf(dmu, -gu * dK * dK, lamK_bar);
            }
        }
        zb[u] = zbar;
    }
    lamK_bar = group_sum<L>(lamK_bar);

    // ---- reverse sweeps k = K..1, u = U..1 on the staged columns
    float2 rb[NPL];
#pragma unroll
    for (int i = 0; i < NPL; ++i) rb[i] = make_float2(0.f, 0.f);
    float beta_bar = 0.f;
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    auto park = [&](int e, float x) {   // per-wave partial of entry e, parked in LDS
        const float ws = wave_sum(active && j == 0 ? x : 0.f);
        if ((threadIdx.x & 63) == 0) sm.part[e * nwaves + wave] = ws;
    };
    __builtin_amdgcn_wave_barrier();   // z_bar rows written by their owner lanes
    for (int k = K - 1; k >= 0; --k) {
        const float2 *zvk = zh + (size_t)k * U;
        const float2 *dpk = dps + (P.per_sweep ? k : 0) * U;
        float lam_bar = (k == K - 1) ? lamK_bar : 0.f;
        if constexpr (UC > 0) {
            constexpr int BP = L * NPL;
#pragma unroll
            for (int u = UC - 1; u >= 0; --u) {
                float2 h[NPL];
                load_column<L, NPL>(Hs + u * BP, j, h);
                zb[u] = adjoint_update<L, NPL, BOX>(h, dpk[u], zvk[u], zb[u], beta, rb, lam_bar,
                                                    beta_bar);
            }
        } else {
            for (int u = U - 1; u >= 0; --u) {
                float2 h[NPL];
                load_column<L, NPL>(Hs + (size_t)u * Bpad, j, h);
                zb[u] = adjoint_update<L, NPL, BOX>(h, dpk[u], zvk[u], zb[u], beta, rb, lam_bar,
                                                    beta_bar);
            }
        }
        park(k, lam_bar);
        __builtin_amdgcn_wave_barrier();
    }
    park(K, beta_bar);
    {   // the loss terms of every lane of the group, not only lane 0's
        const float ws = wave_sum(active ? loss_acc : 0.f);
        if ((threadIdx.x & 63) == 0) sm.part[(K + 1) * nwaves + wave] = ws;
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
    const int E = K + 2;
    float *part_out = P.partials + (size_t)bid * E;
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
        float sum = 0.f;
        for (int w = 0; w < nwaves; ++w) sum += sm.part[e * nwaves + w];
        store_partial(part_out + e, sum);
    }
    finish_partials(P, E);
}

template <int L, int NPL, bool F16, bool BOX, int UC>
static hipError_t launch_train_u(const Params &p, int threads, size_t lds, hipStream_t s)
{
    auto fn = k_train<L, NPL, F16, BOX, UC>;
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
static hipError_t launch_train_t(const Params &p, int threads, size_t lds, hipStream_t s)
{
    if constexpr (NPL <= 8) {
        if (p.U == 8) return launch_train_u<L, NPL, F16, BOX, 8>(p, threads, lds, s);
        if (p.U == 16) return launch_train_u<L, NPL, F16, BOX, 16>(p, threads, lds, s);
    }
    return launch_train_u<L, NPL, F16, BOX, 0>(p, threads, lds, s);
}

template <int L, int NPL>
static hipError_t launch_train_ln(bool f16, const Params &p, int threads, size_t lds,
                                  hipStream_t s)
{
    if (f16) return p.box ? launch_train_t<L, NPL, true, true>(p, threads, lds, s)
                          : launch_train_t<L, NPL, true, false>(p, threads, lds, s);
    return p.box ? launch_train_t<L, NPL, false, true>(p, threads, lds, s)
                 : launch_train_t<L, NPL, false, false>(p, threads, lds, s);
}

template <int L>
static hipError_t launch_train_l(int NPL, bool f16, const Params &p, int threads, size_t lds,
                                 hipStream_t s)
{
    switch (NPL) {
    case 2: return launch_train_ln<L, 2>(f16, p, threads, lds, s);
    case 4: return launch_train_ln<L, 4>(f16, p, threads, lds, s);
    case 8: return launch_train_ln<L, 8>(f16, p, threads, lds, s);
    case 16: return launch_train_ln<L, 16>(f16, p, threads, lds, s);
    case 32: return launch_train_ln<L, 32>(f16, p, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_train(int L, int NPL, bool f16, const Params &p, int threads, size_t lds,
                        hipStream_t s)
{
    switch (L) {
    case 4: return launch_train_l<4>(NPL, f16, p, threads, lds, s);
    case 8: return launch_train_l<8>(NPL, f16, p, threads, lds, s);
    case 16: return launch_train_l<16>(NPL, f16, p, threads, lds, s);
    case 32: return launch_train_l<32>(NPL, f16, p, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ocd
