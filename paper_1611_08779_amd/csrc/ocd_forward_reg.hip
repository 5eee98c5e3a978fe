// ocd_forward_reg.hip -- Algorithm 1 plus the soft output with every vector's
// channel columns held in the registers of its lane group: no LDS and no
// workgroup barrier.
//
// When few OFDM symbols share a channel matrix (S small) staging H_w in LDS buys
// no reuse, and the kernel is bound by streaming H and y from HBM.  Here each
// group issues the loads of its receive vector and then of its columns in the
// order the first sweep consumes them, and does the preprocessing of user u just
// before that user's first update, so the early updates of the first sweep
// overlap the round trip of the later columns.  The user count has a compile-time
// bound UC (U <= UC = 8); z, d^-1, p and g live in registers as well.
#include "ocd_stage.h"

namespace ocd {

// a[idx] for a register array with a compile-time bound, without dynamic
// register indexing: one conditional move per entry.
template <int N, typename T>
__device__ __forceinline__ T pick(const T (&a)[N], int idx)
{
    T out = a[0];
#pragma unroll
    for (int i = 1; i < N; ++i) out = idx == i ? a[i] : out;
    return out;
}

template <int L, int NPL, int UC, bool F16, bool BOX>
__global__ __launch_bounds__(256) void k_forward_reg(Params P)
{
    const int U = P.U, B = P.B;
    const int grp = threadIdx.x / L, j = threadIdx.x % L;
    Tile tile;
    tile.vbase = (int)blockIdx.x * P.vpb;
    tile.nvb = min(P.vpb, P.W * P.S - tile.vbase);
    tile.w_first = tile.vbase / P.S;
    tile.nslots = 0;   // unused: nothing is staged
    const bool active = grp < tile.nvb;
    const int g0 = active ? grp : 0;
    const int v = tile.vbase + g0;
    const int w = tile.w_first + slot_of_group(P, tile, g0);   // this vector's subcarrier

    // initialisation r = y, then the columns of H_w in the order sweep 1 reads them.
    // All UC column loads are issued unconditionally (columns past U re-read column
    // U-1, valid memory that is never used), so that no branch separates them from
    // the updates and each update of sweep 1 waits only for its own column.  The
    // host launches this kernel only with 16-byte aligned FP32 (8-byte FP16) rows
    // of even length and with the preprocessing fused.
    float2 r[NPL];
    {
        const unsigned char *yb =
            static_cast<const unsigned char *>(P.y) + (size_t)tile.vbase * B * cbytes<F16>();
#pragma unroll
        for (int c = 0; c < NPL / 2; ++c) {
            const int b = 2 * (j + L * c);
            const bool ok = active && b < B;
            const float4 q = load_pair_at<F16>(yb, ok ? (unsigned)(grp * B + b) * cbytes<F16>() : 0u);
            r[2 * c] = make_float2(q.x, q.y);
            r[2 * c + 1] = make_float2(q.z, q.w);
        }
    }
    float2 h[UC][NPL];
    {
        const unsigned char *hb =
            static_cast<const unsigned char *>(P.H) + (size_t)tile.w_first * U * B * cbytes<F16>();
        const int wrow = (w - tile.w_first) * U;
#pragma unroll
        for (int u = 0; u < UC; ++u) {
            const int cu = u < U ? u : U - 1;
#pragma unroll
            for (int c = 0; c < NPL / 2; ++c) {
                const int b = 2 * (j + L * c);
                const bool ok = active && b < B;
                const float4 q =
                    load_pair_at<F16>(hb, ok ? (unsigned)((wrow + cu) * B + b) * cbytes<F16>() : 0u);
                h[u][2 * c] = make_float2(q.x, q.y);
                h[u][2 * c + 1] = make_float2(q.z, q.w);
            }
        }
    }
    if (B != P.Bpad) {
#pragma unroll
        for (int c = 0; c < NPL / 2; ++c) {
            const bool ok = 2 * (j + L * c) < B;
            r[2 * c] = ok ? r[2 * c] : make_float2(0.f, 0.f);
            r[2 * c + 1] = ok ? r[2 * c + 1] : make_float2(0.f, 0.f);
        }
        // antennas past B were loaded from a placeholder address
#pragma unroll
        for (int u = 0; u < UC; ++u)
#pragma unroll
            for (int c = 0; c < NPL / 2; ++c) {
                const bool ok = 2 * (j + L * c) < B;
                h[u][2 * c] = ok ? h[u][2 * c] : make_float2(0.f, 0.f);
                h[u][2 * c + 1] = ok ? h[u][2 * c + 1] : make_float2(0.f, 0.f);
            }
    }

    // Algorithm 1's preprocessing (g_u, d_u^-1, p_u) for sweep k, user u
    float gv[UC], dv[UC], pv[UC];
    auto coefs = [&](int k, int u) {
        if (k == 0) {
            float acc = 0.f;
#pragma unroll
            for (int i = 0; i < NPL; ++i) acc = fmaf(h[u][i].x, h[u][i].x, fmaf(h[u][i].y, h[u][i].y, acc));
            gv[u] = group_sum<L>(acc);
        }
        const float lam = P.lambda ? P.lambda[k] : P.lam_default;
        const float den = gv[u] + lam;
        const float di = den > 0.f ? 1.0f / den : 0.f;
        dv[u] = di;
        pv[u] = di * gv[u];
    };

    float2 z[UC];
#pragma unroll
    for (int u = 0; u < UC; ++u) z[u] = make_float2(0.f, 0.f);   // z^(0) = 0
    const float beta = P.beta;
    auto sweep_done = [&](int k) {
        if (P.z_hist && active)
            for (int u = j; u < U; u += L)
                P.z_hist[((long)v * P.K + k) * U + u] = pick(z, u);
    };

    // sweep 1: user u's preprocessing right before its first update
#pragma unroll
    for (int u = 0; u < UC; ++u) {
        if (u < U) {
            coefs(0, u);
            z[u] = coordinate_update<L, NPL, BOX, 2>(h[u], make_float2(dv[u], pv[u]), z[u], beta, r);
        }
    }
    sweep_done(0);
    for (int k = 1; k < P.K; ++k) {
        if (P.per_sweep) {
#pragma unroll
            for (int u = 0; u < UC; ++u)
                if (u < U) coefs(k, u);
        }
#pragma unroll
        for (int u = 0; u < UC; ++u)
            if (u < U)
                z[u] = coordinate_update<L, NPL, BOX, 2>(h[u], make_float2(dv[u], pv[u]), z[u], beta, r);
        sweep_done(k);
    }

    if (!active) return;
    if (P.z) {
        float2 *zt = P.z + (size_t)tile.vbase * U;
        for (int u = j; u < U; u += L) zt[grp * U + u] = pick(z, u);
    }
    if (P.llr) {
        const int Q = P.Q, half = Q >> 1;
        const float lamK = P.lambda ? P.lambda[P.K - 1] : P.lam_default;
        float *lt = P.llr + (size_t)tile.vbase * U * Q;
        for (int idx = j; idx < 2 * U; idx += L) {
            const int u = idx >> 1, ax = idx & 1;
            const float2 co = llr_coef(P, pick(gv, u), pick(pv, u), lamK);
            const float2 zu = pick(z, u);
            const float t = (ax ? zu.y : zu.x) * co.x;
            float *dst = lt + (grp * U + u) * Q + ax * half;
            if (half == 3) axis_llrs<3>(t, co.y, dst);
            else if (half == 2) axis_llrs<2>(t, co.y, dst);
            else axis_llrs<1>(t, co.y, dst);
        }
    }
}

template <int L, int NPL, int UC>
static hipError_t launch_reg_t(bool f16, const Params &p, int threads, hipStream_t s)
{
    const dim3 grid(p.nblocks), block(threads);
    if (f16) {
        if (p.box) hipLaunchKernelGGL((k_forward_reg<L, NPL, UC, true, true>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_forward_reg<L, NPL, UC, true, false>), grid, block, 0, s, p);
    } else {
        if (p.box) hipLaunchKernelGGL((k_forward_reg<L, NPL, UC, false, true>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_forward_reg<L, NPL, UC, false, false>), grid, block, 0, s, p);
    }
    return hipGetLastError();
}

template <int L>
static hipError_t launch_reg_l(int NPL, int UC, bool f16, const Params &p, int threads,
                               hipStream_t s)
{
    if (UC != 8) return hipErrorInvalidValue;
    switch (NPL) {
    case 2: return launch_reg_t<L, 2, 8>(f16, p, threads, s);
    case 4: return launch_reg_t<L, 4, 8>(f16, p, threads, s);
    case 8: return launch_reg_t<L, 8, 8>(f16, p, threads, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward_reg(int L, int NPL, int UC, bool f16, const Params &p, int threads,
                              hipStream_t s)
{
    switch (L) {
    case 16: return launch_reg_l<16>(NPL, UC, f16, p, threads, s);
    case 32: return launch_reg_l<32>(NPL, UC, f16, p, threads, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ocd
