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
// bound UC (U <= UC = 8); z, d^-1, p and g live in registers as well.  With every
// workgroup resident at once, all of them would wait for their loads together and
// then compute together; the plan's stagger delays later workgroups
// (stagger_loads) so that earlier ones compute while later ones load.
#include <type_traits>

#include "ocd_stage.h"

namespace ocd {

// One vector's operands in a lane group's registers: the lane's share of the UC
// channel columns (float2, or packed half pairs for FP16 storage) and of r.
template <int NPL, int UC, bool F16>
struct RegVec {
    using HT = typename std::conditional<F16, uint32_t, float2>::type;
    HT h[UC][NPL];
    float2 r[NPL];
};

// Issues the loads of vector vb + grp (vb: a workgroup-uniform vector index):
// first the receive vector (r = y), then the columns in the order sweep 1 reads
// them.  All UC column loads are unconditional (columns past U re-read column
// U-1, valid memory that is never used) and inactive groups read the uniform
// base, so no branch separates the loads from their uses and each update of the
// first sweep waits only for its own column.  The host launches these kernels
// only with 16-byte aligned FP32 (8-byte FP16) rows of even length.
template <int L, int NPL, int UC, bool F16>
__device__ __forceinline__ void reg_load(const Params &P, int vb, int grp, int j, bool active,
                                         RegVec<NPL, UC, F16> &x)
{
    const int U = P.U, B = P.B;
    const unsigned char *yb =
        static_cast<const unsigned char *>(P.y) + (size_t)vb * B * cbytes<F16>();
#pragma unroll
    for (int c = 0; c < NPL / 2; ++c) {
        const int b = 2 * (j + L * c);
        const bool ok = active && b < B;
        const float4 q = load_pair_at<F16>(yb, ok ? (unsigned)(grp * B + b) * cbytes<F16>() : 0u);
        x.r[2 * c] = make_float2(q.x, q.y);
        x.r[2 * c + 1] = make_float2(q.z, q.w);
    }
    // subcarriers of vb and of this group's vector
    const int wb = (int)divide_invariant((unsigned)vb, P.divS_m, P.divS_s1, P.divS_s2);
    const int w = (int)divide_invariant((unsigned)(vb + (active ? grp : 0)), P.divS_m, P.divS_s1,
                                        P.divS_s2);
    const unsigned char *hb =
        static_cast<const unsigned char *>(P.H) + (size_t)wb * U * B * cbytes<F16>();
    const int wrow = (w - wb) * U;
#pragma unroll
    for (int u = 0; u < UC; ++u) {
        const int cu = u < U ? u : U - 1;
#pragma unroll
        for (int c = 0; c < NPL / 2; ++c) {
            const int b = 2 * (j + L * c);
            const bool ok = active && b < B;
            const unsigned off = ok ? (unsigned)((wrow + cu) * B + b) * cbytes<F16>() : 0u;
            if constexpr (F16) {
                const u32x2_t q = load_pair_raw16(hb, off);
                x.h[u][2 * c] = q.x;
                x.h[u][2 * c + 1] = q.y;
            } else {
                const float4 q = load_pair_at<F16>(hb, off);
                x.h[u][2 * c] = make_float2(q.x, q.y);
                x.h[u][2 * c + 1] = make_float2(q.z, q.w);
            }
        }
    }
}

// Algorithm 1 and the soft output of vector vb + grp from its registers, then its
// outputs.  User u's preprocessing (g_u, d_u^-1, p_u) happens right before its
// first update.  z, d^-1, p and g live in registers.
// Per-group LDS row through which lanes exchange the per-user values (z, g, p):
// every lane of the group holds all of them; the lane that stores user u reads
// them back by a run-time index.  (Register arrays indexed at run time would go
// to scratch memory, whose accesses share the wait counter of the channel
// prefetch.)  Groups never span waves, so the wave's own LDS order suffices.
template <int UC>
struct UserRow {
    float4 e[UC];   // (Re z_u, Im z_u, g_u, p_u)
};

template <int L, int NPL, int UC, bool F16, bool BOX>
__device__ __forceinline__ void reg_compute(const Params &P, int vb, int grp, int j, bool active,
                                            RegVec<NPL, UC, F16> &x, UserRow<UC> &row)
{
    using HT = typename RegVec<NPL, UC, F16>::HT;
    const int U = P.U, B = P.B;
    const int v = vb + (active ? grp : 0);
    if (B != P.Bpad) {
        // antennas past B were loaded from a placeholder address
#pragma unroll
        for (int c = 0; c < NPL / 2; ++c) {
            const bool ok = 2 * (j + L * c) < B;
            x.r[2 * c] = ok ? x.r[2 * c] : make_float2(0.f, 0.f);
            x.r[2 * c + 1] = ok ? x.r[2 * c + 1] : make_float2(0.f, 0.f);
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                x.h[u][2 * c] = ok ? x.h[u][2 * c] : HT{};
                x.h[u][2 * c + 1] = ok ? x.h[u][2 * c + 1] : HT{};
            }
        }
    }

    float gv[UC], dv[UC], pv[UC];
    auto coefs = [&](int k, int u) {
        if (k == 0) {
            float acc = 0.f;
#pragma unroll
            for (int i = 0; i < NPL; ++i)
                acc = fmaf(hre(x.h[u][i]), hre(x.h[u][i]), fmaf(him(x.h[u][i]), him(x.h[u][i]), acc));
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
    auto publish = [&]() {
#pragma unroll
        for (int u = 0; u < UC; ++u) row.e[u] = make_float4(z[u].x, z[u].y, gv[u], pv[u]);
        __builtin_amdgcn_wave_barrier();
    };
    auto sweep_done = [&](int k) {
        if (!P.z_hist) return;
        publish();
        if (active)
            for (int u = j; u < U; u += L) {
                const float4 e = row.e[u];
                P.z_hist[((long)v * P.K + k) * U + u] = make_float2(e.x, e.y);
            }
        __builtin_amdgcn_wave_barrier();
    };

#pragma unroll
    for (int u = 0; u < UC; ++u) {
        if (u < U) {
            coefs(0, u);
            z[u] = coordinate_update<L, NPL, BOX, 2>(x.h[u], make_float2(dv[u], pv[u]), z[u], beta,
                                                     x.r);
        }
    }
    sweep_done(0);
    for (int k = 1; k < P.K; ++k) {
        if constexpr (F16) {
            // keep the channel packed: without this the compiler hoists one FP32 copy
            // of every entry out of the sweep loop (twice the registers) instead of
            // feeding the half operands to the FMAs
#pragma unroll
            for (int u = 0; u < UC; ++u)
#pragma unroll
                for (int i = 0; i < NPL; ++i) asm volatile("" : "+v"(x.h[u][i]));
        }
        if (P.per_sweep) {
#pragma unroll
            for (int u = 0; u < UC; ++u)
                if (u < U) coefs(k, u);
        }
#pragma unroll
        for (int u = 0; u < UC; ++u)
            if (u < U)
                z[u] = coordinate_update<L, NPL, BOX, 2>(x.h[u], make_float2(dv[u], pv[u]), z[u],
                                                         beta, x.r);
        sweep_done(k);
    }

    publish();
    if (active) {
        if (P.z) {
            float2 *zt = P.z + (size_t)vb * U;
            for (int u = j; u < U; u += L) {
                const float4 e = row.e[u];
                zt[grp * U + u] = make_float2(e.x, e.y);
            }
        }
        if (P.llr) {
            const int Q = P.Q, half = Q >> 1;
            const float lamK = P.lambda ? P.lambda[P.K - 1] : P.lam_default;
            float *lt = P.llr + (size_t)vb * U * Q;
            for (int idx = j; idx < 2 * U; idx += L) {
                const int u = idx >> 1, ax = idx & 1;
                const float4 e = row.e[u];
                const float2 co = llr_coef(P, e.z, e.w, lamK);
                const float t = (ax ? e.y : e.x) * co.x;
                float *dst = lt + (grp * U + u) * Q + ax * half;
                if (half == 3) axis_llrs<3>(t, co.y, dst);
                else if (half == 2) axis_llrs<2>(t, co.y, dst);
                else axis_llrs<1>(t, co.y, dst);
            }
        }
    }
}

// One vector per lane group.
template <int L, int NPL, int UC, bool F16, bool BOX>
__global__ __launch_bounds__(256) void k_forward_reg(Params P)
{
    const int grp = threadIdx.x / L, j = threadIdx.x % L;
    const int vb = (int)blockIdx.x * P.vpb;
    const bool active = grp < min(P.vpb, P.W * P.S - vb);
    __shared__ UserRow<UC> rows[256 / L];
    stagger_loads(P);
    RegVec<NPL, UC, F16> x;
    reg_load<L, NPL, UC>(P, vb, grp, j, active, x);
    reg_compute<L, NPL, UC, F16, BOX>(P, vb, grp, j, active, x, rows[grp]);
}

template <int L, int NPL, int UC, bool F16, bool BOX>
static hipError_t launch_reg_k(const Params &p, int threads, hipStream_t s)
{
    auto fn = k_forward_reg<L, NPL, UC, F16, BOX>;
    Params q = p;
    if (q.stagger > 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(fn), threads, 0);
        if (e != hipSuccess) return e;
        q.stagger_cap = per_cu * device_cu_count();
    }
    hipLaunchKernelGGL(fn, dim3(q.nblocks), dim3(threads), 0, s, q);
    return hipGetLastError();
}

template <int L, int NPL, int UC>
static hipError_t launch_reg_t(bool f16, const Params &p, int threads, hipStream_t s)
{
    if (f16) return p.box ? launch_reg_k<L, NPL, UC, true, true>(p, threads, s)
                          : launch_reg_k<L, NPL, UC, true, false>(p, threads, s);
    return p.box ? launch_reg_k<L, NPL, UC, false, true>(p, threads, s)
                 : launch_reg_k<L, NPL, UC, false, false>(p, threads, s);
}

template <int L>
static hipError_t launch_reg_l(int NPL, int UC, bool f16, const Params &p, int threads, hipStream_t s)
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
