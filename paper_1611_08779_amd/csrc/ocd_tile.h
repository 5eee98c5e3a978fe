// ocd_tile.h -- Algorithm 1 (OCD) plus the approximate max-log soft output for
// the vectors of one tile; shared by the one-problem kernel and the persistent
// batched kernel.
//
// Mapping: a workgroup owns a tile of consecutive (subcarrier, symbol) vectors;
// the H_w of every subcarrier they touch is staged once into LDS (FP32) and read
// by all K*U coordinate updates of all of its vectors, so H is read from HBM
// once per tile.  A vector is owned by L lanes; its residual r lives in their
// registers for the whole of Algorithm 1, z in LDS.  One coordinate update
// (Alg. 1, the three equalisation lines) is: NPL complex MACs per lane for
// h_u^H r, an all-reduce over the L lanes in DPP, a few scalar ops for the new
// z_u and its change, and NPL complex MACs per lane for r <- r - h_u Delta.
#pragma once

#include "ocd_stage.h"

namespace ocd {

// Algorithm 1 and the soft output for the vectors of one tile.  The caller has
// carved LDS; this function stages H_w and returns after writing z, z_hist and
// the LLRs.  Every thread of the workgroup must call it (it contains barriers);
// threads of idle lane groups may return before the others finish, so a caller
// that reuses the LDS for another tile must synchronise first.
//
// UC > 0: U == UC and the user loop is unrolled: z stays in registers, every
// LDS address of a coordinate update is a compile-time offset from one base (the
// rows of H_w are L * NPL apart) and the straight-line sweep lets the compiler
// read the next column while the current update computes; UC = 0: U is a
// run-time bound.
// PIPE: with a run-time U, read the next update's operands while the current
// one computes (a second operand buffer); off where registers are scarce.
// PREFETCH (UC > 0): read the next update's column one update ahead, into a
// second register buffer: the launches with few waves per SIMD have nothing else
// to hide the LDS latency behind, and the registers to spare (same arithmetic).
// CHUNKED (UC > 0): U is a multiple of UC and the sweep runs as U / UC unrolled
// chunks of UC users with z in LDS (one more LDS read and write per update, no
// registers per user): the straight-line chunk keeps the compile-time LDS offsets
// and the early column reads of the unrolled loop for any such U.
template <int L, int NPL, bool F16, bool BOX, int UC = 0, bool PIPE = true, bool PREFETCH = false,
          bool CHUNKED = false>
__device__ void forward_tile(const Params &P, const Smem &sm, const Tile &tile)
{
    const int U = P.U, Bpad = P.Bpad;
    const int Kt = P.per_sweep ? P.K : 1;

    const int grp = threadIdx.x / L, j = threadIdx.x % L;
    const bool active = grp < tile.nvb;
    const int v = tile.vbase + (active ? grp : 0);
    const int slot = slot_of_group(P, tile, active ? grp : 0);

    // H_w chunk loads first, then the receive vector (initialisation r = y):
    // both global round trips are in flight together, and the LDS stores of H
    // wait only for the H chunks.
    const int chunks = tile.nslots * U * (Bpad >> 1);
    float4 hbuf[STAGE_CHUNKS];
    stage_h_load<F16>(P, tile.w_first, tile.nslots, chunks, 0, hbuf);
    float2 r[NPL];
    load_vector<L, NPL, F16>(P, P.y, tile, grp, j, active, r);
    stage_h_store(P, sm, tile.nslots, chunks, 0, hbuf);
    stage_h_copy<F16>(P, sm, tile.w_first, tile.nslots, chunks, STAGE_CHUNKS * (int)blockDim.x);
    stage_preprocess<L * NPL>(P, sm, tile.w_first, tile.nslots);
    clear_padding<L, NPL>(P, j, active, r);

    const float2 *Hs = sm.H + (size_t)slot * P.slot_stride;
    const float2 *dps = sm.dp + (size_t)slot * Kt * U;
    float2 *zv = sm.z + (size_t)zrow_of(P, grp) * U;
    for (int u = 0; u < U; ++u) zv[u] = make_float2(0.f, 0.f);   // z^(0) = 0

    // K sweeps over the users in order (Alg. 1).
    const float beta = P.beta;
    auto sweep_done = [&](int k) {
        if (P.z_hist && active)
            for (int u = j; u < U; u += L) global_store2(P.z_hist + ((long)v * P.K + k) * U + u, zv[u]);
    };
    if constexpr (UC > 0 && CHUNKED) {
        constexpr int BP = L * NPL;
        for (int k = 0; k < P.K; ++k) {
            const float2 *dpk = dps + (P.per_sweep ? k : 0) * U;
            const bool last_sweep = k == P.K - 1;
            for (int c = 0; c < U; c += UC) {
                const float2 *Hc = Hs + (size_t)c * BP;
                const float2 *dpc = dpk + c;
                float2 *zc = zv + c;
                const bool last_chunk = last_sweep && c + UC == U;
#pragma unroll
                for (int u = 0; u < UC; ++u) {
                    float2 h[NPL];
                    load_column<L, NPL>(Hc + u * BP, j, h);
                    if (u == UC - 1 && last_chunk)   // r is not read after the last update
                        zc[u] = coordinate_update<L, NPL, BOX, 1, false>(h, dpc[u], zc[u], beta, r);
                    else
                        zc[u] = coordinate_update<L, NPL, BOX>(h, dpc[u], zc[u], beta, r);
                }
            }
            sweep_done(k);
        }
    } else if constexpr (UC > 0) {
        constexpr int BP = L * NPL;
        float2 zr[UC];
#pragma unroll
        for (int u = 0; u < UC; ++u) zr[u] = make_float2(0.f, 0.f);
        float2 hn[NPL];   // PREFETCH: the next update's column
        if constexpr (PREFETCH) load_column<L, NPL>(Hs, j, hn);
        for (int k = 0; k < P.K; ++k) {
            const float2 *dpk = dps + (P.per_sweep ? k : 0) * U;
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                float2 h[NPL];
                if constexpr (PREFETCH) {
#pragma unroll
                    for (int i = 0; i < NPL; ++i) h[i] = hn[i];
                    load_column<L, NPL>(Hs + ((u + 1) % UC) * BP, j, hn);
                } else {
                    load_column<L, NPL>(Hs + u * BP, j, h);
                }
                if (u == UC - 1 && k == P.K - 1)   // r is not read after the last update
                    zr[u] = coordinate_update<L, NPL, BOX, 1, false>(h, dpk[u], zr[u], beta, r);
                else
                    zr[u] = coordinate_update<L, NPL, BOX>(h, dpk[u], zr[u], beta, r);
            }
            if (P.z_hist) {
#pragma unroll
                for (int u = 0; u < UC; ++u) zv[u] = zr[u];
                sweep_done(k);
            }
        }
#pragma unroll
        for (int u = 0; u < UC; ++u) zv[u] = zr[u];   // for the outputs below
    } else if (!PIPE || U == 1 || NPL > 8) {
        // a single user: every update reads the z it wrote the step before; with
        // more than 8 entries per lane a second operand buffer would cost more
        // occupancy than it hides latency
        for (int k = 0; k < P.K; ++k) {
            for (int u = 0; u < U; ++u) {
                UpdateOperands<NPL> a;
                fetch_operands<L, NPL>(Hs, Bpad, dps + (P.per_sweep ? k : 0) * U, zv, u, j, a);
                zv[u] = coordinate_update<L, NPL, BOX>(a.h, a.dp, a.zo, beta, r);
            }
            sweep_done(k);
        }
    } else {
        // The K*U updates as one sequence, two operand buffers: the LDS reads of
        // the next update are in flight while the current one computes.  With
        // U >= 2 the next update never reads the z_u the current one writes.
        UpdateOperands<NPL> a, b;
        int k = 0, u = 0;
        fetch_operands<L, NPL>(Hs, Bpad, dps, zv, 0, j, a);
        for (;;) {
            int kn = k, un = u + 1;
            if (un == U) { un = 0; ++kn; }
            if (kn < P.K)
                fetch_operands<L, NPL>(Hs, Bpad, dps + (P.per_sweep ? kn : 0) * U, zv, un, j, b);
            zv[u] = coordinate_update<L, NPL, BOX>(a.h, a.dp, a.zo, beta, r);
            if (un == 0) sweep_done(k);
            if (kn == P.K) break;
            k = kn;
            u = un;
            kn = k;
            un = u + 1;
            if (un == U) { un = 0; ++kn; }
            if (kn < P.K)
                fetch_operands<L, NPL>(Hs, Bpad, dps + (P.per_sweep ? kn : 0) * U, zv, un, j, a);
            zv[u] = coordinate_update<L, NPL, BOX>(b.h, b.dp, b.zo, beta, r);
            if (un == 0) sweep_done(k);
            if (kn == P.K) break;
            k = kn;
            u = un;
        }
    }

    if (!active) return;
    // outputs: lanes of the group take users (z) and (user, axis) pairs (LLRs)
    if (P.z) {
        float2 *zt = P.z + (size_t)tile.vbase * U;   // workgroup-uniform base
        for (int u = j; u < U; u += L) global_store2(zt + grp * U + u, zv[u]);
    }
    if (P.llr) {
        const int Q = P.Q, half = Q >> 1;
        const auto lt = global_ptr(P.llr + (size_t)tile.vbase * U * Q);
        const float2 *lcs = sm.lc + (size_t)slot * U;
        for (int idx = j; idx < 2 * U; idx += L) {
            const int u = idx >> 1, ax = idx & 1;
            const float2 zu = zv[u], co = lcs[u];
            const float t = (ax ? zu.y : zu.x) * co.x;
            const auto dst = lt + (grp * U + u) * Q + ax * half;
            if (half == 3) axis_llrs<3>(t, co.y, dst);
            else if (half == 2) axis_llrs<2>(t, co.y, dst);
            else axis_llrs<1>(t, co.y, dst);
        }
    }
}

}  // namespace ocd
