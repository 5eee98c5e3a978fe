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

template <int HALF>
__device__ __forceinline__ void user_llr(float xr, float xi, float scale, float rho, float *out)
{
    axis_llr<HALF>(xr, scale, rho, out);         // in-phase bits
    axis_llr<HALF>(xi, scale, rho, out + HALF);  // quadrature bits
}

// Algorithm 1 and the soft output for the vectors of one tile.  The caller has
// carved LDS; this function stages H_w and returns after writing z, z_hist and
// the LLRs.  Every thread of the workgroup must call it (it contains barriers);
// threads of idle lane groups may return before the others finish, so a caller
// that reuses the LDS for another tile must synchronise first.
template <int L, int NPL, bool F16, bool BOX>
__device__ void forward_tile(const Params &P, const Smem &sm, const Tile &tile)
{
    const int U = P.U, Bpad = P.Bpad;
    const int Kt = P.per_sweep ? P.K : 1;

    const int grp = threadIdx.x / L, j = threadIdx.x % L;
    const bool active = grp < tile.nvb;
    const int v = tile.vbase + (active ? grp : 0);
    const int slot = v / P.S - tile.w_first;

    // H_w chunk loads first, then the receive vector (initialisation r = y):
    // both global round trips are in flight together, and the LDS stores of H
    // wait only for the H chunks.
    const int chunks = tile.nslots * U * (Bpad >> 1);
    float4 hbuf[STAGE_CHUNKS];
    stage_h_load<F16>(P, tile.w_first, chunks, 0, hbuf);
    float2 r[NPL];
    load_vector<L, NPL, F16>(P, P.y, v, j, active, r);
    stage_h_store(P, sm, chunks, 0, hbuf);
    stage_h_copy<F16>(P, sm, tile.w_first, chunks, STAGE_CHUNKS * (int)blockDim.x);
    stage_preprocess(P, sm, tile.w_first, tile.nslots);
    clear_padding<L, NPL>(P, j, active, r);

    const float2 *Hs = sm.H + (size_t)slot * P.slot_stride;
    const float2 *dps = sm.dp + (size_t)slot * Kt * U;
    float2 *zv = sm.z + (size_t)zrow_of(P, grp) * U;
    for (int u = 0; u < U; ++u) zv[u] = make_float2(0.f, 0.f);   // z^(0) = 0

    // K sweeps over the users in order (Alg. 1); with several waves per SIMD
    // the LDS latency of each update is hidden by the other waves.
    const float beta = P.beta;
    for (int k = 0; k < P.K; ++k) {
        const float2 *dpk = dps + (P.per_sweep ? k : 0) * U;
        for (int u = 0; u < U; ++u) {
            float2 h[NPL];
            load_column<L, NPL>(Hs + (size_t)u * Bpad, j, h);
            const float2 dp = dpk[u];
            const float2 zo = zv[u];
            zv[u] = coordinate_update<L, NPL, BOX>(h, dp, zo, beta, r);
        }
        if (P.z_hist && active)
            for (int u = j; u < U; u += L) P.z_hist[((long)v * P.K + k) * U + u] = zv[u];
    }

    if (!active) return;
    const float lamK = P.lambda ? P.lambda[P.K - 1] : P.lam_default;
    const float2 *dpK = dps + (P.per_sweep ? P.K - 1 : 0) * U;
    const float sqEs = sqrtf(P.Es), scale = qam_scale(P.Q);
    for (int u = j; u < U; u += L) {
        const float2 zu = zv[u];
        if (P.z) P.z[(long)v * U + u] = zu;
        if (!P.llr) continue;
        float mu, rho;
        gain_sinr(P, lamK, sm.g[slot * U + u], dpK[u].y, &mu, &rho);
        float out[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (rho > 0.f && mu > 0.f) {
            const float s = 1.0f / (mu * sqEs);
            const float xr = zu.x * s, xi = zu.y * s;
            if (P.Q == 2) user_llr<1>(xr, xi, scale, rho, out);
            else if (P.Q == 4) user_llr<2>(xr, xi, scale, rho, out);
            else user_llr<3>(xr, xi, scale, rho, out);
        }
        float *dst = P.llr + ((long)v * U + u) * P.Q;
        for (int b = 0; b < P.Q; ++b) dst[b] = out[b];
    }
}

}  // namespace ocd
