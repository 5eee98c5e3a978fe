// ocd_stage.h -- per-workgroup staging shared by the forward and adjoint kernels:
// LDS carving, the copy of H_w into LDS and Algorithm 1's preprocessing.
#pragma once

#include "ocd_device.h"
#include "ocd_internal.h"

namespace ocd {

struct Smem {
    float2 *H;     // [maxslots][slot_stride]: H_w columns, FP32, zero-padded to Bpad
    float *g;      // [maxslots][U]: ||h_u||^2
    float2 *dp;    // [maxslots][Kt][U]: (d_u^-1, p_u)
    float2 *z;     // [vpb_cap][U]: current z of each vector
    float2 *zprev; // [vpb_cap][U]: adjoint only, z^(k-1) of the sweep being reversed
    float2 *zbar;  // [vpb_cap][U]: adjoint only, dLoss/dz
    float *part;   // [vpb_cap][2]: adjoint only, per-group partial sums
};

__device__ __forceinline__ Smem carve(unsigned char *smem, const Params &P, int vpb_cap,
                                      bool backward)
{
    const int Kt = P.per_sweep ? P.K : 1;
    Smem s;
    size_t off = 0;
    s.H = reinterpret_cast<float2 *>(smem);
    off += (size_t)P.maxslots * P.slot_stride * 8;
    s.g = reinterpret_cast<float *>(smem + off);
    off += (size_t)P.maxslots * P.U * 4;
    off = (off + 7) & ~(size_t)7;
    s.dp = reinterpret_cast<float2 *>(smem + off);
    off += (size_t)P.maxslots * Kt * P.U * 8;
    s.z = reinterpret_cast<float2 *>(smem + off);
    off += (size_t)vpb_cap * P.U * 8;
    s.zprev = s.zbar = nullptr;
    s.part = nullptr;
    if (backward) {
        s.zprev = reinterpret_cast<float2 *>(smem + off);
        off += (size_t)vpb_cap * P.U * 8;
        s.zbar = reinterpret_cast<float2 *>(smem + off);
        off += (size_t)vpb_cap * P.U * 8;
        s.part = reinterpret_cast<float *>(smem + off);
    }
    return s;
}

// The vectors of one workgroup: [vbase, vbase + nvb) in (subcarrier, symbol)
// order; they touch subcarriers w_first .. w_first + nslots - 1.
struct Tile {
    long vbase;
    int nvb, w_first, nslots;
};

__device__ __forceinline__ Tile tile_of(const Params &P, int bid)
{
    Tile t;
    const long nvec = (long)P.W * P.S;
    t.vbase = (long)bid * P.vpb;
    long rem = nvec - t.vbase;
    t.nvb = (int)(rem < P.vpb ? rem : P.vpb);
    t.w_first = (int)(t.vbase / P.S);
    t.nslots = (int)((t.vbase + t.nvb - 1) / P.S) - t.w_first + 1;
    return t;
}

// Copies H_w of every touched subcarrier into LDS (FP32, zero padded to Bpad)
// and computes Algorithm 1's preprocessing once per subcarrier:
// g_u = ||h_u||^2, d_u^-1 = (g_u + lambda_k)^-1 (0 if that is 1/0), p_u = d_u^-1 g_u.
// Ends with a workgroup barrier.
template <bool F16>
__device__ void stage_subcarriers(const Params &P, const Smem &sm, int w_first, int nslots)
{
    const int U = P.U, B = P.B, Bpad = P.Bpad;
    const int Kt = P.per_sweep ? P.K : 1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
    const int rows = nslots * U;
    for (int row = wave; row < rows; row += nwaves) {
        const int slot = row / U, u = row - slot * U;
        const long e0 = ((long)(w_first + slot) * U + u) * B;
        float2 *dst = sm.H + (size_t)slot * P.slot_stride + (size_t)u * Bpad;
        for (int b = 2 * lane; b < Bpad; b += 128) {
            float2 v[2];
            load_chunk<F16, 2>(P.H, e0 + b, b, B, P.vec_ok != 0, v);
            *reinterpret_cast<float4 *>(dst + b) = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
        }
    }
    if (P.g_in) {
        for (int i = threadIdx.x; i < rows; i += blockDim.x)
            sm.g[i] = P.g_in[(long)w_first * U + i];
        for (int i = threadIdx.x; i < nslots * Kt * U; i += blockDim.x) {
            const long gi = (long)w_first * Kt * U + i;
            sm.dp[i] = make_float2(P.dinv_in[gi], P.p_in[gi]);
        }
        __syncthreads();
        return;
    }
    __syncthreads();
    for (int row = wave; row < rows; row += nwaves) {
        const int slot = row / U, u = row - slot * U;
        const float2 *h = sm.H + (size_t)slot * P.slot_stride + (size_t)u * Bpad;
        float acc = 0.f;
        for (int b = lane; b < Bpad; b += 64) acc = fmaf(h[b].x, h[b].x, fmaf(h[b].y, h[b].y, acc));
        acc = wave_sum(acc);
        if (lane == 0) sm.g[row] = acc;
        for (int kt = lane; kt < Kt; kt += 64) {
            const float lam = P.lambda ? P.lambda[kt] : P.lam_default;
            const float den = acc + lam;
            const float di = den > 0.f ? 1.0f / den : 0.f;
            sm.dp[((size_t)slot * Kt + kt) * U + u] = make_float2(di, di * acc);
        }
    }
    __syncthreads();
}

// Loads this lane's NPL receive entries of vector v (zeros when inactive).
template <int L, int NPL, bool F16>
__device__ __forceinline__ void load_vector(const Params &P, const void *base, long v, int j,
                                            bool active, float2 *r)
{
#pragma unroll
    for (int c = 0; c < NPL / 2; ++c) {
        const int b = 2 * (j + L * c);
        if (active) load_chunk<F16, 2>(base, v * P.B + b, b, P.B, P.vec_ok != 0, &r[2 * c]);
        else r[2 * c] = r[2 * c + 1] = make_float2(0.f, 0.f);
    }
}

// Reads this lane's part of column u from LDS.
template <int L, int NPL>
__device__ __forceinline__ void load_column(const float2 *col, int j, float2 *h)
{
#pragma unroll
    for (int c = 0; c < NPL / 2; ++c) {
        const float4 q = *reinterpret_cast<const float4 *>(col + 2 * (j + L * c));
        h[2 * c] = make_float2(q.x, q.y);
        h[2 * c + 1] = make_float2(q.z, q.w);
    }
}

// conj(h)^T r over this lane's entries, two independent accumulator pairs.
template <int NPL>
__device__ __forceinline__ float2 partial_inner(const float2 *h, const float2 *r)
{
    float ar0 = 0.f, ai0 = 0.f, ar1 = 0.f, ai1 = 0.f;
#pragma unroll
    for (int i = 0; i < NPL; i += 2) {
        ar0 = fmaf(h[i].x, r[i].x, ar0);
        ar0 = fmaf(h[i].y, r[i].y, ar0);
        ai0 = fmaf(h[i].x, r[i].y, ai0);
        ai0 = fmaf(-h[i].y, r[i].x, ai0);
        ar1 = fmaf(h[i + 1].x, r[i + 1].x, ar1);
        ar1 = fmaf(h[i + 1].y, r[i + 1].y, ar1);
        ai1 = fmaf(h[i + 1].x, r[i + 1].y, ai1);
        ai1 = fmaf(-h[i + 1].y, r[i + 1].x, ai1);
    }
    return make_float2(ar0 + ar1, ai0 + ai1);
}

// r <- r - h * delta (complex), this lane's entries.
template <int NPL>
__device__ __forceinline__ void axpy_sub(const float2 *h, float2 delta, float2 *r)
{
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        r[i].x = fmaf(-h[i].x, delta.x, r[i].x);
        r[i].x = fmaf(h[i].y, delta.y, r[i].x);
        r[i].y = fmaf(-h[i].x, delta.y, r[i].y);
        r[i].y = fmaf(-h[i].y, delta.x, r[i].y);
    }
}

// r <- r + h * a (complex), this lane's entries.
template <int NPL>
__device__ __forceinline__ void axpy_add(const float2 *h, float2 a, float2 *r)
{
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        r[i].x = fmaf(h[i].x, a.x, r[i].x);
        r[i].x = fmaf(-h[i].y, a.y, r[i].x);
        r[i].y = fmaf(h[i].x, a.y, r[i].y);
        r[i].y = fmaf(h[i].y, a.x, r[i].y);
    }
}

// Section III-C: approximate channel gain mu = d^-1 g (= p of the last sweep) and
// SINR rho = mu/(1-mu) = g/lambda_K; with lambda_K = 0 (BOX) mu = 1 and the
// finite rho = g Es/N0 is used.
__device__ __forceinline__ void gain_sinr(const Params &P, float lamK, float g, float pK,
                                          float *mu, float *rho)
{
    if (lamK > 0.f) {
        *mu = pK;
        *rho = g / lamK;
    } else {
        *mu = 1.0f;
        *rho = g * P.Es / P.N0;
    }
}

}  // namespace ocd
