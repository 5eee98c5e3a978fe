// ocd_mmse.hip -- explicit MMSE soft-output detection (Section II-B: the
// regularised Gram matrix and its inverse; Section II-E: exact channel gain and
// post-equalisation SINR).  This is the detector OCD approximates without forming
// the Gram matrix; it gives the reference error rate and throughput.
//
// One workgroup per tile of vectors, as in the OCD forward kernel: the H_w of the
// subcarriers a tile touches are staged once into LDS and shared by its vectors.
//   1. Lane groups form the upper triangle of A = H_w^H H_w + lambda I, one entry
//      per group at a time (a DPP sum over the group), and mirror it.
//   2. One wave per subcarrier inverts A in place by Gauss-Jordan elimination.  A
//      is Hermitian positive definite, so every pivot is a positive Schur
//      complement and no pivoting is needed.  Each step reads one LDS copy of the
//      work matrix and writes the other, so no step overwrites what it still reads.
//   3. A^-1 G = I - lambda A^-1 gives the gain mu_u = 1 - lambda [A^-1]_uu and
//      1 - mu_u = lambda [A^-1]_uu directly, without cancellation, hence the SINR
//      rho_u = mu_u / (1 - mu_u) and the soft-output coefficients.
//   4. Per vector: s = H_w^H y (lane group, DPP sums; it overlaps step 2 on the
//      waves that do not invert), then z = A^-1 s with one (user, axis) pair per
//      lane, and the per-axis max-log LLRs.
#include "ocd_stage.h"

namespace ocd {

struct MmseSmem {
    float2 *H;   // [maxslots][slot_stride]: H_w columns, FP32, zero-padded to Bpad
    float2 *A;   // [maxslots][2][U][U]: the two copies of the elimination's work matrix
    float *gd;   // [maxslots][U]: diagonal of G (zero for an all-zero column)
    float2 *lc;  // [maxslots][U]: soft-output coefficients (see llr_coef)
    float2 *s;   // [vpb][U]: matched-filter output of each vector
};

__device__ __forceinline__ MmseSmem mmse_carve(unsigned char *smem, const Params &P)
{
    MmseSmem s;
    size_t off = 0;
    s.H = reinterpret_cast<float2 *>(smem);
    off += (size_t)P.maxslots * P.slot_stride * 8;
    s.A = reinterpret_cast<float2 *>(smem + off);
    off += (size_t)P.maxslots * 2 * P.U * P.U * 8;
    s.lc = reinterpret_cast<float2 *>(smem + off);
    off += (size_t)P.maxslots * P.U * 8;
    s.s = reinterpret_cast<float2 *>(smem + off);
    off += (size_t)P.vpb * P.U * 8;
    s.gd = reinterpret_cast<float *>(smem + off);
    return s;
}

// Gauss-Jordan inversion in place by one wave.  Step k maps the work matrix M to M'
// with
//   M'_kk = 1/M_kk,  M'_kc = M_kc / M_kk,  M'_ik = -M_ik / M_kk,
//   M'_ic = M_ic - M_ik M_kc / M_kk  (i, c != k);
// after U steps M' = A^-1.  A0 holds the two copies of the U x U work matrix (the
// first one filled with A); each step reads one and writes the other, and the
// lanes of a wave issue their LDS operations in program order, so step k + 1 sees
// every write of step k.  Then the gain, SINR and soft-output coefficients of each
// user from the diagonal of A^-1 (A^-1 G = I - lambda A^-1); gd is the diagonal
// of G (zero for an all-zero column, whose coefficients are zero).
__device__ void invert_and_coefficients(const Params &P, float2 *A0, const float *gd, float2 *lc,
                                        int lane)
{
    const int U = P.U, E = U * U;
    const float lam = P.lam_default;
    for (int k = 0; k < U; ++k) {
        const float2 *src = A0 + (k & 1) * E;
        float2 *dst = A0 + ((k + 1) & 1) * E;
        const float piv = 1.0f / src[k * U + k].x;   // Hermitian: a real pivot
        const float2 *rowk = src + k * U;
        for (int e = lane; e < E; e += 64) {
            const int i = slot_of_row(P, e), c = e - i * U;   // e / U (e < 2^10)
            const float2 aik = src[i * U + k], akc = rowk[c], aic = src[e];
            float2 out;
            if (i == k) {
                out = c == k ? make_float2(piv, 0.f) : make_float2(akc.x * piv, akc.y * piv);
            } else if (c == k) {
                out = make_float2(-aik.x * piv, -aik.y * piv);
            } else {
                const float mx = aik.x * akc.x - aik.y * akc.y;
                const float my = aik.x * akc.y + aik.y * akc.x;
                out = make_float2(fmaf(-mx, piv, aic.x), fmaf(-my, piv, aic.y));
            }
            dst[e] = out;
        }
        __builtin_amdgcn_wave_barrier();
    }
    const float2 *Ai = A0 + (U & 1) * E;
    for (int u = lane; u < U; u += 64) {
        const float one_minus_mu = lam * Ai[u * U + u].x;
        const float mu = 1.0f - one_minus_mu, rho = mu / one_minus_mu;
        float2 co = make_float2(0.f, 0.f);
        if (gd[u] > 0.f && mu > 0.f && rho > 0.f)
            co = make_float2(1.0f / (mu * P.sqEs * P.qscale), rho * P.qscale * P.qscale);
        lc[u] = co;
    }
}

// z = A^-1 s for one (user, axis) pair, then its LLRs (item idx = 2u + axis of
// vector v): Ai the inverse, sv the vector's matched-filter row, co the user's
// soft-output coefficients.
__device__ __forceinline__ void solve_and_llr(const Params &P, const float2 *Ai, const float2 *sv,
                                              float2 co, long v, int idx)
{
    const int U = P.U, u = idx >> 1, ax = idx & 1;
    const float2 *row = Ai + (size_t)u * U;
    float acc = 0.f;
    for (int c = 0; c < U; ++c) {
        const float2 a = row[c], sc = sv[c];
        // Re: a.x s.x - a.y s.y;  Im: a.x s.y + a.y s.x
        const float s1 = ax ? sc.y : sc.x, s2 = ax ? sc.x : -sc.y;
        acc = fmaf(a.x, s1, fmaf(a.y, s2, acc));
    }
    if (P.z) reinterpret_cast<float *>(P.z)[v * 2 * U + idx] = acc;
    if (P.llr) {
        const int Q = P.Q, half = Q >> 1;
        float *dst = P.llr + (v * U + u) * Q + ax * half;
        const float t = acc * co.x;
        if (half == 3) axis_llrs<3>(t, co.y, dst);
        else if (half == 2) axis_llrs<2>(t, co.y, dst);
        else axis_llrs<1>(t, co.y, dst);
    }
}

template <int L, int NPL, bool F16>
__global__ __launch_bounds__(512) void k_mmse(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const MmseSmem sm = mmse_carve(smem, P);
    const int bid = P.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    stagger_loads(P);
    const Tile tile = tile_of(P, bid);
    const int U = P.U, Bpad = P.Bpad, E = U * U;
    const int grp = threadIdx.x / L, j = threadIdx.x % L, ngrp = blockDim.x / L;
    const bool active = grp < tile.nvb;
    const float lam = P.lam_default;

    // H_w chunk loads, then the receive vector: both round trips in flight together
    Smem hs = {};
    hs.H = sm.H;
    const int chunks = tile.nslots * U * (Bpad >> 1);
    float4 hbuf[STAGE_CHUNKS];
    stage_h_load<F16>(P, tile.w_first, tile.nslots, chunks, 0, hbuf);
    float2 r[NPL];
    load_vector<L, NPL, F16>(P, P.y, tile, grp, j, active, r);
    stage_h_store(P, hs, tile.nslots, chunks, 0, hbuf);
    stage_h_copy<F16>(P, hs, tile.w_first, tile.nslots, chunks, STAGE_CHUNKS * (int)blockDim.x);
    __syncthreads();
    clear_padding<L, NPL>(P, j, active, r);

    // 1. upper triangle of A = G + lambda I (entry (i, c), c >= i), mirrored below
    const int T = U * (U + 1) / 2;
    for (int t = grp; t < tile.nslots * T; t += ngrp) {
        const int sl = t / T;
        int q = t - sl * T, i = 0;
        while (q >= U - i) {   // row i of the triangle holds U - i entries
            q -= U - i;
            ++i;
        }
        const int c = i + q;
        const float2 *Hs = sm.H + (size_t)sl * P.slot_stride;
        float2 hi[NPL], hc[NPL];
        load_column<L, NPL>(Hs + (size_t)i * Bpad, j, hi);
        load_column<L, NPL>(Hs + (size_t)c * Bpad, j, hc);
        float re = 0.f, im = 0.f;   // conj(h_i)^T h_c over this lane's entries
#pragma unroll
        for (int e = 0; e < NPL; ++e) {
            re = fmaf(hi[e].x, hc[e].x, fmaf(hi[e].y, hc[e].y, re));
            im = fmaf(hi[e].x, hc[e].y, fmaf(-hi[e].y, hc[e].x, im));
        }
        re = group_sum<L>(re);
        im = group_sum<L>(im);
        if (j == 0) {
            float2 *A = sm.A + (size_t)sl * 2 * E;
            if (i == c) {
                A[i * U + i] = make_float2(re + lam, 0.f);
                sm.gd[sl * U + i] = re;
            } else {
                A[i * U + c] = make_float2(re, im);
                A[c * U + i] = make_float2(re, -im);
            }
        }
    }
    __syncthreads();

    // 2, 3. inversion and soft-output coefficients, one wave per staged subcarrier
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
    for (int sl = wave; sl < tile.nslots; sl += nwaves)
        invert_and_coefficients(P, sm.A + (size_t)sl * 2 * E, sm.gd + sl * U, sm.lc + sl * U, lane);

    // 4. matched filter s = H_w^H y (needs only the staged H_w, so the other waves
    // run it while a wave inverts); lane u mod L keeps s_u in the vector's LDS row
    const int slot = slot_of_group(P, tile, active ? grp : 0);
    float2 *sv = sm.s + (size_t)(active ? grp : 0) * U;
    if (active) {
        const float2 *Hs = sm.H + (size_t)slot * P.slot_stride;
        for (int u = 0; u < U; ++u) {
            float2 h[NPL];
            load_column<L, NPL>(Hs + (size_t)u * Bpad, j, h);
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int e = 0; e < NPL; ++e) {
                re = fmaf(h[e].x, r[e].x, fmaf(h[e].y, r[e].y, re));
                im = fmaf(h[e].x, r[e].y, fmaf(-h[e].y, r[e].x, im));
            }
            re = group_sum<L>(re);
            im = group_sum<L>(im);
            if (j == (u & (L - 1))) sv[u] = make_float2(re, im);
        }
    }
    __syncthreads();
    if (!active) return;

    // z = A^-1 s: lane pair index idx = 2u + axis computes one real component
    const float2 *Ai = sm.A + (size_t)slot * 2 * E + (U & 1) * E;
    const long v = (long)tile.vbase + grp;
    for (int idx = j; idx < 2 * U; idx += L)
        solve_and_llr(P, Ai, sv, sm.lc[slot * U + (idx >> 1)], v, idx);
}

// ------------------------------------------------------------------ matrix cores
//
// One subcarrier per 256-thread workgroup (U <= 8 users, S <= 16 symbols).  With
// X = [Re H, Im H] (B x 16, users past U zero) and Z = [Re Y, Im Y] (B x 32, the S
// receive vectors, columns past 2S zero), the Gram matrix and the matched filters
// of all S symbols are the real products X^T X (16 x 16) and X^T Z (16 x 32):
//   Re G_ij = (X^T X)_{i,j} + (X^T X)_{8+i,8+j},  Im G_ij = (X^T X)_{i,8+j} - (X^T X)_{8+i,j},
//   Re s_uv = (X^T Z)_{u,v} + (X^T Z)_{8+u,S+v},  Im s_uv = (X^T Z)_{u,S+v} - (X^T Z)_{8+u,v}.
// Wave 0 forms X^T X and waves 1, 2 the two 16-column tiles of X^T Z on the FP32
// matrix cores (v_mfma_f32_16x16x4f32: lane l supplies A[l mod 16][l / 16] and
// B[l / 16][l mod 16] and receives D[4 (l / 16) + r][l mod 16] in register r).  X
// and Z are staged antenna-major (16 and 32 floats per antenna), so each K step
// reads one conflict-free float per lane, and for X^T X the A and B operands are
// the same value.  Then the elimination, z = A^-1 s and the LLRs as above.

typedef float f32x4_mma __attribute__((ext_vector_type(4)));

// Bytes of dynamic LDS of the matrix-core kernel for K = Bpad antennas (a
// multiple of 4) and the problem's U, S.
size_t mmse_mfma_lds_bytes(int Kp, int U, int S)
{
    return (size_t)Kp * 50 * 4          // X (16 floats) and Z (32 floats) per antenna, padded
           + 16 * 48 * 4                // X^T X | X^T Z
           + (size_t)2 * U * U * 8      // work matrices
           + (size_t)U * 8              // soft-output coefficients
           + (size_t)S * U * 8          // matched filters
           + (size_t)U * 4;             // Gram diagonal
}

template <bool F16>
__global__ __launch_bounds__(256) void k_mmse_mfma(Params P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int U = P.U, S = P.S, B = P.B, Kp = P.Bpad, E = U * U;
    // rows of 17 and 33 floats: consecutive antennas fall in different LDS banks
    constexpr int XS = 17, ZS = 33;
    float *X = reinterpret_cast<float *>(smem);          // [Kp][XS]
    float *Z = X + (size_t)Kp * XS;                       // [Kp][ZS]
    float *D = Z + (size_t)Kp * ZS;                       // [16][48]
    float2 *A0 = reinterpret_cast<float2 *>(D + 16 * 48); // [2][U][U]
    float2 *lc = A0 + 2 * E;                              // [U]
    float2 *sv = lc + U;                                  // [S][U]
    float *gd = reinterpret_cast<float *>(sv + (size_t)S * U);
    const int w = P.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    stagger_loads(P);
    const int tid = threadIdx.x;

    // stage X and Z antenna-major, zero-padded: thread tid takes antenna b = tid
    // (per block of 256 antennas) of every column and every receive vector; all
    // of a block's loads are issued (branch-free: an invalid element reads the
    // first entry and is replaced by zero) before any is stored
    auto load_c = [&](const void *base, size_t i) -> float2 {
        if constexpr (F16) return half2_to_float2(static_cast<const uint32_t *>(base)[i]);
        else return static_cast<const float2 *>(base)[i];
    };
    const float2 zero2 = make_float2(0.f, 0.f);
    for (int b0 = 0; b0 < Kp; b0 += 256) {
        const int bb = b0 + tid;
        const bool ok = bb < B;
        float2 hx[8], hy[16];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool v_ok = ok && u < U;
            const float2 h = load_c(P.H, v_ok ? ((size_t)w * U + u) * B + bb : 0);
            hx[u] = v_ok ? h : zero2;
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const bool v_ok = ok && v < S;
            const float2 yv = load_c(P.y, v_ok ? ((size_t)w * S + v) * B + bb : 0);
            hy[v] = v_ok ? yv : zero2;
        }
        if (bb < Kp) {
            float *xr = X + bb * XS, *zr = Z + bb * ZS;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                xr[u] = hx[u].x;
                xr[8 + u] = hx[u].y;
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                if (v < S) {
                    zr[v] = hy[v].x;
                    zr[S + v] = hy[v].y;
                }
            }
            for (int c = 2 * S; c < 32; ++c) zr[c] = 0.f;   // columns 2S .. 31
        }
    }
    __syncthreads();

    // X^T X (wave 0), X^T Z columns 0-15 (wave 1) and 16-31 (wave 2); two chains
    const int wave = tid >> 6, lane = tid & 63;
    if (wave < 3) {
        const int i = lane & 15, kk = lane >> 4;
        f32x4_mma c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
        const float *zc = Z + (wave > 0 ? (wave - 1) * 16 : 0) + i;
        for (int kb = 0; kb < Kp; kb += 8) {
            const float a0 = X[(kb + kk) * XS + i];
            const float b0 = wave == 0 ? a0 : zc[(kb + kk) * ZS];
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, c0, 0, 0, 0);
            if (kb + 4 < Kp) {
                const float a1 = X[(kb + 4 + kk) * XS + i];
                const float b1 = wave == 0 ? a1 : zc[(kb + 4 + kk) * ZS];
                c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, c1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) D[(4 * kk + r) * 48 + wave * 16 + i] = c0[r] + c1[r];
    }
    __syncthreads();

    // A = G + lambda I and the matched filters from the real blocks
    const float lam = P.lam_default;
    for (int e = tid; e < E; e += 256) {
        const int i = slot_of_row(P, e), j = e - i * U;
        const float gr = D[i * 48 + j] + D[(8 + i) * 48 + 8 + j];
        const float gi = D[i * 48 + 8 + j] - D[(8 + i) * 48 + j];
        if (i == j) {
            A0[e] = make_float2(gr + lam, 0.f);
            gd[i] = gr;
        } else {
            A0[e] = make_float2(gr, gi);
        }
    }
    for (int e = tid; e < S * U; e += 256) {
        const int v = e / U, u = e - v * U;
        const float mr = D[u * 48 + 16 + v] + D[(8 + u) * 48 + 16 + S + v];
        const float mi = D[u * 48 + 16 + S + v] - D[(8 + u) * 48 + 16 + v];
        sv[e] = make_float2(mr, mi);
    }
    __syncthreads();
    if (wave == 0) invert_and_coefficients(P, A0, gd, lc, lane);
    __syncthreads();

    const float2 *Ai = A0 + (U & 1) * E;
    for (int e = tid; e < S * 2 * U; e += 256) {
        const int v = e / (2 * U), idx = e - v * 2 * U;
        solve_and_llr(P, Ai, sv + (size_t)v * U, lc[idx >> 1], (long)w * S + v, idx);
    }
}

// Staggered staging (plan field stagger) delays only the workgroups resident at
// launch: the occupancy of this kernel at this shape gives their count.
static hipError_t with_stagger_cap(const void *fn, int threads, size_t lds, Params &q)
{
    if (q.stagger <= 0) return hipSuccess;
    int per_cu = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
    if (e != hipSuccess) return e;
    q.stagger_cap = per_cu * device_cu_count();
    return hipSuccess;
}

template <bool F16>
static hipError_t launch_mmse_mfma_t(const Params &p, size_t lds, hipStream_t s)
{
    Params q = p;
    const hipError_t e = with_stagger_cap(reinterpret_cast<const void *>(k_mmse_mfma<F16>), 256, lds, q);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mmse_mfma<F16>), dim3(q.nblocks), dim3(256), lds, s, q);
    return hipGetLastError();
}

hipError_t launch_mmse_mfma(bool f16, const Params &p, size_t lds, hipStream_t s)
{
    return f16 ? launch_mmse_mfma_t<true>(p, lds, s) : launch_mmse_mfma_t<false>(p, lds, s);
}

template <int L, int NPL, bool F16>
static hipError_t launch_mmse_f(const Params &p, int threads, size_t lds, hipStream_t s)
{
    Params q = p;
    const hipError_t e =
        with_stagger_cap(reinterpret_cast<const void *>(k_mmse<L, NPL, F16>), threads, lds, q);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mmse<L, NPL, F16>), dim3(q.nblocks), dim3(threads), lds, s, q);
    return hipGetLastError();
}

template <int L, int NPL>
static hipError_t launch_mmse_t(bool f16, const Params &p, int threads, size_t lds, hipStream_t s)
{
    return f16 ? launch_mmse_f<L, NPL, true>(p, threads, lds, s)
               : launch_mmse_f<L, NPL, false>(p, threads, lds, s);
}

template <int L>
static hipError_t launch_mmse_l(int NPL, bool f16, const Params &p, int threads, size_t lds,
                                hipStream_t s)
{
    switch (NPL) {
    case 2: return launch_mmse_t<L, 2>(f16, p, threads, lds, s);
    case 4: return launch_mmse_t<L, 4>(f16, p, threads, lds, s);
    case 8: return launch_mmse_t<L, 8>(f16, p, threads, lds, s);
    case 16: return launch_mmse_t<L, 16>(f16, p, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mmse(int L, int NPL, bool f16, const Params &p, int threads, size_t lds,
                       hipStream_t s)
{
    switch (L) {
    case 8: return launch_mmse_l<8>(NPL, f16, p, threads, lds, s);
    case 16: return launch_mmse_l<16>(NPL, f16, p, threads, lds, s);
    case 32: return launch_mmse_l<32>(NPL, f16, p, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ocd
