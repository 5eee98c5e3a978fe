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
    float2 *lc;    // [maxslots][U]: soft-output coefficients (see llr_coef)
    float2 *z;     // [vpb + 1][U]: current z of each vector; idle groups share the last row
    float2 *zbar;  // [vpb + 1][U]: adjoint only, dLoss/dz
    float *part;   // [(K + 2) * waves]: adjoint only, per-wave partial sums (sweeps, beta, loss)
    float2 *zh;    // [vpb + 1][K][U]: training step only, z after every sweep
};

// Row of the per-vector LDS arrays used by lane group grp.
__device__ __forceinline__ int zrow_of(const Params &P, int grp) { return grp < P.vpb ? grp : P.vpb; }

__device__ __forceinline__ Smem carve(unsigned char *smem, const Params &P, int vpb_cap,
                                      bool backward, bool train = false)
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
    s.lc = reinterpret_cast<float2 *>(smem + off);
    off += (size_t)P.maxslots * P.U * 8;
    const size_t zrows = (size_t)(P.vpb + 1) * P.U * 8;
    s.z = reinterpret_cast<float2 *>(smem + off);
    off += zrows;
    s.zbar = nullptr;
    s.part = nullptr;
    s.zh = nullptr;
    if (train) {   // 8-byte aligned here: before the partials
        s.zh = reinterpret_cast<float2 *>(smem + off);
        off += (size_t)(P.vpb + 1) * P.K * P.U * 8;
    }
    if (backward) {
        s.zbar = reinterpret_cast<float2 *>(smem + off);
        off += zrows;
        s.part = reinterpret_cast<float *>(smem + off);
    }
    (void)vpb_cap;
    return s;
}

// The vectors of one workgroup: [vbase, vbase + nvb) in (subcarrier, symbol)
// order; they touch subcarriers w_first .. w_first + nslots - 1.
// Vector indices fit in 32 bits (W * S <= 2^30 is checked on the host).
struct Tile {
    int vbase;
    int nvb, w_first, nslots;
};

// Staged slot of lane group grp's vector: (vbase + grp) / S - w_first, from the
// offset of the group in its first subcarrier (non-negative, below 2^31).
__device__ __forceinline__ int slot_of_group(const Params &P, const Tile &tile, int grp)
{
    const int x = tile.vbase - tile.w_first * P.S + grp;
    return (int)divide_invariant((unsigned)x, P.divS_m, P.divS_s1, P.divS_s2);
}

// Staggered staging: workgroups are dispatched in blockIdx order, so the ones
// launched first sit on every CU before later ones arrive.  If all of them issue
// their loads at once, HBM serves the requests interleaved and every workgroup
// gets its data late; delaying workgroup b by max(0, b/128 - 1) * stagger units of
// 512 clocks lets the first ones (the first 256 unchanged) start computing while
// later ones load.  Workgroups beyond the first stagger_cap (those resident at
// once) are dispatched only as earlier ones retire and do not wait.
__device__ __forceinline__ void stagger_loads(const Params &P)
{
    if (P.stagger <= 0 || (int)blockIdx.x >= P.stagger_cap) return;
    const int n = ((int)blockIdx.x / 128 - 1) * P.stagger;
    for (int i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(8);   // 8 x 64 clocks
}

__device__ __forceinline__ Tile tile_of(const Params &P, int bid)
{
    Tile t;
    const int nvec = P.W * P.S;
    t.vbase = bid * P.vpb;
    const int rem = nvec - t.vbase;
    t.nvb = rem < P.vpb ? rem : P.vpb;
    t.w_first = t.vbase / P.S;
    t.nslots = (t.vbase + t.nvb - 1) / P.S - t.w_first + 1;
    return t;
}

// Copy of H_w into LDS in two halves, so that the caller can put other global
// loads (its receive vectors) in flight between them: stage_h_load issues the
// loads of up to STAGE_CHUNKS chunks (two complex entries each) per thread into
// registers, stage_h_store writes them to LDS (FP32, zero padded to Bpad).  Chunk
// c of a tile is row c / (Bpad/2) (the rows of the touched subcarriers are
// consecutive in [W][U][B]) and antennas 2 (c mod Bpad/2) and the next one.
constexpr int STAGE_CHUNKS = 4;

// Dense staging: rows of even length B = Bpad, aligned, and one subcarrier per
// tile.  Then chunk c is complex entries 2c and 2c + 1 both of the tile's rows in
// global memory and of the LDS slot, and needs no row/antenna arithmetic.
__device__ __forceinline__ bool dense_stage(const Params &P, int nslots)
{
    return P.vec_ok && P.B == P.Bpad && nslots == 1;
}

template <bool F16>
__device__ __forceinline__ void stage_h_load(const Params &P, int w_first, int nslots, int total,
                                             int c0, float4 (&buf)[STAGE_CHUNKS])
{
    const int half = P.Bpad >> 1;
    const int sh = __ffs(half) - 1;   // Bpad is a power of two
    const long rbase = (long)w_first * P.U;
    if (dense_stage(P, nslots)) {
        const unsigned char *hb =
            static_cast<const unsigned char *>(P.H) + (size_t)rbase * P.B * cbytes<F16>();
#pragma unroll
        for (int i = 0; i < STAGE_CHUNKS; ++i) {
            const int c = c0 + i * (int)blockDim.x + (int)threadIdx.x;
            buf[i] = load_pair_at<F16>(hb, c < total ? (unsigned)c * 2u * cbytes<F16>() : 0u);
        }
        return;
    }
    if (P.vec_ok) {
        // B even: a chunk is wholly inside or wholly outside the row.  Out-of-range
        // chunks load a valid address and are replaced by zeros, so no load sits
        // behind a branch and all of them are in flight together.  The rows of the
        // tile start at a workgroup-uniform address; per-lane offsets are 32-bit.
        const unsigned char *hb =
            static_cast<const unsigned char *>(P.H) + (size_t)rbase * P.B * cbytes<F16>();
#pragma unroll
        for (int i = 0; i < STAGE_CHUNKS; ++i) {
            const int c = c0 + i * (int)blockDim.x + (int)threadIdx.x;
            const int row = c >> sh, b = (c & (half - 1)) << 1;
            const bool ok = c < total && b < P.B;
            buf[i] = load_pair_at<F16>(hb, ok ? (unsigned)(row * P.B + b) * cbytes<F16>() : 0u);
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < STAGE_CHUNKS; ++i) {
        const int c = c0 + i * (int)blockDim.x + (int)threadIdx.x;
        float2 v[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
        if (c < total) {
            const int row = c >> sh, b = (c & (half - 1)) << 1;
            load_chunk<F16, 2>(P.H, (rbase + row) * P.B + b, b, P.B, false, v);
        }
        buf[i] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
    }
}

// row / U for the row index of a staged H_w row (row < 2^16, U <= 32): the float
// product is within 0.5 / U of an integer plus one half, so truncation is exact.
__device__ __forceinline__ int slot_of_row(const Params &P, int row)
{
    return (int)fmaf((float)row, P.invU, 0.5f * P.invU);
}

__device__ __forceinline__ void stage_h_store(const Params &P, const Smem &sm, int nslots,
                                              int total, int c0, const float4 (&buf)[STAGE_CHUNKS])
{
    if (dense_stage(P, nslots)) {
#pragma unroll
        for (int i = 0; i < STAGE_CHUNKS; ++i) {
            const int c = c0 + i * (int)blockDim.x + (int)threadIdx.x;
            if (c < total) *reinterpret_cast<float4 *>(sm.H + 2 * c) = buf[i];
        }
        return;
    }
    const int half = P.Bpad >> 1;
    const int sh = __ffs(half) - 1;
    const int gap = P.slot_stride - P.U * P.Bpad;   // padding between LDS slots
#pragma unroll
    for (int i = 0; i < STAGE_CHUNKS; ++i) {
        const int c = c0 + i * (int)blockDim.x + (int)threadIdx.x;
        if (c < total) {
            const int row = c >> sh, b = (c & (half - 1)) << 1;
            const int slot = slot_of_row(P, row);
            // antennas past B (loaded from a placeholder address) become zero padding
            const float4 q = b < P.B ? buf[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            *reinterpret_cast<float4 *>(sm.H + (size_t)row * P.Bpad + (size_t)slot * gap + b) = q;
        }
    }
}

// Copies H_w of every touched subcarrier into LDS (all passes).
template <bool F16>
__device__ __forceinline__ void stage_h_copy(const Params &P, const Smem &sm, int w_first,
                                             int nslots, int total, int c0)
{
    for (; c0 < total; c0 += STAGE_CHUNKS * (int)blockDim.x) {
        float4 buf[STAGE_CHUNKS];
        stage_h_load<F16>(P, w_first, nslots, total, c0, buf);
        stage_h_store(P, sm, nslots, total, c0, buf);
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

// Per (subcarrier, user) constants of the soft output, so that the LLRs of a
// vector are L_b = c D_b(t) with t = z_u a (z in units of the level spacing of
// the unit-energy constellation, after the 1/(mu sqrt(Es)) unbiasing of
// Section III-C) and D_b the per-axis max-log metric: a = 1/(mu sqrt(Es) scale),
// c = rho scale^2.  A user with rho or mu not positive (zero column) gets (0, 0):
// all of its LLRs are zero.
__device__ __forceinline__ float2 llr_coef(const Params &P, float g, float pK, float lamK)
{
    float mu, rho;
    gain_sinr(P, lamK, g, pK, &mu, &rho);
    if (!(rho > 0.f && mu > 0.f)) return make_float2(0.f, 0.f);
    return make_float2(1.0f / (mu * P.sqEs * P.qscale), rho * P.qscale * P.qscale);
}

// Soft output of one axis of one user: t = the axis of z_u times a, c = the
// LLR scale (llr_coef); writes the HALF LLRs of that axis, MSB first.
template <int HALF, typename Dst>
__device__ __forceinline__ void axis_llrs(float t, float c, Dst dst)
{
    float D[HALF];
    pam_metrics<HALF>(t, D);
#pragma unroll
    for (int b = 0; b < HALF; ++b) dst[b] = c * D[b];
}

// Algorithm 1's preprocessing once per staged subcarrier (or a copy of the
// precomputed values): g_u = ||h_u||^2, d_u^-1 = (g_u + lambda_k)^-1 (0 if that
// is 1/0), p_u = d_u^-1 g_u.  Ends with a workgroup barrier, after which the
// staged H_w is visible to every thread.
// BP = L * NPL (= P.Bpad) is a compile-time constant, so the row reads unroll and
// issue together.
template <int BP>
__device__ void stage_preprocess(const Params &P, const Smem &sm, int w_first, int nslots)
{
    const int U = P.U, Bpad = BP;
    const int Kt = P.per_sweep ? P.K : 1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
    const int rows = nslots * U;
    const float lamK = P.lambda ? global_ptr(P.lambda)[P.K - 1] : P.lam_default;
    if (P.g_in) {
        for (int i = threadIdx.x; i < rows; i += blockDim.x) {
            const int slot = slot_of_row(P, i), u = i - slot * U;
            const float g = global_ptr(P.g_in)[(long)w_first * U + i];
            sm.g[i] = g;
            sm.lc[i] = llr_coef(P, g, global_ptr(P.p_in)[((long)(w_first + slot) * Kt + Kt - 1) * U + u],
                                lamK);
        }
        for (int i = threadIdx.x; i < nslots * Kt * U; i += blockDim.x) {
            const long gi = (long)w_first * Kt * U + i;
            sm.dp[i] = make_float2(global_ptr(P.dinv_in)[gi], global_ptr(P.p_in)[gi]);
        }
        __syncthreads();
        return;
    }
    __syncthreads();
    // a 16-lane group per row (one DPP row), rows dealt round-robin over the waves;
    // lane l of the group sums entries l, l + 16, ... (k_preprocess sums the same way)
    const int grp16 = lane >> 4, l16 = lane & 15;
    for (int base = 0; base < rows; base += 4 * nwaves) {
        const int row = base + wave + grp16 * nwaves;
        const bool live = row < rows;
        const int slot = live ? slot_of_row(P, row) : 0, u = live ? row - slot * U : 0;
        float acc = 0.f;
        if (live) {
            const float2 *h = sm.H + (size_t)slot * P.slot_stride + (size_t)u * Bpad;
#pragma unroll
            for (int i = 0; i < (BP + 15) / 16; ++i) {   // entries l16, l16 + 16, ... < BP
                const int b = l16 + 16 * i;
                if (b < BP) acc = fmaf(h[b].x, h[b].x, fmaf(h[b].y, h[b].y, acc));
            }
        }
        acc = group_sum<16>(acc);
        if (!live) continue;
        if (l16 == 0) {
            sm.g[row] = acc;
            // p of the last sweep, computed as for sm.dp below
            const float den = acc + lamK;
            const float di = den > 0.f ? 1.0f / den : 0.f;
            sm.lc[row] = llr_coef(P, acc, di * acc, lamK);
        }
        for (int kt = l16; kt < Kt; kt += 16) {
            const float lam = P.lambda ? global_ptr(P.lambda)[kt] : P.lam_default;
            const float den = acc + lam;
            const float di = den > 0.f ? 1.0f / den : 0.f;
            sm.dp[((size_t)slot * Kt + kt) * U + u] = make_float2(di, di * acc);
        }
    }
    __syncthreads();
}

// Loads this lane's NPL receive entries of vector v.  On the vector path the
// loads are branch-free and nothing reads them here, so they stay in flight
// while the caller stages H; antennas past B and idle groups load a placeholder
// address and must be cleared with clear_padding() before first use.
template <int L, int NPL, bool F16>
__device__ __forceinline__ void load_vector(const Params &P, const void *base, const Tile &tile,
                                            int grp, int j, bool active, float2 *r)
{
    if (P.vec_ok) {
        // the tile's vectors start at a workgroup-uniform address; 32-bit offsets
        const unsigned char *tb =
            static_cast<const unsigned char *>(base) + (size_t)tile.vbase * P.B * cbytes<F16>();
#pragma unroll
        for (int c = 0; c < NPL / 2; ++c) {
            const int b = 2 * (j + L * c);
            const bool ok = active && b < P.B;
            const float4 q =
                load_pair_at<F16>(tb, ok ? (unsigned)(grp * P.B + b) * cbytes<F16>() : 0u);
            r[2 * c] = make_float2(q.x, q.y);
            r[2 * c + 1] = make_float2(q.z, q.w);
        }
        return;
    }
    const long v = (long)tile.vbase + grp;
#pragma unroll
    for (int c = 0; c < NPL / 2; ++c) {
        const int b = 2 * (j + L * c);
        if (active) load_chunk<F16, 2>(base, v * P.B + b, b, P.B, false, &r[2 * c]);
        else r[2 * c] = r[2 * c + 1] = make_float2(0.f, 0.f);
    }
}

// Zeroes the entries load_vector filled from placeholder addresses.  With
// B = L * NPL there is no padding, and the residuals of idle groups are never
// stored nor mixed into another group's sums, so nothing needs clearing.
template <int L, int NPL>
__device__ __forceinline__ void clear_padding(const Params &P, int j, bool active, float2 *r)
{
    if (!P.vec_ok || P.B == P.Bpad) return;
#pragma unroll
    for (int c = 0; c < NPL / 2; ++c) {
        const bool ok = active && 2 * (j + L * c) < P.B;
        r[2 * c] = ok ? r[2 * c] : make_float2(0.f, 0.f);
        r[2 * c + 1] = ok ? r[2 * c + 1] : make_float2(0.f, 0.f);
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

// Operands of one coordinate update: this lane's part of column u, (d_u^-1, p_u)
// and the current z_u.
template <int NPL>
struct UpdateOperands {
    float2 h[NPL];
    float2 dp, zo;
};

template <int L, int NPL>
__device__ __forceinline__ void fetch_operands(const float2 *Hs, int Bpad, const float2 *dpk,
                                               const float2 *zv, int u, int j,
                                               UpdateOperands<NPL> &o)
{
    load_column<L, NPL>(Hs + (size_t)u * Bpad, j, o.h);
    o.dp = dpk[u];
    o.zo = zv[u];
}

// conj(h)^T r over this lane's entries with CHAINS accumulators per component.
// One chain: the real and imaginary chains alternate, which keeps dependent FMAs
// two issue slots apart (their latency), and there is no final merge -- the
// choice when several waves share a SIMD.  Two chains halve the dependency
// depth for one merge per component -- the choice when few waves do.
// Channel entries are float2, or an IEEE half pair packed in 32 bits (FP16 storage
// kept as is in registers): the FMAs below then take the half operands directly
// (mixed-precision FMA, exact conversion, one rounding), with the same results as
// converting first.
__device__ __forceinline__ float hre(const float2 &v) { return v.x; }
__device__ __forceinline__ float him(const float2 &v) { return v.y; }
__device__ __forceinline__ float hre(const uint32_t &v)
{
    return __low2float(*reinterpret_cast<const __half2 *>(&v));
}
__device__ __forceinline__ float him(const uint32_t &v)
{
    return __high2float(*reinterpret_cast<const __half2 *>(&v));
}

template <int NPL, int CHAINS = 1, typename HT>
__device__ __forceinline__ float2 partial_inner(const HT *h, const float2 *r)
{
    static_assert(CHAINS == 1 || (CHAINS == 2 && NPL % 2 == 0), "one or two chains");
    float ar[CHAINS], ai[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) ar[c] = ai[c] = 0.f;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        const int c = i % CHAINS;
        ar[c] = fmaf(hre(h[i]), r[i].x, ar[c]);
        ai[c] = fmaf(hre(h[i]), r[i].y, ai[c]);
        ar[c] = fmaf(him(h[i]), r[i].y, ar[c]);
        ai[c] = fmaf(-him(h[i]), r[i].x, ai[c]);
    }
    if constexpr (CHAINS == 2) return make_float2(ar[0] + ar[1], ai[0] + ai[1]);
    return make_float2(ar[0], ai[0]);
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

// One coordinate update of Algorithm 1 for the lanes of a group:
//   z_u' = proj(d_u^-1 h_u^H r + p_u z_u),  r <- r - h_u (z_u' - z_u).
// h: this lane's part of column u; dp = (d_u^-1, p_u); zo = z_u.  Returns z_u'.
// UPDATE_R = false leaves r as it is: the last update of the last sweep, after
// which the residual is never read again.
template <int L, int NPL, bool BOX, int CHAINS = 1, bool UPDATE_R = true, typename HT>
__device__ __forceinline__ float2 coordinate_update(const HT *h, float2 dp, float2 zo,
                                                    float beta, float2 *r)
{
    const float2 ip = group_sum2<L>(partial_inner<NPL, CHAINS>(h, r));
    float cr = fmaf(dp.x, ip.x, dp.y * zo.x);
    float ci = fmaf(dp.x, ip.y, dp.y * zo.y);
    if constexpr (BOX) {
        cr = fminf(fmaxf(cr, -beta), beta);
        ci = fminf(fmaxf(ci, -beta), beta);
    }
    // r <- r - h Delta with Delta = z_u' - z_u, written with -Delta so that h enters
    // only with positive sign (the inner product above already uses -Im h; a shared
    // negated copy would cost one instruction per entry).  Im Delta = -ndi enters as a
    // negated operand, which the FMA takes for free (a - b is exactly -(b - a)).
    // Same bits as axpy_sub.
    if constexpr (!UPDATE_R) return make_float2(cr, ci);
    const float ndr = zo.x - cr, ndi = zo.y - ci;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        r[i].x = fmaf(hre(h[i]), ndr, r[i].x);
        r[i].x = fmaf(him(h[i]), -ndi, r[i].x);
        r[i].y = fmaf(hre(h[i]), ndi, r[i].y);
        r[i].y = fmaf(him(h[i]), ndr, r[i].y);
    }
    return make_float2(cr, ci);
}


}  // namespace ocd
