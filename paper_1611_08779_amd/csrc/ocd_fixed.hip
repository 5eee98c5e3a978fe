// ocd_fixed.hip -- Algorithm 1 in the fixed-point datapath of Section IV-C, for
// comparing the paper's 16-bit design with floating point on the same inputs.
//
// Words (H, y, the residual r, z, beta, d^-1, p) are 16-bit two's complement with
// 11 fractional bits (Q5.11).  Products of two words are exact; the inner
// products are exact 64-bit sums of them (the paper's 36-bit adder tree, which
// they fit on any input whose sums stay in 36 bits).  ||h_u||^2 + alpha and
// h_u^H r are shifted right by b = ceil(log2 B); the two shifts cancel in
// d^-1 h^H r.  The reciprocal d^-1 comes from normalising its input to [1/2, 1),
// indexing a 2048-entry table of 18-bit normalised reciprocals with the 11 bits
// after the leading one, and shifting back.  Every narrowing to 16 bits rounds
// half up and saturates.  The paper's design has no soft-output unit: the LLRs
// are formed in FP32 from the fixed-point z and p, as in the floating-point path.
//
// One lane group of L lanes per vector; lane j holds residual entries
// b = j + L i.  The updates run in FP64 on integer values: every intermediate of
// the datapath is an integer below 2^53 (products below 2^32, sums below 2^41,
// d^-1 times a shifted inner product below 2^51), so every FP64 operation on them
// is exact, a floor after a power-of-two scale is the arithmetic shift, and
// clamps are the saturation; MI355X runs FP64 FMAs at the FP32 vector rate.  The
// sums are exact, so the order of the cross-lane sums does not matter and the
// result is bit-exact.  The H_w a workgroup touches are staged in LDS once, their
// int16 values held exactly in FP32 (where they fit in 32 KB), so that an update's
// column read is an LDS read rather than a round trip to the L2, and each entry
// reaches FP64 in one conversion.
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "ocd_api_internal.h"
#include "ocd_stage.h"

namespace ocd {

struct FxParams {
    int B, U, W, S, K, Q, box, b;
    long long lam_q;    // alpha in Q.22
    int beta_fx;        // box half-width in Q.11
    float lam, Es, N0, sqEs, qscale;
    const int16_t *H;   // [W][U][B][2]
    const int16_t *y;   // [W][S][B][2]
    int16_t *z;         // [W][S][U][2] or nullptr
    float *llr;         // [W][S][U][Q] or nullptr
};

__device__ __forceinline__ long long fx_sat16(long long v)
{
    return v < -32768 ? -32768 : (v > 32767 ? 32767 : v);
}

// v / 2^s rounded half up (s >= 1)
__device__ __forceinline__ long long fx_round_shift(long long v, int s)
{
    return (v + (1ll << (s - 1))) >> s;
}

// Q.11 reciprocal of x > 0 given in Q.22 units: normalise, index the table with
// the 11 bits after the leading one, denormalise; 0 for x <= 0.  The table entry
// round(2^18 / (1 + (i + 1/2) / 2048)) is evaluated where it is needed (IEEE
// double division is correctly rounded, so it is the table's value).
__device__ __forceinline__ long long fx_recip(long long x)
{
    if (x <= 0) return 0;
    const int n = 64 - __clzll(x);   // bit length
    const long long idx = n >= 12 ? (x >> (n - 12)) & 2047 : (x << (12 - n)) & 2047;
    const long long lut = (long long)floor(262144.0 / (1.0 + ((double)idx + 0.5) / 2048.0) + 0.5);
    const long long d = (16 - n >= 0) ? lut * (1ll << (16 - n)) : fx_round_shift(lut, n - 16);
    return fx_sat16(d);
}

// A 64-bit lane value from another lane of the row: the DPP move of both halves.
template <int CTRL>
__device__ __forceinline__ long long dpp_get_i64(long long x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)x, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xF, 0xF, false);
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Exact FP64 helpers on integer values (see the header).
__device__ __forceinline__ double fx_sat16d(double v) { return fmin(fmax(v, -32768.0), 32767.0); }

// v / 2^s rounded half up: floor((v + 2^(s-1)) 2^-s), exact for integer v < 2^53
__device__ __forceinline__ double fx_round_shiftd(double v, double half, double inv)
{
    return floor((v + half) * inv);
}

template <int CTRL>
__device__ __forceinline__ double dpp_get_f64(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the L lanes of an aligned group (L = 16 or 32), the same in every lane;
// the values are integers below 2^53, so every partial sum is exact.
template <int L>
__device__ __forceinline__ double group_sum_f64(double x)
{
    x += dpp_get_f64<DPP_QUAD_XOR1>(x);
    x += dpp_get_f64<DPP_QUAD_XOR2>(x);
    x += dpp_get_f64<DPP_ROW_HALF_MIRROR>(x);
    x += dpp_get_f64<DPP_ROW_MIRROR>(x);
    if constexpr (L >= 32) x += __shfl_xor(x, 16, 32);
    return x;
}

// Exact sum over the L lanes of an aligned group (L = 16 or 32), the same in
// every lane; integer addition is associative, so the order does not matter.
template <int L>
__device__ __forceinline__ long long group_sum_i64(long long x)
{
    x += dpp_get_i64<DPP_QUAD_XOR1>(x);
    x += dpp_get_i64<DPP_QUAD_XOR2>(x);
    x += dpp_get_i64<DPP_ROW_HALF_MIRROR>(x);
    x += dpp_get_i64<DPP_ROW_MIRROR>(x);
    if constexpr (L >= 32) x += __shfl_xor(x, 16, 32);
    return x;
}

// STAGED: the H_w of the subcarriers a workgroup touches are copied into LDS once
// (int16 values held exactly in FP32), and every update reads its column there;
// otherwise (channels too large for the LDS budget) each update reads its column
// from global memory, where the S symbols of a subcarrier share it through the
// caches.  The arithmetic is the same either way.
template <int L, int NPL, bool STAGED>
__global__ __launch_bounds__(256) void k_forward_fx(FxParams P)
{
    constexpr int G = 256 / L;
    __shared__ int zs[G][32][2];
    __shared__ int ds[G][32], ps[G][32];
    __shared__ long long gs[G][32];
    extern __shared__ __align__(16) float2 hst[];    // STAGED: [slots][U][B] int16 values in FP32
    const int grp = threadIdx.x / L, j = threadIdx.x % L;
    const long v = (long)blockIdx.x * G + grp;
    const long nvec = (long)P.W * P.S;
    const int U = P.U, B = P.B, b = P.b;
    const float2 *Hs = nullptr;
    if constexpr (STAGED) {
        const long v0 = (long)blockIdx.x * G, vl = (v0 + G < nvec ? v0 + G : nvec) - 1;
        const long w_first = v0 / P.S;
        const int total = (int)(vl / P.S - w_first + 1) * U * B;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(P.H) + (size_t)w_first * U * B;
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
            const uint32_t e = src[i];
            hst[i] = make_float2((float)(int16_t)(e & 0xFFFFu), (float)(int16_t)(e >> 16));
        }
        __syncthreads();
        Hs = hst + (size_t)((v < nvec ? v : v0) / P.S - w_first) * U * B;
    }
    if (v >= nvec) return;   // a whole lane group at once
    const int16_t *Hw = P.H + (size_t)(v / P.S) * U * B * 2;
    const int16_t *yv = P.y + (size_t)v * B * 2;

    double rr[NPL], ri[NPL];   // residual entries j + L i, Q.11 integers
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        const int a = j + L * i;
        rr[i] = a < B ? (double)yv[2 * a] : 0.0;
        ri[i] = a < B ? (double)yv[2 * a + 1] : 0.0;
    }

    // preprocessing (Alg. 1, initialisation): ||h_u||^2, d_u^-1, p_u
    for (int u = 0; u < U; ++u) {
        const int16_t *hu = Hw + (size_t)u * B * 2;
        long long g = 0;
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            const int a = j + L * i;
            if (a < B) {
                const long long hr = hu[2 * a], hi = hu[2 * a + 1];
                g += hr * hr + hi * hi;
            }
        }
        g = group_sum_i64<L>(g);
        if (j == 0) {
            const long long d = fx_recip((g + P.lam_q) >> b);
            gs[grp][u] = g;
            ds[grp][u] = (int)d;
            ps[grp][u] = (int)fx_sat16(fx_round_shift(d * (g >> b), 22));
            zs[grp][u][0] = 0;
            zs[grp][u][1] = 0;
        }
    }
    __builtin_amdgcn_wave_barrier();

    // column entries as (re, im) int16 pairs in one dword; lanes past B hold 0
    auto load_col = [&](int u, uint32_t (&h)[NPL]) {
        const uint32_t *hu = reinterpret_cast<const uint32_t *>(Hw) + (size_t)u * B;
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            const int a = j + L * i;
            h[i] = a < B ? hu[a] : 0u;
        }
    };
    // the same column from the staged copy (int16 values held exactly in FP32)
    auto load_col_s = [&](int u, float2 (&h)[NPL]) {
        const float2 *hu = Hs + (size_t)u * B;
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            const int a = j + L * i;
            h[i] = a < B ? hu[a] : make_float2(0.f, 0.f);
        }
    };
    const double inv_b = ldexp(1.0, -b);
    uint32_t hn[NPL];
    float2 hf[NPL];
    if constexpr (STAGED) load_col_s(0, hf);
    else load_col(0, hn);
    for (int k = 0; k < P.K; ++k)
        for (int u = 0; u < U; ++u) {
            double hr[NPL], hi[NPL];
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
                hr[i] = STAGED ? (double)hf[i].x : (double)(int16_t)(hn[i] & 0xFFFFu);
                hi[i] = STAGED ? (double)hf[i].y : (double)(int16_t)(hn[i] >> 16);
            }
            // the next update's column is in flight while this one computes
            if constexpr (STAGED) load_col_s(u + 1 < U ? u + 1 : 0, hf);
            else load_col(u + 1 < U ? u + 1 : 0, hn);
            double ire = 0.0, iim = 0.0;   // h_u^H r, Q.22 integers
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
                ire = fma(hr[i], rr[i], fma(hi[i], ri[i], ire));
                iim = fma(hr[i], ri[i], fma(-hi[i], rr[i], iim));
            }
            ire = floor(group_sum_f64<L>(ire) * inv_b);   // arithmetic shift by b
            iim = floor(group_sum_f64<L>(iim) * inv_b);
            const double d = ds[grp][u], p = ps[grp][u];
            const double zr = zs[grp][u][0], zi = zs[grp][u][1];
            // c = d^-1 h^H r + p z in Q.33, narrowed to Q.11
            const double h22 = 2097152.0, i22 = 1.0 / 4194304.0;
            double cre = fx_sat16d(fx_round_shiftd(fma(d, ire, p * zr * 2048.0), h22, i22));
            double cim = fx_sat16d(fx_round_shiftd(fma(d, iim, p * zi * 2048.0), h22, i22));
            if (P.box) {
                const double bt = P.beta_fx;
                cre = fmin(fmax(cre, -bt), bt);
                cim = fmin(fmax(cim, -bt), bt);
            }
            // r - round(h (c - z) / 2^11), each component saturated.  The 2^-11 is
            // folded into (c - z): every product and partial sum is then an integer
            // times 2^-11 below 2^22, exact in FP64, so the floor sees the same value
            // as with the scale applied after the sum.
            const double dre = (cre - zr) * (1.0 / 2048.0), dim = (cim - zi) * (1.0 / 2048.0);
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
                const double tr = floor(fma(hr[i], dre, fma(-hi[i], dim, 0.5)));
                const double ti = floor(fma(hr[i], dim, fma(hi[i], dre, 0.5)));
                rr[i] = fx_sat16d(rr[i] - tr);
                ri[i] = fx_sat16d(ri[i] - ti);
            }
            __builtin_amdgcn_wave_barrier();   // every lane has read z_u
            if (j == 0) {
                zs[grp][u][0] = (int)cre;
                zs[grp][u][1] = (int)cim;
            }
            __builtin_amdgcn_wave_barrier();
        }

    // outputs: lane pair index idx = 2u + axis
    const int Q = P.Q, half = Q >> 1;
    for (int idx = j; idx < 2 * U; idx += L) {
        const int u = idx >> 1, ax = idx & 1;
        const int zv = zs[grp][u][ax];
        if (P.z) P.z[(size_t)v * U * 2 + idx] = (int16_t)zv;
        if (P.llr) {
            const float g = (float)gs[grp][u] * (1.0f / 4194304.0f);
            float mu, rho;
            if (P.lam > 0.f) {
                mu = (float)ps[grp][u] * (1.0f / 2048.0f);
                rho = g / P.lam;
            } else {
                mu = 1.0f;
                rho = g * P.Es / P.N0;
            }
            float a = 0.f, c = 0.f;
            if (mu > 0.f && rho > 0.f) {
                a = 1.0f / (mu * P.sqEs * P.qscale);
                c = rho * P.qscale * P.qscale;
            }
            const float t = (float)zv * (1.0f / 2048.0f) * a;
            float *dst = P.llr + ((size_t)v * U + u) * Q + ax * half;
            if (half == 3) axis_llrs<3>(t, c, dst);
            else if (half == 2) axis_llrs<2>(t, c, dst);
            else axis_llrs<1>(t, c, dst);
        }
    }
}

// Channels are staged when the subcarriers a workgroup can touch fit in 32 KB of
// LDS (B = 128, U = 8, S = 14: two subcarriers, 16 KB).
template <int L, int NPL>
static hipError_t launch_fx_t(const FxParams &p, hipStream_t s)
{
    constexpr int G = 256 / L;
    const long nvec = (long)p.W * p.S;
    const dim3 grid((unsigned)((nvec + G - 1) / G));
    const long slots = std::min<long>(G, (G - 1) / p.S + 2);
    const size_t lds = (size_t)slots * p.U * p.B * sizeof(float2);
    if (lds <= 32768)
        hipLaunchKernelGGL((k_forward_fx<L, NPL, true>), grid, dim3(256), lds, s, p);
    else
        hipLaunchKernelGGL((k_forward_fx<L, NPL, false>), grid, dim3(256), 0, s, p);
    return hipGetLastError();
}

// 16 lanes per vector up to B = 128, 32 above: each update is a serial chain (64-bit
// sums across the group, then the narrowing), so with many entries per lane more,
// shorter lanes hide it better (B = 256: 199 -> 154 us per 16,800 vectors at 32
// lanes; B = 64 is faster at 16 lanes, 51 against 63 us).  At B = 128 the columns'
// global-memory round trips made 32 lanes the faster (88 against 84 us); with the
// columns staged in LDS, 16 lanes are (77.5 against 80.1 us, int16 pairs staged).
// At B = 256 32 lanes stay ahead when staged (U = 8, 600 x 14 vectors: 81 against
// 105 us; U = 32, 330 x 14: 229 against 244 us).
static hipError_t launch_fx(const FxParams &p, hipStream_t s)
{
    if (p.B <= 32) return launch_fx_t<16, 2>(p, s);
    if (p.B <= 64) return launch_fx_t<16, 4>(p, s);
    if (p.B <= 128) return launch_fx_t<16, 8>(p, s);
    if (p.B <= 256) return launch_fx_t<32, 8>(p, s);
    if (p.B <= 512) return launch_fx_t<32, 16>(p, s);
    return launch_fx_t<32, 32>(p, s);
}

}  // namespace ocd

extern "C" ocd_status ocd_detect_fixed(const ocd_problem *pb, const int16_t *H, const int16_t *y,
                                       int16_t *z, float *llr, hipStream_t stream)
{
    using namespace ocd;
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    if (!H || !y || (!z && !llr)) return OCD_EINVAL;
    if (pb->mode == OCD_HYBRID) return OCD_EUNSUPPORTED;
    FxParams P;
    P.B = pb->B; P.U = pb->U; P.W = pb->W; P.S = pb->S; P.K = pb->K; P.Q = pb->Q;
    P.box = pb->mode == OCD_BOX;
    P.b = 0;
    while ((1 << P.b) < pb->B) ++P.b;
    const double lam = pb->mode == OCD_MMSE ? (double)pb->N0 / (double)pb->Es : 0.0;
    // alpha = round(lambda 2^22) is an operand of the 36-bit adder beside ||h_u||^2
    const double lam_s = std::floor(lam * 4194304.0 + 0.5);
    if (!(lam_s < 34359738368.0)) return OCD_EINVAL;
    P.lam_q = (long long)lam_s;
    const int M = 1 << (pb->Q / 2);
    const double edge = (double)(M - 1) / std::sqrt(2.0 * (double)(M * M - 1) / 3.0);
    const double beta = pb->beta > 0.f ? (double)pb->beta : edge * std::sqrt((double)pb->Es);
    // c is narrowed to a 16-bit word before the clip, so a bound of 2^15 LSB or
    // more clips nothing: 2^15 stands for all of them
    const double beta_s = std::floor(beta * 2048.0 + 0.5);
    P.beta_fx = beta_s < 32768.0 ? (int)beta_s : 32768;
    if (pb->W == 0) return OCD_OK;
    P.lam = (float)lam;
    P.Es = pb->Es; P.N0 = pb->N0;
    P.sqEs = std::sqrt(pb->Es);
    P.qscale = qam_scale(pb->Q);
    P.H = H; P.y = y; P.z = z; P.llr = llr;
    return launch_fx(P, stream) == hipSuccess ? OCD_OK : OCD_EDEVICE;
}
