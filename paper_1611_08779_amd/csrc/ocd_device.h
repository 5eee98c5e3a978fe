// ocd_device.h -- device-side building blocks of the OCD detector (gfx950).
//
// A (subcarrier, symbol) vector is owned by a group of L consecutive lanes of
// one wavefront.  Lane j of the group holds NPL of the B receive entries,
// in chunks of CH consecutive antennas: entry i of the lane is antenna
//   b = CH * (j + L * (i / CH)) + i % CH
// so that a group reads whole contiguous rows of y and of the H columns.
// Antennas b >= B are zero padding (they add nothing to any inner product
// and are never updated).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace ocd {

// ------------------------------------------------------------------ layout

template <int NPL, bool F16>
struct Layout {
    // complex entries per contiguous chunk of one lane
    static constexpr int CH = NPL < 2 ? NPL : 2;
    static constexpr int NCH = NPL / CH;
};

__device__ __forceinline__ int lane_antenna(int j, int i, int L, int CH)
{
    return CH * (j + L * (i / CH)) + i % CH;
}

// ------------------------------------------------------------------ cross-lane sums

// DPP control words (GFX9 encoding).
enum : int {
    DPP_QUAD_XOR1 = 0xB1,  // quad_perm [1,0,3,2]
    DPP_QUAD_XOR2 = 0x4E,  // quad_perm [2,3,0,1]
    DPP_ROW_MIRROR = 0x140,
    DPP_ROW_HALF_MIRROR = 0x141,
};

template <int CTRL>
__device__ __forceinline__ float dpp_get(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Sum over the L lanes of an aligned group; every lane of the group receives
// the same bits (each level adds a commutative pair).  L <= 16 stays in DPP
// row operations; 32 and 64 add a swizzle / permute across rows.
template <int L>
__device__ __forceinline__ float group_sum(float x)
{
    if constexpr (L >= 2) x += dpp_get<DPP_QUAD_XOR1>(x);
    if constexpr (L >= 4) x += dpp_get<DPP_QUAD_XOR2>(x);
    if constexpr (L >= 8) x += dpp_get<DPP_ROW_HALF_MIRROR>(x);
    if constexpr (L >= 16) x += dpp_get<DPP_ROW_MIRROR>(x);
    if constexpr (L >= 32)  // lane ^ 16 within 32 lanes: ds_swizzle bit-mask mode
        x += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x401F));
    if constexpr (L >= 64) {
        int src = (static_cast<int>(__lane_id()) ^ 32) << 2;
        x += __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(x)));
    }
    return x;
}

// group_sum of two values, level by level: each DPP add reads a register written
// two instructions earlier, so the two chains cover each other's DPP read
// hazard.  The scheduling barriers keep the levels interleaved (left alone, the
// scheduler runs one chain after the other and pads each level with wait states).
template <int L>
__device__ __forceinline__ float2 group_sum2(float2 v)
{
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (L >= 2) {
        v.x += dpp_get<DPP_QUAD_XOR1>(v.x);
        v.y += dpp_get<DPP_QUAD_XOR1>(v.y);
    }
    if constexpr (L >= 4) {
        v.x += dpp_get<DPP_QUAD_XOR2>(v.x);
        v.y += dpp_get<DPP_QUAD_XOR2>(v.y);
    }
    if constexpr (L >= 8) {
        v.x += dpp_get<DPP_ROW_HALF_MIRROR>(v.x);
        v.y += dpp_get<DPP_ROW_HALF_MIRROR>(v.y);
    }
    if constexpr (L >= 16) {
        v.x += dpp_get<DPP_ROW_MIRROR>(v.x);
        v.y += dpp_get<DPP_ROW_MIRROR>(v.y);
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (L >= 32) {
        v.x += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v.x), 0x401F));
        v.y += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v.y), 0x401F));
    }
    if constexpr (L >= 64) {
        const int src = (static_cast<int>(__lane_id()) ^ 32) << 2;
        v.x += __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v.x)));
        v.y += __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v.y)));
    }
    return v;
}

// Full-wavefront sum (64 lanes), identical in every lane.
__device__ __forceinline__ float wave_sum(float x) { return group_sum<64>(x); }

// ------------------------------------------------------------------ loads

__device__ __forceinline__ float2 half2_to_float2(uint32_t bits)
{
    __half2 h = *reinterpret_cast<const __half2 *>(&bits);
    return __half22float2(h);
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

// A caller's device buffer as a global-address-space pointer.  Kernels that read
// their buffer pointers from memory (the batched kernel's job table) would
// otherwise address them as generic (FLAT) pointers, whose loads and stores also
// count against the LDS wait counter: every LDS wait would then wait for the
// global accesses in flight as well.  Only ever applied to the caller's buffers.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *global_ptr(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// One complex FP32 entry of a caller's buffer, loaded or stored through the global
// address space (as a plain two-float vector: the float2 class type cannot be
// accessed through an address-space-qualified pointer).
typedef float f32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 global_load2(const float2 *p)
{
    const f32x2_t q = *global_ptr(reinterpret_cast<const f32x2_t *>(p));
    return make_float2(q.x, q.y);
}

__device__ __forceinline__ void global_store2(float2 *p, float2 v)
{
    f32x2_t q;
    q.x = v.x;
    q.y = v.y;
    *global_ptr(reinterpret_cast<f32x2_t *>(p)) = q;
}

// Two consecutive complex entries at element e (aligned: e even), FP32 out.
// No branch: the caller passes an address that is always valid and selects.
template <bool F16>
__device__ __forceinline__ float4 load_pair(const void *base, long e)
{
    if constexpr (!F16) {
        const f32x4_t q = __builtin_nontemporal_load(global_ptr(
            reinterpret_cast<const f32x4_t *>(reinterpret_cast<const float2 *>(base) + e)));
        return make_float4(q.x, q.y, q.z, q.w);
    } else {
        const u32x2_t q = __builtin_nontemporal_load(global_ptr(
            reinterpret_cast<const u32x2_t *>(reinterpret_cast<const uint32_t *>(base) + e)));
        const float2 a = half2_to_float2(q.x), b = half2_to_float2(q.y);
        return make_float4(a.x, a.y, b.x, b.y);
    }
}

// Bytes per complex entry in storage.
template <bool F16>
__device__ __forceinline__ constexpr unsigned cbytes() { return F16 ? 4u : 8u; }

// Two consecutive complex entries at byte offset `off` from a workgroup-uniform
// base: the address is a scalar base plus a 32-bit lane offset.
template <bool F16>
__device__ __forceinline__ float4 load_pair_at(const unsigned char *base, unsigned off)
{
    if constexpr (!F16) {
        const f32x4_t q =
            __builtin_nontemporal_load(global_ptr(reinterpret_cast<const f32x4_t *>(base + off)));
        return make_float4(q.x, q.y, q.z, q.w);
    } else {
        const u32x2_t q =
            __builtin_nontemporal_load(global_ptr(reinterpret_cast<const u32x2_t *>(base + off)));
        const float2 a = half2_to_float2(q.x), b = half2_to_float2(q.y);
        return make_float4(a.x, a.y, b.x, b.y);
    }
}

// FP16 storage: two consecutive complex entries as they are stored (two packed
// half pairs), from a workgroup-uniform base plus a 32-bit byte offset.
__device__ __forceinline__ u32x2_t load_pair_raw16(const unsigned char *base, unsigned off)
{
    return __builtin_nontemporal_load(global_ptr(reinterpret_cast<const u32x2_t *>(base + off)));
}

// Load `N` consecutive complex entries starting at element `e` of a row,
// converting to FP32; entries at or beyond `limit` read as zero.  General
// (branchy) path, used where vector loads are not allowed.

template <bool F16, int N>
__device__ __forceinline__ void load_chunk(const void *base, long e, int b, int limit, bool vec_ok,
                                           float2 *out)
{
    if (vec_ok && b + N <= limit) {
        if constexpr (!F16) {
            const float2 *p = reinterpret_cast<const float2 *>(base) + e;
            if constexpr (N == 2) {
                f32x4_t q =
                    __builtin_nontemporal_load(global_ptr(reinterpret_cast<const f32x4_t *>(p)));
                out[0] = make_float2(q.x, q.y);
                out[1] = make_float2(q.z, q.w);
            } else {
                for (int t = 0; t < N; ++t) out[t] = global_load2(p + t);
            }
        } else {
            const auto p = global_ptr(reinterpret_cast<const uint32_t *>(base) + e);
            if constexpr (N == 2) {
                u32x2_t q = __builtin_nontemporal_load(
                    reinterpret_cast<const __attribute__((address_space(1))) u32x2_t *>(p));
                out[0] = half2_to_float2(q.x);
                out[1] = half2_to_float2(q.y);
            } else {
                for (int t = 0; t < N; ++t) out[t] = half2_to_float2(p[t]);
            }
        }
        return;
    }
    for (int t = 0; t < N; ++t) {
        if (b + t < limit) {
            if constexpr (!F16) out[t] = global_load2(reinterpret_cast<const float2 *>(base) + e + t);
            else out[t] = half2_to_float2(global_ptr(reinterpret_cast<const uint32_t *>(base))[e + t]);
        } else {
            out[t] = make_float2(0.f, 0.f);
        }
    }
}

// ------------------------------------------------------------------ soft output

// Max-log LLRs of one axis of Gray square QAM (HALF = Q/2 bits per axis):
// L_b = rho * (min over levels whose label bit b is 0 of (x - A)^2
//            - min over levels whose label bit b is 1 of (x - A)^2).
// Levels A_m = (2m - M + 1) * scale, label of level m = m ^ (m >> 1), MSB first.
// For a product constellation the other axis' minimum is common to both sets
// and cancels, so this equals the two-dimensional minimum of the definition.
template <int HALF>
__device__ __forceinline__ void axis_llr(float xc, float scale, float rho, float *out)
{
    constexpr int M = 1 << HALF;
    float d[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float e = xc - (float)(2 * m - M + 1) * scale;
        d[m] = e * e;
    }
#pragma unroll
    for (int bb = 0; bb < HALF; ++bb) {
        float d0 = INFINITY, d1 = INFINITY;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int bit = ((m ^ (m >> 1)) >> (HALF - 1 - bb)) & 1;
            if (bit) d1 = fminf(d1, d[m]);
            else d0 = fminf(d0, d[m]);
        }
        out[bb] = rho * (d0 - d1);
    }
}

// The same metrics in closed form, t = xc / scale (levels at the odd integers
// of [-(M-1), M-1]), D_b = min over bit b = 0 of (t - A)^2 - min over bit b = 1.
//
// MSB: the label bit is 1 exactly for the positive levels.  For t >= 0 the
// nearest negative level is -1 and the nearest positive one is the odd integer
// n nearest to t clamped to [1, M-1], so D = (t+1)^2 - (t-n)^2 = (n+1)(2t+1-n);
// D is odd in t.  Every further bit of the reflected Gray label takes the same
// value on A and -A, so its two minima depend on |t| only; about the centre M/2
// of the positive half its levels form an M/2-PAM whose labels are those of an
// M/2-PAM with the MSB inverted.  Hence D_1 = -msb_{M/2}(|t| - M/2) and each
// further bit folds once more.
template <int M>
__device__ __forceinline__ float pam_msb_metric(float t)
{
    const float u = fabsf(t);
    float e;
    if constexpr (M == 2) {
        e = 4.0f * u;
    } else {
        const float n = fminf(fmaxf(fmaf(2.0f, floorf(0.5f * u), 1.0f), 1.0f), (float)(M - 1));
        e = (n + 1.0f) * fmaf(2.0f, u, 1.0f - n);
    }
    return copysignf(e, t);
}

template <int HALF>
__device__ __forceinline__ void pam_metrics(float t, float *D)
{
    constexpr int M = 1 << HALF;
    D[0] = pam_msb_metric<M>(t);
    if constexpr (HALF >= 2) {
        const float w1 = fabsf(t) - (float)(M / 2);
        D[1] = -pam_msb_metric<M / 2>(w1);
        if constexpr (HALF >= 3) {
            const float w2 = fabsf(w1) - (float)(M / 4);
            D[2] = -pam_msb_metric<M / 4>(w2);
        }
    }
}

// Index of the level nearest to xc among the two minimisers used for bit bb
// (first minimiser in level order on ties); returns the adjoint factor
// dD/dxc = 2 (A_{m1} - A_{m0}) for D = (xc - A_{m0})^2 - (xc - A_{m1})^2.
template <int HALF>
__device__ __forceinline__ float axis_llr_slope(float xc, float scale, int bb)
{
    constexpr int M = 1 << HALF;
    float d0 = INFINITY, d1 = INFINITY;
    int m0 = 0, m1 = 0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float e = xc - (float)(2 * m - M + 1) * scale;
        float dm = e * e;
        const int bit = ((m ^ (m >> 1)) >> (HALF - 1 - bb)) & 1;
        if (bit) {
            if (dm < d1) { d1 = dm; m1 = m; }
        } else {
            if (dm < d0) { d0 = dm; m0 = m; }
        }
    }
    return 2.0f * (float)(2 * (m1 - m0)) * scale;
}

// Square-QAM level spacing for unit average energy: 1 / sqrt(2 (M^2 - 1) / 3).
__host__ __device__ inline float qam_scale(int Q)
{
    const int M = 1 << (Q / 2);
    return 1.0f / sqrtf(2.0f * (float)(M * M - 1) / 3.0f);
}

// ------------------------------------------------------------------ block mapping

// Permutes block ids so that consecutive tiles land on the same XCD (blocks are
// dispatched round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ int xcd_tile(int bx, int nblocks)
{
    const int q = nblocks >> 3, r = nblocks & 7;
    const int xcd = bx & 7, idx = bx >> 3;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

}  // namespace ocd
