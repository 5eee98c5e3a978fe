// ocd_internal.h -- launch parameters shared by the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ocd {

// Everything a forward or backward launch needs, by value.
struct Params {
    int B, U, W, S, K, Q;
    int box;         // projection onto the box is active (BOX, HYBRID)
    int per_sweep;   // a per-sweep regulariser array was given: dinv, p are [Kt = K][U]
    int Bpad;        // L * NPL >= B
    int vpb;         // vectors per workgroup
    int maxslots;    // LDS slots for distinct subcarriers per workgroup
    int slot_stride; // float2 elements between slots (padded)
    int xcd_remap;
    int vec_ok;      // vector loads allowed (B even, 16-byte aligned bases)
    int nblocks;
    int reg_uc;      // channel-in-registers plans: compile-time bound on U (else 0)
    int stagger;     // staged loads: sleep units per 128 workgroups (see stagger_loads)
    int stagger_cap; // workgroups resident at once: later ones start late anyway
    float Es, N0, beta;
    float lam_default;   // regulariser when lambda == nullptr
    float sqEs;          // sqrt(Es)
    float qscale;        // level spacing of the unit-energy square QAM
    float invU;          // 1 / U (slot of a staged H row without an integer divide)
    unsigned divS_m;     // n / S = divide_invariant(n, divS_m, divS_s1, divS_s2) (see
    int divS_s1, divS_s2;// set_divisor): exact, with no integer divide on the GPU
    const float *lambda; // device [K] or nullptr
    const void *H;       // [W][U][B] complex (FP32 or FP16 pairs)
    const void *y;       // [W][S][B]
    const float *g_in;   // [W][U] or nullptr (then preprocessing is fused)
    const float *dinv_in;// [W][Kt][U]
    const float *p_in;   // [W][Kt][U]
    float2 *z;           // [W][S][U] or nullptr
    float *llr;          // [W][S][U][Q] or nullptr
    float2 *z_hist;      // [W][S][K][U] or nullptr
    // backward only
    const float2 *zh_in; // [W][S][K][U]
    const float *dllr;   // [W][S][U][Q], or nullptr when bits is given
    const unsigned char *bits;  // [W][S][U][Q] 0/1, or nullptr: the adjoint forms
                                // dLoss/dLLR itself for the mean BCE of the LLRs
    float inv_nbits;     // 1 / (W S U Q), with bits
    float2 *dy;          // [W][S][B] or nullptr
    float *partials;     // [nblocks][K + 1] (adjoint), [nblocks][K + 2] (training step)
    unsigned *ticket;    // completion ticket of the adjoint's workgroups (zero between launches)
    float *dlambda;      // [K] adjoint output
    float *dbeta;        // [1] adjoint output
    float *loss;         // [1] training step: mean cross-entropy of the LLRs, or nullptr
};

// Unsigned 32-bit division by a divisor d fixed for a launch, as a multiply-high,
// an add and two shifts (Granlund and Montgomery, "Division by invariant integers
// using multiplication", 1994, the round-up method for all 32-bit dividends):
// with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
//   t = mulhi(m, n),  n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0).
inline void set_divisor(unsigned d, unsigned &m, int &s1, int &s2)
{
    int l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    m = (unsigned)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
    s1 = l < 1 ? l : 1;
    s2 = l > 1 ? l - 1 : 0;
}

__host__ __device__ inline unsigned divide_invariant(unsigned n, unsigned m, int s1, int s2)
{
    const unsigned t = (unsigned)(((unsigned long long)m * n) >> 32);
    return (t + ((n - t) >> s1)) >> s2;
}

// Compute units of the current device (cached per device; 0 on error).
int device_cu_count();

// Bytes of dynamic LDS a launch of this shape needs (train: the fused training
// step, which also keeps every vector's K rows of z history and one more partial).
inline size_t lds_bytes(const Params &p, int vpb_cap, bool backward, int nwaves = 0,
                        bool train = false)
{
    const int Kt = p.per_sweep ? p.K : 1;
    size_t b = 0;
    b += (size_t)p.maxslots * p.slot_stride * 8;     // H slots (FP32 complex)
    b += (size_t)p.maxslots * p.U * 4;               // g
    b = (b + 7) & ~(size_t)7;
    b += (size_t)p.maxslots * Kt * p.U * 8;          // (dinv, p) pairs
    b += (size_t)p.maxslots * p.U * 8;               // soft-output coefficients
    b += (size_t)(p.vpb + 1) * p.U * 8;              // z per vector (+ idle groups' row)
    if (backward) {
        b += (size_t)(p.vpb + 1) * p.U * 8;          // z_bar per vector
        b += (size_t)(p.K + 2) * (size_t)nwaves * 4; // per-wave partials (sweeps, beta, loss)
    }
    if (train) b += (size_t)(p.vpb + 1) * p.K * p.U * 8;   // z^(k) rows per vector
    return b;
}

// Bytes of dynamic LDS of an explicit-MMSE launch: staged H_w, two U x U work
// matrices and the soft-output coefficients per slot, a matched-filter row per
// vector and the Gram diagonal per slot.
inline size_t mmse_lds_bytes(const Params &p)
{
    size_t b = (size_t)p.maxslots * p.slot_stride * 8;
    b += (size_t)p.maxslots * 2 * p.U * p.U * 8;
    b += (size_t)p.maxslots * p.U * 8;
    b += (size_t)p.vpb * p.U * 8;
    b += (size_t)p.maxslots * p.U * 4;
    return b;
}

// A launch with at most two waves per SIMD (the grid's waves over 4 SIMDs per CU)
// has no other waves to hide a wave's latencies behind: the unrolled sweeps then
// prefetch their operands one update ahead.
inline bool latency_bound(const Params &p, int threads)
{
    const int cus = device_cu_count();
    return cus > 0 && (long)p.nblocks * (threads / 64) <= 2L * 4 * cus;
}

// Launchers (one per template instantiation, selected at run time).
hipError_t launch_forward(int L, int NPL, bool f16, const Params &p, int threads, size_t lds,
                          hipStream_t s);
hipError_t launch_backward(int L, int NPL, bool f16, const Params &p, int threads, size_t lds,
                           hipStream_t s);
hipError_t launch_forward_reg(int L, int NPL, int UC, bool f16, const Params &p,
                              int threads, hipStream_t s);
hipError_t launch_mmse(int L, int NPL, bool f16, const Params &p, int threads, size_t lds,
                       hipStream_t s);
hipError_t launch_mmse_mfma(bool f16, const Params &p, size_t lds, hipStream_t s);
size_t mmse_mfma_lds_bytes(int Kp, int U, int S);
hipError_t launch_preprocess(bool f16, const Params &p, float *g, float *dinv, float *pp,
                             hipStream_t s);
hipError_t launch_reduce_partials(const Params &p, float *dlambda, float *dbeta, float *loss,
                                  hipStream_t s);
hipError_t launch_train(int L, int NPL, bool f16, const Params &p, int threads, size_t lds,
                        hipStream_t s);

}  // namespace ocd
