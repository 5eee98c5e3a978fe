// ocd_probe.hip -- measurement support: the FP32 FMA issue rate the GPU reaches.
//
// Every thread runs 8 independent FMA chains (x <- x a + b), 16 updates per chain
// per iteration, so each wave always has an independent FMA to issue and a SIMD with
// a few waves issues one VALU FMA per cycle.  Built like every other kernel here
// (packed FP32 instruction selection off), it measures the non-packed FP32 rate the
// detection kernels can reach, against which their VALU fraction is read.  The
// result is written only if it equals a value it never takes, so the chains stay
// live without a store per thread.
#include "ocd.h"
#include "ocd_internal.h"

namespace ocd {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_CHAINS = 8;
constexpr int PROBE_UNROLL = 16;

__global__ __launch_bounds__(PROBE_THREADS) void k_fma_rate(float *out, int iters, float a, float b)
{
    float x[PROBE_CHAINS];
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; ++i) x[i] = (float)threadIdx.x * 1e-3f + (float)i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < PROBE_UNROLL; ++r)
#pragma unroll
            for (int i = 0; i < PROBE_CHAINS; ++i) x[i] = fmaf(x[i], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; ++i) s += x[i];
    if (s == -1.0f) out[blockIdx.x & 255] = s;
}

}  // namespace ocd

extern "C" ocd_status ocd_probe_fma(int blocks, int iters, float *out, double *flops,
                                    hipStream_t stream)
{
    if (blocks < 1 || iters < 1 || !out || !flops) return OCD_EINVAL;
    *flops = 2.0 * (double)blocks * ocd::PROBE_THREADS * (double)iters * ocd::PROBE_UNROLL *
             ocd::PROBE_CHAINS;
    // a = 1 - 2^-20, b = 2^-10: every chain converges towards b / (1 - a) = 1024
    // without overflow or denormals, whatever the iteration count
    hipLaunchKernelGGL(ocd::k_fma_rate, dim3(blocks), dim3(ocd::PROBE_THREADS), 0, stream, out,
                       iters, 1.0f - 9.5367431640625e-7f, 9.765625e-4f);
    return hipGetLastError() == hipSuccess ? OCD_OK : OCD_EDEVICE;
}
