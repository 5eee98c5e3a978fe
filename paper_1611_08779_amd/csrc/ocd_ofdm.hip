// ocd_ofdm.hip -- OFDM demodulation at the base station, the step before
// detection (Section II-A): per receive antenna and OFDM symbol, drop the cyclic
// prefix, take the unitary N-point DFT, and keep the W used subcarriers (bins
// -W/2 .. -1 and +1 .. +W/2, DC empty), written straight into the detector's
// [W][S][B] layout.
//
// One FFT per N/8 threads, 8 NT / N FFTs per workgroup of NT = 1024, 512 or 256
// threads (the host's choice, by batch size), Stockham
// auto-sort passes of radix 8 (then one of radix 4 or 2 when log2 N is not a
// multiple of 3).  Pass with stride Ns and radix R, butterfly j:
//   k = j mod Ns,  v_r = in[j + r N/R] * w^(r k), w = exp(-2 pi i / (Ns R)),
//   out[(j / Ns) Ns R + k + q Ns] = sum_r v_r exp(-2 pi i r q / R).
// The first pass reads its operands straight from HBM (in[t + r N/8] is the
// time-domain symbol after the prefix); the passes exchange through LDS.  Each
// butterfly takes one twiddle w = exp(-2 pi i k / (Ns R)) from a 4096-entry table
// (built at compile time in double precision, rounded to FP32) and forms
// w^2 .. w^(R-1) by complex products.  A thread's twiddles for all of its passes
// are loaded at the start, with its operands: loaded after each pass's barrier,
// every pass waited for an L2 round trip in the workgroup's serial chain.
//
// Consecutive subcarriers are S B entries apart in y, so one FFT's outputs are
// scattered.  A workgroup holds the FFTs of consecutive antennas of one symbol
// and writes the used bins with the antenna index fastest: contiguous runs of
// 8 F bytes.  Workgroups are mapped so that consecutive antenna blocks of a
// symbol run on the same XCD, whose L2 merges the runs into whole lines before
// they reach HBM.
#include <atomic>
#include <cmath>

#include "ocd.h"
#include "ocd_device.h"

namespace ocd {

// ------------------------------------------------------------------ twiddle table

constexpr int TW_N = 4096;
constexpr double TW_PI = 3.14159265358979323846264338327950288;

// Taylor series of sin and cos about 0, for |x| <= pi (20 terms: the first
// neglected term is below 1e-24)
constexpr double ct_sin(double x)
{
    double term = x, sum = x;
    for (int i = 1; i < 20; ++i) {
        term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        sum += term;
    }
    return sum;
}

constexpr double ct_cos(double x)
{
    double term = 1.0, sum = 1.0;
    for (int i = 1; i < 20; ++i) {
        term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}

struct TwEntry {
    float re, im;
};

struct TwTable {
    TwEntry e[TW_N];
};

// exp(-2 pi i m / 4096), the angle taken in (-pi, pi]
constexpr TwTable make_twiddles()
{
    TwTable t{};
    for (int m = 0; m < TW_N; ++m) {
        const int mm = m <= TW_N / 2 ? m : m - TW_N;
        const double a = 2.0 * TW_PI * (double)mm / (double)TW_N;
        t.e[m].re = (float)ct_cos(a);
        t.e[m].im = (float)-ct_sin(a);
    }
    return t;
}

__device__ const TwTable g_twiddle = make_twiddles();

template <int N>
__device__ __forceinline__ float2 twiddle(int m)   // exp(-2 pi i m / N), 0 <= m < N
{
    const TwEntry t = g_twiddle.e[m * (TW_N / N)];   // one 8-byte load
    return make_float2(t.re, t.im);
}

// ------------------------------------------------------------------ small DFTs

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 mul_neg_i(float2 a) { return make_float2(a.y, -a.x); }

// v_r *= w^r for r = 1 .. R-1, from one table value w (each power one complex
// product away from earlier ones, so the error stays a few FP32 ulps)
template <int R>
__device__ __forceinline__ void twiddle_powers(float2 *v, float2 w)
{
    float2 p[R];
    p[1] = w;
    if constexpr (R > 2) p[2] = cmul(w, w);
    if constexpr (R > 3) p[3] = cmul(p[2], w);
    if constexpr (R > 4) {
        p[4] = cmul(p[2], p[2]);
        p[5] = cmul(p[4], w);
        p[6] = cmul(p[3], p[3]);
        p[7] = cmul(p[6], w);
    }
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], p[r]);
}

// forward DFT of 4 points: X_q = sum_r x_r exp(-2 pi i r q / 4)
__device__ __forceinline__ void dft4(float2 &a, float2 &b, float2 &c, float2 &d)
{
    const float2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = mul_neg_i(csub(b, d));
    a = cadd(t0, t2);
    c = csub(t0, t2);
    b = cadd(t1, t3);
    d = csub(t1, t3);
}

// forward DFT of 8 points: two DFTs of 4 (even, odd inputs) and the W8 twiddles
__device__ __forceinline__ void dft8(float2 (&v)[8])
{
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const float h = 0.70710678118654752440f;
    o1 = make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));    // * exp(-i pi/4)
    o2 = mul_neg_i(o2);                                        // * exp(-i pi/2)
    o3 = make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));   // * exp(-3i pi/4)
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

// ------------------------------------------------------------------ kernel

struct OfdmParams {
    int B, S, N, Ncp, W;
    int xcd_remap;
    float scale;       // N^-1/2
    const float2 *x;   // [B][S][Ncp + N]
    float2 *y;         // [W][S][B]
};

template <int N, int NT>
struct FftShape {
    static constexpr int T = N / 8;        // threads per FFT
    static constexpr int F = NT * 8 / N;   // FFTs per workgroup of NT threads
    static constexpr int LD = N + N / 32 + 8;   // LDS row of one FFT (padded, see lds_index)
    static constexpr int LOG = N == 256 ? 8 : N == 512 ? 9 : N == 1024 ? 10 : N == 2048 ? 11 : 12;
    static constexpr int P8 = LOG / 3;     // radix-8 passes
    static constexpr int REM = LOG % 3;    // last pass: 0 none, 1 radix 2, 2 radix 4
};

// LDS position of element a of an FFT row: one float2 of padding after every 32.
// The Stockham passes write with strides of 8 and 64 elements; unpadded, those
// put 8 or 16 lanes of a wave on the same banks, padded at most 2 (the floor for
// 8-byte accesses).
__device__ __forceinline__ int lds_index(int a) { return a + (a >> 5); }

// Bin of used subcarrier w: -W/2 .. -1 first, then +1 .. +W/2.
__device__ __forceinline__ int used_bin(int N, int W, int w)
{
    return w < (W >> 1) ? N - (W >> 1) + w : w - (W >> 1) + 1;
}

template <int N, int NT>
__global__ __launch_bounds__(NT) void k_ofdm_fft(OfdmParams P)
{
    using Sh = FftShape<N, NT>;
    constexpr int T = Sh::T, F = Sh::F, LD = Sh::LD;
    __shared__ float2 buf[F * LD];
    const int f = threadIdx.x / T, t = threadIdx.x % T;
    const int tile = P.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    // FFT indices s B + b fit an int: the host admits B S <= 2^30
    const int g0 = tile * F;                           // first FFT of the workgroup
    const int nfft = P.S * P.B;
    // FFTs past the end (last workgroup only) transform the last one again and
    // are never written, so no branch separates the loads
    const int g = min(g0 + f, nfft - 1);
    const int s = g / P.B, b = g - s * P.B;
    float2 *sh = buf + f * LD;

    // pass 1 (Ns = 1, no twiddles): operands straight from the time-domain symbol
    const float2 *x = P.x + ((size_t)b * P.S + s) * (P.Ncp + N) + P.Ncp;
    float2 v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = x[t + r * T];
    // the twiddles of every later pass depend only on t: their table loads go out
    // with the operands', so no pass waits on memory after its barrier
    float2 tw8[Sh::P8 > 1 ? Sh::P8 - 1 : 1];
#pragma unroll
    for (int pass = 1, ns = 8; pass < Sh::P8; ++pass, ns *= 8)
        tw8[pass - 1] = twiddle<N>((t & (ns - 1)) * (N / (ns * 8)));
    constexpr int NREM = Sh::REM == 2 ? 2 : Sh::REM == 1 ? 4 : 1;
    float2 twr[NREM];
    if constexpr (Sh::REM != 0) {
#pragma unroll
        for (int h = 0; h < NREM; ++h) twr[h] = twiddle<N>(t + h * T);
    }
    dft8(v);
#pragma unroll
    for (int q = 0; q < 8; ++q) sh[lds_index(8 * t + q)] = v[q];
    int Ns = 8;
    __syncthreads();

    // the other radix-8 passes, in place in LDS (all operands read before a barrier)
#pragma unroll
    for (int pass = 1; pass < Sh::P8; ++pass) {
        const int j = t, k = j & (Ns - 1);
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = sh[lds_index(j + r * T)];
        __syncthreads();
        twiddle_powers<8>(v, tw8[pass - 1]);
        dft8(v);
        const int base = (j / Ns) * Ns * 8 + k;
#pragma unroll
        for (int q = 0; q < 8; ++q) sh[lds_index(base + q * Ns)] = v[q];
        Ns *= 8;
        __syncthreads();
    }

    if constexpr (Sh::REM == 2) {
        // radix-4 last pass, Ns = N/4: butterflies j = t, t + T, in place
        float2 u[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = t + h * T;
#pragma unroll
            for (int r = 0; r < 4; ++r) u[h][r] = sh[lds_index(j + r * (N / 4))];
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = t + h * T;
            twiddle_powers<4>(u[h], twr[h]);
            dft4(u[h][0], u[h][1], u[h][2], u[h][3]);
#pragma unroll
            for (int q = 0; q < 4; ++q) sh[lds_index(j + q * (N / 4))] = u[h][q];
        }
        __syncthreads();
    } else if constexpr (Sh::REM == 1) {
        // radix-2 last pass, Ns = N/2: butterflies j = t + h T (h < 4), in place
        float2 u[4][2];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int j = t + h * T;
            u[h][0] = sh[lds_index(j)];
            u[h][1] = sh[lds_index(j + N / 2)];
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int j = t + h * T;
            twiddle_powers<2>(u[h], twr[h]);
            sh[lds_index(j)] = cadd(u[h][0], u[h][1]);
            sh[lds_index(j + N / 2)] = csub(u[h][0], u[h][1]);
        }
        __syncthreads();
    }
    // (a power-of-8 size ends with its last radix-8 pass, already in natural order)

    // write-out: item i = (w, a), a fastest, so F consecutive antennas of one
    // symbol store one contiguous run of y[w][s][b0 .. b0 + F).  NT is a
    // multiple of F, so every item of a thread has the same a = FFT g0 + a: its
    // (symbol, antenna) and output column are fixed, and only w steps.
    const int W = P.W;
    const int a = threadIdx.x % F, ga = g0 + a;
    if (ga < nfft) {
        const int sa = ga / P.B, ba = ga - sa * P.B;
        const size_t wstride = (size_t)P.S * P.B;      // between subcarriers in y
        const float2 *row = buf + a * LD;
        float2 *yo = P.y + (size_t)sa * P.B + ba;
        for (int w = threadIdx.x / F; w < W; w += NT / F) {
            const float2 X = row[lds_index(used_bin(N, W, w))];
            yo[(size_t)w * wstride] = make_float2(X.x * P.scale, X.y * P.scale);
        }
    }
}

template <int N, int NT>
static hipError_t launch_ofdm_nt(const OfdmParams &p, hipStream_t st)
{
    using Sh = FftShape<N, NT>;
    const long nfft = (long)p.B * p.S;
    const unsigned blocks = (unsigned)((nfft + Sh::F - 1) / Sh::F);
    hipLaunchKernelGGL((k_ofdm_fft<N, NT>), dim3(blocks), dim3(NT), 0, st, p);
    return hipGetLastError();
}

// The largest workgroup whose grid still gives every CU one: a small batch of
// FFTs is spread over more, smaller workgroups (N = 512, B = 64, S = 14 runs in
// 5.2 us at 256 threads against 6.6 us at 1024), a large one keeps the longest
// contiguous output runs.
template <int N>
static hipError_t launch_ofdm_t(const OfdmParams &p, int ncu, hipStream_t st)
{
    const long nfft = (long)p.B * p.S;
    auto blocks_for = [&](int nt) {
        const int F = nt * 8 / N;
        return (nfft + F - 1) / F;
    };
    if (blocks_for(1024) >= ncu) return launch_ofdm_nt<N, 1024>(p, st);
    if constexpr (N <= 2048) {
        if (blocks_for(512) < ncu) return launch_ofdm_nt<N, 256>(p, st);
    }
    return launch_ofdm_nt<N, 512>(p, st);
}

// Compute units of the current device (cached per device; 0 on error).
static int device_cus()
{
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
    if (dev < 64) {
        const int c = cus[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (dev < 64) cus[dev].store(n, std::memory_order_relaxed);
    return n;
}

}  // namespace ocd

extern "C" ocd_status ocd_ofdm_demodulate(const ocd_ofdm_shape *sh, const float *x, float *y,
                                          hipStream_t stream)
{
    using namespace ocd;
    if (!sh || !x || !y) return OCD_EINVAL;
    const int N = sh->N;
    if (N != 256 && N != 512 && N != 1024 && N != 2048 && N != 4096) return OCD_EINVAL;
    if (sh->B < 1 || sh->S < 1 || sh->Ncp < 0 || sh->Ncp > N) return OCD_EINVAL;
    if (sh->W < 2 || sh->W % 2 || sh->W / 2 >= N / 2) return OCD_EINVAL;
    if ((long long)sh->B * sh->S > (1LL << 30)) return OCD_EUNSUPPORTED;
    OfdmParams P;
    P.B = sh->B; P.S = sh->S; P.N = N; P.Ncp = sh->Ncp; P.W = sh->W;
    P.xcd_remap = 1;
    P.scale = (float)(1.0 / std::sqrt((double)N));
    P.x = reinterpret_cast<const float2 *>(x);
    P.y = reinterpret_cast<float2 *>(y);
    const int ncu = device_cus();
    if (ncu <= 0) return OCD_EDEVICE;
    hipError_t e;
    switch (N) {
    case 256: e = launch_ofdm_t<256>(P, ncu, stream); break;
    case 512: e = launch_ofdm_t<512>(P, ncu, stream); break;
    case 1024: e = launch_ofdm_t<1024>(P, ncu, stream); break;
    case 2048: e = launch_ofdm_t<2048>(P, ncu, stream); break;
    default: e = launch_ofdm_t<4096>(P, ncu, stream); break;
    }
    return e == hipSuccess ? OCD_OK : OCD_EDEVICE;
}
