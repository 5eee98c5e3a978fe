/*
 * ocd.h -- C ABI of libocd.so: optimized coordinate descent (OCD) soft-output
 * data detection for massive MU-MIMO-OFDM on AMD Instinct MI355X (gfx950).
 *
 * Paper: M. Wu, C. Dick, J. R. Cavallaro, C. Studer, "High-Throughput Data
 * Detection for Massive MU-MIMO-OFDM using Coordinate Descent", arXiv 1611.08779.
 *
 * What is computed.  For every subcarrier w and every OFDM symbol s sharing
 * the channel matrix H_w, the receive vector y_{w,s} (B antennas) is equalised
 * by Algorithm 1 (OCD, Section III-B) in MMSE mode (regulariser N0/Es, no
 * constraint), BOX mode (no regulariser, every real and imaginary part clipped
 * to [-beta, beta], equation eq:projection) or HYBRID mode (both, with one
 * regulariser per sweep).  The K sweeps visit users u = 1..U in order and keep
 * the residual r = y - H z up to date incrementally (equation eq:residual).
 * The soft output is the max-log LLR of equation eq:exactinversellr with
 * Section III-C's approximations mu = d_u^-1 ||h_u||^2 and
 * rho = mu / (1 - mu) (= ||h_u||^2 / lambda_K).  In BOX mode, where that
 * formula gives mu = 1 and an infinite rho, rho = ||h_u||^2 Es / N0 is used.
 * LLR sign: L > 0 favours bit 1.  Constellation: Gray square QAM with Q in
 * {2, 4, 6} bits, unit average energy times Es; per axis the level index m
 * (increasing amplitude) carries the label m ^ (m >> 1), Q/2 bits MSB first,
 * in-phase bits before quadrature bits.
 *
 * Memory.  Every array argument is a DEVICE pointer, allocated, owned and
 * freed by the caller; the library never keeps a pointer after the call
 * returns (except inside a graph built by ocd_detect_jobs, see there), and
 * never allocates device memory itself.  Complex arrays hold interleaved
 * (re, im) pairs: float2 for OCD_STORE_F32, IEEE half pairs for OCD_STORE_F16
 * (inputs H and y only; every output is FP32).  Layouts, C order:
 *   H      [W][U][B]      column h_u of subcarrier w contiguous
 *   y      [W][S][B]
 *   z      [W][S][U]      complex FP32, the equalised estimate z^(K)
 *   z_hist [W][S][K][U]   complex FP32, z^(k) after every sweep k = 1..K
 *   llr    [W][S][U][Q]   FP32
 *   g      [W][U]         FP32, ||h_u||^2
 *   dinv,p [W][Kt][U]     FP32, Kt = K if lambda != NULL else 1
 *   dy     [W][S][B]      complex FP32
 *
 * Execution.  Work is enqueued asynchronously on `stream` (NULL = the default
 * stream of the current device); nothing synchronises the host except where
 * stated.  Calls that overlap on one stream are ordered by the stream.
 *
 * Errors.  Every entry point returns an ocd_status.  Arguments are validated
 * before any device work is enqueued; on OCD_EINVAL or OCD_EUNSUPPORTED
 * nothing was launched and no output was touched.  OCD_EDEVICE reports a HIP
 * runtime error from a launch (outputs are then unspecified).  Nothing throws,
 * aborts or prints across the ABI.
 *
 * Building against it.  The header is C99 as well as C++.  It includes
 * <hip/hip_runtime_api.h> for hipStream_t, which a compiler other than hipcc
 * reads with -D__HIP_PLATFORM_AMD__ -I/opt/rocm/include; link with -locd.
 */
#ifndef OCD_H
#define OCD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OCD_OK = 0,
    OCD_EINVAL = -1,       /* bad shape, scalar or pointer */
    OCD_EUNSUPPORTED = -2, /* valid problem this build does not handle (e.g. LDS too small) */
    OCD_EDEVICE = -3,      /* HIP runtime error */
    OCD_ESCRATCH = -4      /* problem too large for the static scratch of a no-allocation entry point */
} ocd_status;

typedef enum { OCD_MMSE = 0, OCD_BOX = 1, OCD_HYBRID = 2 } ocd_mode;
typedef enum { OCD_STORE_F32 = 0, OCD_STORE_F16 = 1 } ocd_storage;

/* The problem statement (Section II-A and Algorithm 1's inputs).
 *   B        BS antennas (rows of H_w), 1 <= B <= 1024
 *   U        users (columns of H_w), 1 <= U <= min(B, 32)   (run-time limit U <= 32, Section V-A)
 *   W        subcarriers, >= 0
 *   S        OFDM symbols sharing H_w, >= 1
 *   Q        bits per QAM symbol: 2, 4 or 6
 *   K        OCD sweeps, 1 <= K <= 256                       (run-time limit K <= 256, Section V-A)
 *   mode     ocd_mode
 *   storage  ocd_storage of H and y
 *   N0       noise variance per complex receive entry, > 0 (sets the MMSE regulariser
 *            N0/Es and the BOX-mode SINR)
 *   Es       average symbol energy, > 0
 *   beta     box half-width for BOX/HYBRID; <= 0 selects the constellation edge
 *            max Re{a} * sqrt(Es) (Section II-D). Ignored in MMSE mode. */
typedef struct {
    int B, U, W, S, Q, K;
    int mode;
    int storage;
    float N0, Es, beta;
} ocd_problem;

/* Human-readable name of a status code (static string). */
const char *ocd_status_str(int status);

/* Library version, major * 10000 + minor * 100 + patch. */
int ocd_version(void);

/* Algorithm 1 preprocessing: g_u = ||h_u||^2, d_u^-1 = (g_u + lambda_k)^-1 and
 * p_u = d_u^-1 g_u for every subcarrier.
 *   lambda  device [K] per-sweep regulariser, or NULL for the mode's default
 *           (N0/Es in MMSE and HYBRID, 0 in BOX); entries must be >= 0.
 *   g       device [W][U], dinv and p device [W][Kt][U] (Kt = K if lambda else 1).
 * A column with g_u + lambda_k = 0 gets dinv = 0 (that user is never updated). */
ocd_status ocd_preprocess(const ocd_problem *pb, const void *H, const float *lambda,
                          float *g, float *dinv, float *p, hipStream_t stream);

/* Algorithm 1 plus the soft output, fused in one launch.
 *   g, dinv, p  either all NULL (preprocessing fused into the kernel) or all outputs
 *               of ocd_preprocess for the same H and lambda.
 *   z, llr, z_hist  outputs, each may be NULL (not written); z_hist is what
 *               ocd_detect_backward needs.
 * Uses the launch plan cached for this shape (see ocd_autotune), else a heuristic. */
ocd_status ocd_detect(const ocd_problem *pb, const void *H, const void *y, const float *lambda,
                      const float *g, const float *dinv, const float *p,
                      float *z, float *llr, float *z_hist, hipStream_t stream);

/* Bytes of device workspace ocd_detect_backward and ocd_detect_train_bce need for
 * this problem: 256 bytes holding a completion counter, then up to K + 2 partial sums
 * per workgroup. */
size_t ocd_backward_workspace_bytes(const ocd_problem *pb);

/* Adjoint of ocd_detect with respect to the per-sweep regularisers, the box
 * half-width and the receive vectors (H is not differentiated).  The K sweeps
 * are reversed one coordinate update at a time.  Only z_hist is kept from the
 * forward pass, and the residual is never rebuilt: the update computes
 * c = d_u^-1 (h_u^H r + g_u z_u), so dc/dlambda_k = -d_u^-1 c, and c equals the
 * stored z_u' wherever it was not clipped (where it was, its adjoint is zero).
 *   y           the receive vectors of the forward call; not read (the adjoint
 *               depends on y only through z_hist), but must be a valid pointer
 *   z_hist      device [W][S][K][U], written by ocd_detect with the same arguments
 *   dllr        device [W][S][U][Q], dLoss/dLLR
 *   dlambda     device [K]  dLoss/dlambda_k (overwritten)
 *   dbeta       device [1]  dLoss/dbeta (overwritten; 0 in MMSE mode)
 *   dy          device [W][S][B] complex FP32, dLoss/dRe y + j dLoss/dIm y (may be NULL)
 *   workspace   device, >= ocd_backward_workspace_bytes(pb) bytes, 16-byte aligned,
 *               owned by the caller.  Its first 4 bytes are the adjoint's completion
 *               counter: they must be zero before the first call with this workspace
 *               (allocate it zeroed) and every call leaves them zero again, so a
 *               workspace is reused without clearing.  Calls that share a workspace
 *               must not overlap in time (same stream, or ordered by events).
 * dlambda and dbeta are reduced in a fixed order (the last workgroup to finish sums
 * every workgroup's partials in workgroup order): repeated calls give identical bits.
 * Subgradient conventions: a component of z_u' strictly inside (-beta, beta) is
 * unclipped and one at +-beta clipped (c exactly at +-beta, where the projection's
 * derivative is one-sided, has measure zero); the max-log minimisers are the first
 * ones found. */
ocd_status ocd_detect_backward(const ocd_problem *pb, const void *H, const void *y,
                               const float *lambda, const float *z_hist, const float *dllr,
                               float *dlambda, float *dbeta, float *dy,
                               void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ocd_detect_backward for the mean binary cross-entropy of the LLRs against the
 * transmitted bits, with dLoss/dLLR formed inside the adjoint kernel:
 *   loss = mean over the W S U Q bits of softplus(L) - bit L   (P(bit = 1) = sigmoid(L)),
 *   dLoss/dL = (sigmoid(L) - bit) / (W S U Q),
 * L being the max-log LLR of Section III-C of the last sweep's z (z_hist), recomputed (the
 * value ocd_detect writes, up to rounding).  This is the training step's usual loss
 * at one launch fewer and with no dLoss/dLLR array.
 *   bits        device uint8 [W][S][U][Q], 0 or 1, in the LLR layout (MSB of the
 *               I-axis label first, then the Q-axis label)
 * Every other argument, the outputs, the workspace and the conventions are those of
 * ocd_detect_backward; the plan is the one ocd_autotune_backward caches. */
ocd_status ocd_detect_backward_bce(const ocd_problem *pb, const void *H, const void *y,
                                   const float *lambda, const float *z_hist, const uint8_t *bits,
                                   float *dlambda, float *dbeta, float *dy,
                                   void *workspace, size_t workspace_bytes, hipStream_t stream);

/* One training step of the unfolded detector in one launch: Algorithm 1 and the
 * soft output of Section III-C (as ocd_detect), the mean binary cross-entropy of the
 * LLRs against the transmitted bits (as ocd_detect_backward_bce),
 *   loss = mean over the W S U Q bits of softplus(L) - bit L   (P(bit = 1) = sigmoid(L)),
 * and its gradients with respect to the per-sweep regularisers, the box half-width
 * and the receive vectors.  Each workgroup stages its channels once for both passes
 * and keeps every vector's z after each sweep in LDS, so no per-sweep history
 * crosses HBM.  z, the LLRs and dy are those of ocd_detect followed by
 * ocd_detect_backward_bce under the same plan, bit for bit; the loss is summed in a
 * fixed order (repeated calls give identical bits).
 *   bits        device uint8 [W][S][U][Q], 0 or 1, in the LLR layout
 *   z, llr      outputs as in ocd_detect, each may be NULL (not written)
 *   loss        device [1], the mean cross-entropy (overwritten; 0 when W = 0)
 *   dlambda, dbeta, dy, workspace   as in ocd_detect_backward (dy may be NULL)
 * The plan is the one ocd_autotune_train cached for the shape, else the adjoint's
 * (ocd_autotune_backward's cached one, else the heuristic one) with its vectors per
 * workgroup halved until the z history fits in LDS; see ocd_train_plan.  Returns OCD_EINVAL for a NULL loss, dlambda or dbeta, for NULL H, y
 * or bits when W > 0, and for a workspace that is too small or not 16-byte aligned. */
ocd_status ocd_detect_train_bce(const ocd_problem *pb, const void *H, const void *y,
                                const float *lambda, const uint8_t *bits, float *z, float *llr,
                                float *loss, float *dlambda, float *dbeta, float *dy,
                                void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Capacity, per GPU, of the static device scratch of ocd_detect_backward_bce_noalloc. */
#define OCD_NOALLOC_SCRATCH_BYTES (1u << 20)

/* ocd_detect_backward_bce for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving or training loops, harnesses that forbid hipMalloc.
 * The same adjoint and the same kernels, with the completion counter and the
 * per-workgroup partial sums in a static device array of OCD_NOALLOC_SCRATCH_BYTES,
 * which the library holds on every GPU it runs on until the process ends, instead of a
 * caller workspace.  It calls no hipMalloc, hipFree or other allocating routine, and
 * its host side allocates nothing (if OCD_TUNE_CACHE is set, the first plan lookup of
 * the process reads that file: make any other call first where even that is not
 * allowed).
 *   Size limit: 256 + nblocks (K + 1) 4 bytes <= OCD_NOALLOC_SCRATCH_BYTES, where
 *               nblocks = ceil(W S / vectors_per_block) of the adjoint's plan for the
 *               shape (ocd_autotune_backward's cached plan, else the heuristic one).
 *               Larger problems return OCD_ESCRATCH with nothing launched: use
 *               ocd_detect_backward_bce with a workspace.
 *   stream      must belong to the current device (else OCD_EINVAL).
 * Every call on one GPU shares that GPU's scratch, which keeps the last call's partial
 * sums: calls that overlap in time on one GPU (several streams or host threads) race
 * and give wrong gradients, so serialise them.  The counter is zero when the library
 * loads and every call leaves it zero.  Arguments, outputs and conventions are
 * otherwise those of ocd_detect_backward_bce, whose results it reproduces bit for bit
 * under the same plan. */
ocd_status ocd_detect_backward_bce_noalloc(const ocd_problem *pb, const void *H, const void *y,
                                           const float *lambda, const float *z_hist,
                                           const uint8_t *bits, float *dlambda, float *dbeta,
                                           float *dy, hipStream_t stream);

/* A launch plan: how vectors map onto lanes and workgroups.
 *   lanes_per_vector      lanes that share one (subcarrier, symbol) vector: 4, 8, 16 or 32
 *                         (16 or 32 with channel_in_registers)
 *   vectors_per_block     vectors per workgroup: 1..512/lanes_per_vector, or
 *                         1..256/lanes_per_vector with channel_in_registers
 *   xcd_remap             1: consecutive tiles go to the same XCD (shared L2)
 *   channel_in_registers  0: the H_w of every subcarrier a workgroup touches is staged
 *                         once into LDS and shared by its vectors (the choice when many
 *                         symbols share H_w); 1: each vector's lane group keeps the
 *                         columns of its H_w in registers and nothing is staged (the
 *                         choice when few do).  1 needs U <= 8 and
 *                         B <= 8 * lanes_per_vector, and is forward-only.
 *   stagger               0..16: workgroup b waits
 *                         max(0, b / 128 - 1) * stagger * 512 clocks before it loads
 *                         its tile (or its columns, channel_in_registers = 1), so
 *                         that the workgroups dispatched first get their data
 *                         first and start computing while later ones load
 *                         (0: every workgroup loads at once). */
typedef struct {
    int lanes_per_vector;
    int vectors_per_block;
    int xcd_remap;
    int channel_in_registers;
    int stagger;
} ocd_plan;

/* The plan ocd_detect would use for this problem (cached or heuristic). */
ocd_status ocd_get_plan(const ocd_problem *pb, ocd_plan *plan);

/* The launch plan ocd_detect_train_bce takes for this shape (see there). */
ocd_status ocd_train_plan(const ocd_problem *pb, ocd_plan *plan);

/* Force a plan for this problem's shape (B, U, W, S, K, Q, mode, storage), with and
 * without per-sweep regularisers (the backward pass keeps its own choice). */
ocd_status ocd_set_plan(const ocd_problem *pb, const ocd_plan *plan);

/* Autotuner: times every valid plan for this problem on the caller's buffers
 * (outputs are overwritten; z and llr must be non-NULL), after ~20 ms of launches
 * that bring the clocks to their loaded level; then re-times the four fastest,
 * each with stagger 0, 1, 2 and 4, in three interleaved rounds, caches the one
 * with the lowest median for the shape (with and without per-sweep regularisers)
 * and returns it.  Synchronises `stream`.  When the environment
 * variable OCD_TUNE_CACHE names a file, plans are also loaded from and saved
 * to that JSON file, keyed by GPU architecture and shape. */
ocd_status ocd_autotune(const ocd_problem *pb, const void *H, const void *y,
                        float *z, float *llr, int repeats, ocd_plan *best, hipStream_t stream);

/* The same autotuner over 1 <= n <= 65536 input sets: H and y are host arrays of n device
 * pointers (each set laid out as for ocd_detect; the arrays are read during the
 * call only).  Every candidate plan is timed over `repeats` passes through the n
 * sets in order, so that with more sets than the caches hold each launch reads
 * its inputs from HBM, as a stream of distinct slots does; ocd_autotune is the
 * n = 1 case, whose input stays cache-resident between launches and can favour
 * another plan.  z and llr are overwritten.  EINVAL on n outside that range or a NULL
 * pointer. */
ocd_status ocd_autotune_inputs(const ocd_problem *pb, int n, const void *const *H,
                               const void *const *y, float *z, float *llr, int repeats,
                               ocd_plan *best, hipStream_t stream);

/* Autotuner of the training step: times every valid plan of ocd_detect_train_bce
 * (those whose z history fits in LDS, then the staggered staging on the fastest)
 * on the caller's buffers (loss, dlambda, dbeta, dy are overwritten; z and the LLRs
 * are not written; the other arguments are those of ocd_detect_train_bce), caches
 * the fastest for the shape and returns it.  Synchronises `stream`. */
ocd_status ocd_autotune_train(const ocd_problem *pb, const void *H, const void *y,
                              const float *lambda, const uint8_t *bits, float *loss,
                              float *dlambda, float *dbeta, float *dy, void *workspace,
                              size_t workspace_bytes, int repeats, ocd_plan *best,
                              hipStream_t stream);

/* Autotuner of the adjoint: times every valid plan of ocd_detect_backward on the
 * caller's buffers (the outputs dlambda, dbeta, dy are overwritten; the other
 * arguments are those of ocd_detect_backward), caches the fastest for the shape
 * and returns it.  Synchronises `stream`.  Plans with channel_in_registers are
 * forward-only and are not considered. */
ocd_status ocd_autotune_backward(const ocd_problem *pb, const void *H, const void *y,
                                 const float *lambda, const float *z_hist, const float *dllr,
                                 float *dlambda, float *dbeta, float *dy,
                                 void *workspace, size_t workspace_bytes, int repeats,
                                 ocd_plan *best, hipStream_t stream);

/* Batched detection of uneven jobs in one launch.
 * Each job j is a full problem (jobs[j]) with its own device arrays H[j], y[j],
 * z[j] (may be NULL) and llr[j] (may be NULL); every job must use the default
 * regulariser (lambda = NULL), the same storage and the same projection (MMSE,
 * or BOX/HYBRID), and B <= 256.  Jobs are cut into tiles of whole subcarriers,
 * ordered longest-first (LPT), and run by one launch of one kernel: either one
 * workgroup per tile (the hardware dispatcher balances them) or persistent
 * workgroups that pop tiles from a device queue until it is empty.
 *   workspace   device, >= ocd_jobs_workspace_bytes(jobs, n_jobs), 256-byte aligned;
 *               holds the job and tile tables and the queue head.
 *   flags       OCD_JOBS_GRAPH: capture the launch (queue reset and kernel) in a
 *               hipGraph on the first call for this workspace and job list, and
 *               replay it afterwards (job pointers are read from the workspace,
 *               so a change of pointers only re-uploads the tables).
 *               OCD_JOBS_TUNE: before running, time every schedule, tile-size
 *               policy and lane mode on the caller's buffers (outputs are
 *               overwritten; synchronises `stream`), time the fastest three again
 *               in three interleaved rounds, and keep the one with the lowest
 *               median for this list of shapes.
 *               OCD_JOBS_PERSISTENT: use the persistent schedule.
 *               OCD_JOBS_LANE_MODE(m), m = 0, 1, 2: use lane mode m (below)
 *               instead of the tuned one.
 * Lane modes (complex entries per lane, NPL; a job's lanes per vector are B / NPL):
 *   0: NPL = 8 for every job;  1: NPL = 16 for jobs with B > 128, else 8;
 *   2: as 1, and NPL = 4 for jobs with 32 < B <= 128.
 * A job whose (lanes, NPL) pair the kernel is not built for keeps NPL = 8; a job
 * with B <= 16 runs at 4 lanes of 8 entries, the antennas past B zero-padded.
 * When the tables change, the call enqueues a host-to-device copy of them from
 * pinned memory held by the library and first waits for the previous copy from
 * the same workspace, so it may block until earlier work on `stream` consumed
 * it.  Calls that share a workspace must be ordered on one stream. */
#define OCD_JOBS_GRAPH 1
#define OCD_JOBS_TUNE 2
#define OCD_JOBS_PERSISTENT 4
#define OCD_JOBS_LANE_MODE_SHIFT 4
#define OCD_JOBS_LANE_MODE(m) (((m) + 1) << OCD_JOBS_LANE_MODE_SHIFT)
size_t ocd_jobs_workspace_bytes(const ocd_problem *jobs, int n_jobs);
ocd_status ocd_detect_jobs(const ocd_problem *jobs, const void *const *H, const void *const *y,
                           float *const *z, float *const *llr, int n_jobs,
                           void *workspace, size_t workspace_bytes, int flags, hipStream_t stream);

/* The schedule ocd_detect_jobs runs for this list of shapes: the one the last
 * OCD_JOBS_TUNE call chose, else the default (one workgroup per tile, tiles of
 * whole subcarriers, lane mode 0).  Outputs (host): persistent (0 or 1, before the
 * OCD_JOBS_PERSISTENT flag is applied), tile_policy (0: tiles of 512 / L vectors,
 * 1: whole subcarriers, 2: half-size tiles) and lane_mode (above). */
ocd_status ocd_jobs_schedule(const ocd_problem *jobs, int n_jobs, int *persistent,
                             int *tile_policy, int *lane_mode);

/* Explicit MMSE soft-output detection, the baseline that OCD approximates without
 * forming the Gram matrix (Section II-B: regularised Gram matrix and its inverse;
 * Section II-E: exact channel gain and post-equalisation SINR).  Per subcarrier w,
 * with lambda = N0/Es:
 *   G = H_w^H H_w,  A = G + lambda I,  A^-1 (in place, by Gauss-Jordan elimination:
 *   A is Hermitian positive definite, so no pivoting is needed);
 *   mu_u = [A^-1 G]_uu = 1 - lambda [A^-1]_uu,  rho_u = mu_u / (1 - mu_u);
 * and per vector (w, s):
 *   z = A^-1 (H_w^H y),  L_{u,b} = rho_u (min over O_b^0 |x - a|^2 - min over O_b^1 |x - a|^2)
 *   at x = z_u / (mu_u sqrt(Es)) against the unit-energy constellation (the same
 *   sign, labels and layouts as ocd_detect).  A user with an all-zero column gets
 *   z_u = 0 and LLRs 0.
 *   pb          mode must be OCD_MMSE (else OCD_EUNSUPPORTED); K is not used;
 *               B <= 512; FP32 or FP16 storage of H and y as for ocd_detect
 *   H, y        device [W][U][B], [W][S][B] complex, as for ocd_detect
 *   z, llr      device outputs [W][S][U] complex FP32 and [W][S][U][Q] FP32, each
 *               may be NULL (not written), not both
 *   plan        lanes_per_vector 8, 16 or 32 with vectors_per_block
 *               (1..512/lanes_per_vector): lane groups per vector (vector ALUs);
 *               or lanes_per_vector 0 with vectors_per_block 0 or S: one subcarrier
 *               per workgroup, the Gram matrix and the S matched filters as real
 *               matrix products on the FP32 matrix cores (U <= 8, S <= 16).
 *               xcd_remap and stagger honoured; channel_in_registers must be 0.  NULL: lane
 *               groups with whole subcarriers per workgroup where they fit.  OCD_EUNSUPPORTED if the
 *               plan does not fit the problem or its LDS exceeds the device's
 *               per-workgroup limit.
 * Asynchronous on `stream`; no allocation. */
ocd_status ocd_detect_mmse(const ocd_problem *pb, const void *H, const void *y, float *z,
                           float *llr, const ocd_plan *plan, hipStream_t stream);

/* Algorithm 1 in the paper's fixed-point datapath (Section IV-C), for comparison
 * with the floating-point path on the same inputs.  Words are 16-bit with 11
 * fractional bits (Q5.11: value = integer / 2048).  Per vector:
 *   preprocessing  g_u = ||h_u||^2 (exact, Q.22), d_u^-1 = R((g_u + alpha) >> b),
 *                  p_u = d_u^-1 (g_u >> b) narrowed to Q.11, with b = ceil(log2 B) and
 *                  alpha = round(lambda 2^22) (lambda = N0/Es in MMSE mode, 0 in BOX);
 *   each update    c = d_u^-1 ((h_u^H r) >> b) + p_u z_u narrowed to Q.11, clipped to
 *                  +-beta in BOX mode; r <- r - h_u (c - z_u), each entry narrowed;
 * where every narrowing to 16 bits rounds half up and saturates, the inner
 * products are exact sums (the paper's 36-bit adder tree, which they fit when
 * every sum stays within 36 bits), and R is the reciprocal unit: normalise x to
 * [1/2, 1), index a table of round(2^18 / (1 + (i + 1/2)/2048)) with the 11 bits
 * after the leading one, shift back to Q.11.  The shifts by b assume channel
 * entries of unit average power (||h_u||^2 close to B): scale H and y by one
 * factor c and N0 by c^2 to get there, which leaves OCD's estimate unchanged.
 * The soft output is formed in FP32 from the fixed-point z and p (mu = p / 2048 in
 * MMSE mode, 1 in BOX mode; rho = g / lambda, BOX g Es / N0), with ocd_detect's
 * layout and sign.
 *   pb          mode OCD_MMSE or OCD_BOX (OCD_HYBRID: OCD_EUNSUPPORTED); storage is
 *               not used; alpha must be below 2^35 (it shares the 36-bit adder with
 *               g_u), else OCD_EINVAL; beta <= 0 selects the constellation edge,
 *               rounded to Q.11; a beta of 16 or more (beyond the word range) clips
 *               nothing
 *   H, y        device int16 (re, im) pairs, [W][U][B][2] and [W][S][B][2], Q5.11
 *   z           device int16 pairs [W][S][U][2], Q5.11, or NULL
 *   llr         device FP32 [W][S][U][Q], or NULL (not both NULL)
 * Asynchronous on `stream`; no allocation. */
ocd_status ocd_detect_fixed(const ocd_problem *pb, const int16_t *H, const int16_t *y, int16_t *z,
                            float *llr, hipStream_t stream);

/* OFDM demodulation at the base station, the step before detection (Section II-A:
 * after the cyclic prefixes are removed, the time-domain samples of every antenna
 * are transformed back to the frequency domain by a DFT).  For every antenna b
 * and OFDM symbol s:
 *   X[k] = N^-1/2 sum_{n<N} x[b][s][Ncp + n] exp(-2 pi i k n / N)   (unitary DFT)
 *   y[w][s][b] = X[k_w],  k_w = N - W/2 + w for w < W/2 (frequencies -W/2 .. -1),
 *                         k_w = w - W/2 + 1 otherwise (+1 .. +W/2); DC is not used,
 * i.e. y is the detector's receive-vector layout [W][S][B] for ocd_detect.
 *   sh       N in {256, 512, 1024, 2048, 4096}; 0 <= Ncp <= N; W even, 2 <= W and
 *            W/2 < N/2; B, S >= 1 (else OCD_EINVAL)
 *   x        device [B][S][Ncp + N] complex FP32 (interleaved), each symbol's cyclic
 *            prefix first
 *   y        device [W][S][B] complex FP32, overwritten
 * FP32 arithmetic (Stockham FFT, twiddles rounded from double).  B S > 2^30:
 * OCD_EUNSUPPORTED; a failed device query or launch: OCD_EDEVICE.  Asynchronous on
 * `stream`; no allocation. */
typedef struct {
    int B, S;   /* receive antennas, OFDM symbols */
    int N, Ncp; /* DFT size and cyclic-prefix length in samples */
    int W;      /* used subcarriers */
} ocd_ofdm_shape;
ocd_status ocd_ofdm_demodulate(const ocd_ofdm_shape *sh, const float *x, float *y,
                               hipStream_t stream);

/* Measurement support, not part of the detector: launches `blocks` workgroups of
 * 256 threads, each thread running 8 independent FP32 FMA chains for `iters` x 16
 * updates, with packed FP32 instruction selection off like every kernel of this
 * library; *flops receives the launch's flop count (2 per FMA).  Timing it (events
 * on `stream`) gives the non-packed FP32 FMA rate the detection kernels can reach.
 *   out     device, >= 256 floats; written only in a case that never occurs
 * OCD_EINVAL for blocks or iters below 1 or NULL pointers; asynchronous. */
ocd_status ocd_probe_fma(int blocks, int iters, float *out, double *flops, hipStream_t stream);

/* Drops every cached hipGraph and pinned staging buffer (e.g. before freeing a
 * workspace that ocd_detect_jobs captured). */
void ocd_release_graphs(void);

#ifdef __cplusplus
}
#endif

#endif /* OCD_H */
