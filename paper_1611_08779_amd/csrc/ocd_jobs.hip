// ocd_jobs.hip -- uneven detection jobs in one persistent launch.
//
// Every job is cut into tiles of consecutive (subcarrier, symbol) vectors.  A
// tile runs exactly the one-problem code (forward_tile) with NPL = 16 complex
// entries per lane, so a job with B antennas uses L = 4, 8, 16 or 32 lanes per
// vector (B <= 16 L): one register footprint serves every job.  Tiles are sorted
// longest-first (LPT) and persistent workgroups pop them from a device counter
// until the queue is empty.  The queue reset and the persistent kernel can be
// captured once into a hipGraph and replayed; the job and tile tables live in
// the caller's workspace and are re-uploaded on every call, so the graph never
// holds a job pointer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ocd_api_internal.h"
#include "ocd_tile.h"

namespace ocd {

constexpr int JOB_NPL = 16;
constexpr int JOB_THREADS = 256;

struct JobDesc {
    Params P;
    int L;
    int pad_[3];
};

struct TileDesc {
    int vbase;
    int job;
    int nvb;
    int pad_;
};

constexpr size_t HEADER_BYTES = 256;

template <bool F16, bool BOX>
__global__ __launch_bounds__(JOB_THREADS) void k_jobs(const JobDesc *jobs, const TileDesc *tiles,
                                                      unsigned int *next, int ntiles)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_tile;
    for (;;) {
        __syncthreads();   // the previous tile is done with LDS and s_tile
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int ti = __builtin_amdgcn_readfirstlane(s_tile);
        if (ti >= ntiles) break;
        const TileDesc td = tiles[ti];
        const JobDesc &jd = jobs[td.job];
        const Params P = jd.P;
        Tile t;
        t.vbase = td.vbase;
        t.nvb = td.nvb;
        t.w_first = td.vbase / P.S;
        t.nslots = (td.vbase + td.nvb - 1) / P.S - t.w_first + 1;
        switch (jd.L) {
        case 4: forward_tile<4, JOB_NPL, F16, BOX>(P, carve(smem, P, JOB_THREADS / 4, false), t); break;
        case 8: forward_tile<8, JOB_NPL, F16, BOX>(P, carve(smem, P, JOB_THREADS / 8, false), t); break;
        case 16: forward_tile<16, JOB_NPL, F16, BOX>(P, carve(smem, P, JOB_THREADS / 16, false), t); break;
        default: forward_tile<32, JOB_NPL, F16, BOX>(P, carve(smem, P, JOB_THREADS / 32, false), t); break;
        }
    }
}

__global__ void k_reset_queue(unsigned int *next) { *next = 0u; }

// ------------------------------------------------------------------ host planning

struct JobsPlan {
    std::vector<JobDesc> jobs;
    std::vector<TileDesc> tiles;
    size_t lds_max = 0;
    bool f16 = false, box = false;
};

// Tile-size policies the batch tuner chooses from:
//   0  every lane group of the workgroup busy (tiles of 256/L vectors)
//   1  tiles of whole subcarriers (a multiple of S vectors), else policy 0
//   2  half-size tiles (more tiles, better balance, less LDS per tile)
constexpr int N_POLICIES = 3;

static int tile_vectors(int policy, int L, int S)
{
    const int cap = JOB_THREADS / L;
    if (policy == 1 && S <= cap) return (cap / S) * S;
    if (policy == 2) return std::max(1, cap / 2);
    return cap;
}

static ocd_status plan_jobs(const ocd_problem *jobs, int n, int policy, JobsPlan &out)
{
    out = JobsPlan();
    if (n < 1 || !jobs) return OCD_EINVAL;
    out.f16 = jobs[0].storage == OCD_STORE_F16;
    out.box = jobs[0].mode != OCD_MMSE;
    for (int j = 0; j < n; ++j) {
        const ocd_problem *pb = &jobs[j];
        ocd_status st = validate(pb);
        if (st != OCD_OK) return st;
        if ((pb->storage == OCD_STORE_F16) != out.f16) return OCD_EINVAL;
        if ((pb->mode != OCD_MMSE) != out.box) return OCD_EINVAL;
        if (pb->B > 16 * 32) return OCD_EUNSUPPORTED;
        int L = 4;
        while (16 * L < pb->B) L *= 2;
        ocd_plan pl = {L, tile_vectors(policy, L, pb->S), 0, 0};
        Params P;
        int npl, threads;
        size_t lds;
        bool ok = false;
        while (pl.vectors_per_block >= 1) {
            if (make_params(pb, pl, nullptr, false, P, npl, threads, lds) && npl == JOB_NPL) {
                // carve() sizes the per-vector z rows for every lane group
                lds = lds_bytes(P, JOB_THREADS / L, false);
                if (lds <= (size_t)lds_limit_bytes()) {
                    ok = true;
                    break;
                }
            }
            pl.vectors_per_block /= 2;
        }
        if (!ok) return OCD_EUNSUPPORTED;
        JobDesc jd;
        std::memset(&jd, 0, sizeof jd);
        jd.P = P;
        jd.L = L;
        out.jobs.push_back(jd);
        out.lds_max = std::max(out.lds_max, lds);
        const long nvec = (long)pb->W * pb->S;
        for (long v = 0; v < nvec; v += P.vpb) {
            TileDesc td;
            td.vbase = (int)v;
            td.job = j;
            td.nvb = (int)std::min<long>(P.vpb, nvec - v);
            td.pad_ = 0;
            out.tiles.push_back(td);
        }
    }
    // longest processing time first: cost ~ vectors x sweeps x users x padded antennas
    auto cost = [&](const TileDesc &t) {
        const Params &P = out.jobs[t.job].P;
        return (double)t.nvb * P.K * P.U * P.Bpad + 4.0 * P.U * P.Bpad;
    };
    std::stable_sort(out.tiles.begin(), out.tiles.end(),
                     [&](const TileDesc &a, const TileDesc &b) { return cost(a) > cost(b); });
    return OCD_OK;
}

static size_t table_bytes(const JobsPlan &jp)
{
    return jp.jobs.size() * sizeof(JobDesc) + jp.tiles.size() * sizeof(TileDesc);
}

// ------------------------------------------------------------------ launch state

struct Staging {
    void *pinned = nullptr;
    size_t bytes = 0;
    hipEvent_t uploaded = nullptr;
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static std::mutex g_mu;
static std::map<void *, Staging> g_staging;
static std::map<std::string, GraphEntry> g_graphs;
static std::map<std::string, int> g_policy;
static hipStream_t g_capture_stream = nullptr;

static int persistent_grid(const JobsPlan &jp, const void *fn)
{
    int dev = 0, ncu = 256, per_cu = 1;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        ncu = prop.multiProcessorCount;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, JOB_THREADS, jp.lds_max) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const long want = (long)ncu * per_cu;
    return (int)std::max<long>(1, std::min<long>(want, (long)jp.tiles.size()));
}

static const void *jobs_kernel(bool f16, bool box)
{
    if (f16) return box ? reinterpret_cast<const void *>(k_jobs<true, true>)
                        : reinterpret_cast<const void *>(k_jobs<true, false>);
    return box ? reinterpret_cast<const void *>(k_jobs<false, true>)
               : reinterpret_cast<const void *>(k_jobs<false, false>);
}

static hipError_t enqueue_jobs(const JobsPlan &jp, unsigned char *ws, int grid, hipStream_t s)
{
    unsigned int *next = reinterpret_cast<unsigned int *>(ws);
    const JobDesc *jobs = reinterpret_cast<const JobDesc *>(ws + HEADER_BYTES);
    const TileDesc *tiles = reinterpret_cast<const TileDesc *>(ws + HEADER_BYTES +
                                                               jp.jobs.size() * sizeof(JobDesc));
    const int ntiles = (int)jp.tiles.size();
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, s, next);
    if (jp.f16) {
        if (jp.box) hipLaunchKernelGGL((k_jobs<true, true>), dim3(grid), dim3(JOB_THREADS), jp.lds_max, s, jobs, tiles, next, ntiles);
        else hipLaunchKernelGGL((k_jobs<true, false>), dim3(grid), dim3(JOB_THREADS), jp.lds_max, s, jobs, tiles, next, ntiles);
    } else {
        if (jp.box) hipLaunchKernelGGL((k_jobs<false, true>), dim3(grid), dim3(JOB_THREADS), jp.lds_max, s, jobs, tiles, next, ntiles);
        else hipLaunchKernelGGL((k_jobs<false, false>), dim3(grid), dim3(JOB_THREADS), jp.lds_max, s, jobs, tiles, next, ntiles);
    }
    return hipGetLastError();
}

// Uploads the tables through the library's pinned buffer for this workspace.
static hipError_t upload_tables(const JobsPlan &jp, unsigned char *ws, hipStream_t s)
{
    const size_t bytes = table_bytes(jp);
    Staging &st = g_staging[ws];
    hipError_t e = hipSuccess;
    if (st.uploaded) {
        e = hipEventSynchronize(st.uploaded);   // the last copy from this buffer is done
        if (e != hipSuccess) return e;
    } else {
        e = hipEventCreateWithFlags(&st.uploaded, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    if (st.bytes < bytes) {
        if (st.pinned) (void)hipHostFree(st.pinned);
        st.pinned = nullptr;
        st.bytes = 0;
        e = hipHostMalloc(&st.pinned, bytes, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        st.bytes = bytes;
    }
    unsigned char *h = static_cast<unsigned char *>(st.pinned);
    std::memcpy(h, jp.jobs.data(), jp.jobs.size() * sizeof(JobDesc));
    std::memcpy(h + jp.jobs.size() * sizeof(JobDesc), jp.tiles.data(),
                jp.tiles.size() * sizeof(TileDesc));
    e = hipMemcpyAsync(ws + HEADER_BYTES, h, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipEventRecord(st.uploaded, s);
}

static void fill_pointers(JobsPlan &jp, const void *const *H, const void *const *y,
                          float *const *z, float *const *llr)
{
    for (size_t j = 0; j < jp.jobs.size(); ++j) {
        Params &P = jp.jobs[j].P;
        P.H = H[j];
        P.y = y[j];
        P.z = z ? reinterpret_cast<float2 *>(z[j]) : nullptr;
        P.llr = llr ? llr[j] : nullptr;
        P.z_hist = nullptr;
        P.lambda = nullptr;
        P.g_in = P.dinv_in = P.p_in = nullptr;
        ocd_problem pb;
        pb.B = P.B;
        pb.storage = jp.f16 ? OCD_STORE_F16 : OCD_STORE_F32;
        set_vec_ok(P, &pb, P.H, P.y);
    }
}

static std::string jobs_hash(const ocd_problem *jobs, int n)
{
    unsigned long long h = 1469598103934665603ULL;
    auto mix = [&](long long v) { h = (h ^ (unsigned long long)v) * 1099511628211ULL; };
    for (int j = 0; j < n; ++j) {
        const ocd_problem &p = jobs[j];
        mix(p.B); mix(p.U); mix(p.W); mix(p.S); mix(p.Q); mix(p.K); mix(p.mode); mix(p.storage);
    }
    char buf[64];
    std::snprintf(buf, sizeof buf, "%016llx|%d", h, n);
    return buf;
}

static ocd_status run_policy(const ocd_problem *jobs, int n, int policy, const void *const *H,
                             const void *const *y, float *const *z, float *const *llr,
                             unsigned char *ws, size_t ws_bytes, bool use_graph, hipStream_t s)
{
    JobsPlan jp;
    ocd_status st = plan_jobs(jobs, n, policy, jp);
    if (st != OCD_OK) return st;
    if (HEADER_BYTES + table_bytes(jp) > ws_bytes) return OCD_EINVAL;
    if (jp.tiles.empty()) return OCD_OK;
    fill_pointers(jp, H, y, z, llr);
    const void *fn = jobs_kernel(jp.f16, jp.box);
    if (jp.lds_max > 65536 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)jp.lds_max) != hipSuccess)
        return OCD_EDEVICE;
    const int grid = persistent_grid(jp, fn);
    if (upload_tables(jp, ws, s) != hipSuccess) return OCD_EDEVICE;
    if (!use_graph) return enqueue_jobs(jp, ws, grid, s) == hipSuccess ? OCD_OK : OCD_EDEVICE;

    char key[256];
    std::snprintf(key, sizeof key, "%p|%zu|%zu|%zu|%d|%d|%d", (void *)ws, jp.jobs.size(),
                  jp.tiles.size(), jp.lds_max, grid, (int)jp.f16, (int)jp.box);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        if (!g_capture_stream &&
            hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking) != hipSuccess)
            return OCD_EDEVICE;
        GraphEntry ge;
        if (hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return OCD_EDEVICE;
        hipError_t e = enqueue_jobs(jp, ws, grid, g_capture_stream);
        hipError_t e2 = hipStreamEndCapture(g_capture_stream, &ge.graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (ge.graph) (void)hipGraphDestroy(ge.graph);
            return OCD_EDEVICE;
        }
        if (hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(ge.graph);
            return OCD_EDEVICE;
        }
        it = g_graphs.emplace(key, ge).first;
    }
    return hipGraphLaunch(it->second.exec, s) == hipSuccess ? OCD_OK : OCD_EDEVICE;
}

}  // namespace ocd

using namespace ocd;

extern "C" size_t ocd_jobs_workspace_bytes(const ocd_problem *jobs, int n_jobs)
{
    size_t best = 0;
    for (int policy = 0; policy < N_POLICIES; ++policy) {
        JobsPlan jp;
        if (plan_jobs(jobs, n_jobs, policy, jp) != OCD_OK) return 0;
        best = std::max(best, HEADER_BYTES + table_bytes(jp));
    }
    return best;
}

extern "C" ocd_status ocd_detect_jobs(const ocd_problem *jobs, const void *const *H,
                                      const void *const *y, float *const *z, float *const *llr,
                                      int n_jobs, void *workspace, size_t workspace_bytes, int flags,
                                      hipStream_t stream)
{
    if (!jobs || n_jobs < 1 || !H || !y || !workspace) return OCD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return OCD_EINVAL;
    for (int j = 0; j < n_jobs; ++j) {
        ocd_status st = validate(&jobs[j]);
        if (st != OCD_OK) return st;
        if (jobs[j].W > 0 && (!H[j] || !y[j])) return OCD_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    const std::string hk = jobs_hash(jobs, n_jobs);
    int policy = 1;
    auto pit = g_policy.find(hk);
    if (pit != g_policy.end()) policy = pit->second;
    if (flags & OCD_JOBS_TUNE) {
        // batch tuner: time every tile policy on the caller's buffers
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return OCD_EDEVICE;
        if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return OCD_EDEVICE; }
        float best_ms = 1e30f;
        int best = policy;
        for (int pol = 0; pol < N_POLICIES; ++pol) {
            ocd_status st = run_policy(jobs, n_jobs, pol, H, y, z, llr, ws, workspace_bytes, false, stream);
            if (st != OCD_OK) continue;
            (void)hipEventRecord(e0, stream);
            for (int rep = 0; rep < 3 && st == OCD_OK; ++rep)
                st = run_policy(jobs, n_jobs, pol, H, y, z, llr, ws, workspace_bytes, false, stream);
            (void)hipEventRecord(e1, stream);
            if (st != OCD_OK || hipEventSynchronize(e1) != hipSuccess) continue;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) { best_ms = ms; best = pol; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        policy = best;
        g_policy[hk] = policy;
    }
    return run_policy(jobs, n_jobs, policy, H, y, z, llr, ws, workspace_bytes,
                      (flags & OCD_JOBS_GRAPH) != 0, stream);
}

extern "C" void ocd_release_graphs(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    g_graphs.clear();
    for (auto &kv : g_staging) {
        if (kv.second.uploaded) {
            (void)hipEventSynchronize(kv.second.uploaded);
            (void)hipEventDestroy(kv.second.uploaded);
        }
        if (kv.second.pinned) (void)hipHostFree(kv.second.pinned);
    }
    g_staging.clear();
}
