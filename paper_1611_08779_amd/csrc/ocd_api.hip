// ocd_api.hip -- the C ABI of libocd.so: argument validation, launch plans
// (heuristic, cache, autotuner) and the launches of the forward, preprocessing
// and adjoint kernels.  Batched jobs live in ocd_jobs.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <string_view>
#include <vector>

#include "../../include/ocd.h"
#include "ocd_api_internal.h"
#include "ocd_device.h"
#include "ocd_internal.h"

using namespace ocd;

// ------------------------------------------------------------------ status

extern "C" const char *ocd_status_str(int status)
{
    switch (status) {
    case OCD_OK: return "OCD_OK";
    case OCD_EINVAL: return "OCD_EINVAL: invalid argument";
    case OCD_EUNSUPPORTED: return "OCD_EUNSUPPORTED: problem not supported by this build";
    case OCD_EDEVICE: return "OCD_EDEVICE: HIP runtime error";
    case OCD_ESCRATCH:
        return "OCD_ESCRATCH: problem too large for the static scratch of the no-allocation "
               "entry point (use the workspace form)";
    default: return "unknown ocd_status";
    }
}

extern "C" int ocd_version(void) { return 10100; }

// ------------------------------------------------------------------ validation

namespace ocd {

static bool finite_pos(float x) { return std::isfinite(x) && x > 0.f; }

ocd_status validate(const ocd_problem *pb)
{
    if (!pb) return OCD_EINVAL;
    if (pb->B < 1 || pb->B > 1024) return OCD_EINVAL;
    if (pb->U < 1 || pb->U > 32 || pb->U > pb->B) return OCD_EINVAL;
    if (pb->W < 0 || pb->S < 1) return OCD_EINVAL;
    if (pb->Q != 2 && pb->Q != 4 && pb->Q != 6) return OCD_EINVAL;
    if (pb->K < 1 || pb->K > 256) return OCD_EINVAL;
    if (pb->mode != OCD_MMSE && pb->mode != OCD_BOX && pb->mode != OCD_HYBRID) return OCD_EINVAL;
    if (pb->storage != OCD_STORE_F32 && pb->storage != OCD_STORE_F16) return OCD_EINVAL;
    if (!finite_pos(pb->N0) || !finite_pos(pb->Es) || !std::isfinite(pb->beta)) return OCD_EINVAL;
    if ((long long)pb->W * pb->S > (1LL << 30)) return OCD_EUNSUPPORTED;
    return OCD_OK;
}

int lds_limit_bytes()
{
    static int limit = -1;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    if (limit < 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            limit = (int)prop.sharedMemPerBlock;
        else
            limit = 65536;
    }
    return limit;
}

// gfx architecture of the current device, queried once per device into a static
// table, so that a lookup never allocates.
const char *arch_name()
{
    static std::mutex mu;
    static char names[MAX_DEVICES][32];
    static bool known[MAX_DEVICES];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return "unknown";
    std::lock_guard<std::mutex> lk(mu);
    if (!known[dev]) {
        hipDeviceProp_t prop;
        std::snprintf(names[dev], sizeof names[dev], "unknown");
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            std::snprintf(names[dev], sizeof names[dev], "%s", prop.gcnArchName);
            if (char *c = std::strchr(names[dev], ':')) *c = 0;
        }
        known[dev] = true;
    }
    return names[dev];
}

int device_cu_count()
{
    static std::mutex mu;
    static int cus[MAX_DEVICES];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return 0;
    std::lock_guard<std::mutex> lk(mu);
    if (cus[dev] <= 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cus[dev] = n;
    }
    return cus[dev];
}

float box_edge(int Q)
{
    const int M = 1 << (Q / 2);
    return (float)(M - 1) * qam_scale(Q);
}

// Complex entries per lane for a group of L lanes: the smallest power of two
// >= B / L, at least 2; 0 if above 32.
int npl_for(int B, int L)
{
    int n = 2;
    while (n * L < B) n *= 2;
    return n <= 32 ? n : 0;
}

// Fills the launch parameters of a (problem, plan) pair; false if the plan is
// not valid for the problem (group too small for B, LDS too small, ...).
// Channel-in-registers plans: the compile-time bound on U the kernel is built
// for (8), 0 if the problem does not fit (U <= 8 and at most 64 complex entries
// of H_w per lane, so that everything stays in registers).
static int reg_user_bound(int U, int npl)
{
    return (U <= 8 && npl <= 8) ? 8 : 0;
}

bool make_params(const ocd_problem *pb, const ocd_plan &pl, const float *lambda, bool backward,
                 Params &P, int &npl, int &threads, size_t &lds, int min_npl)
{
    const int L = pl.lanes_per_vector;
    if (L != 4 && L != 8 && L != 16 && L != 32) return false;
    npl = npl_for(pb->B, L);
    if (!npl) return false;
    if (npl < min_npl) npl = min_npl;   // more zero-padded entries per lane than B needs
    if (pl.channel_in_registers < 0 || pl.channel_in_registers > 1) return false;
    if (pl.stagger < 0 || pl.stagger > 16) return false;
    const bool reg = pl.channel_in_registers != 0;
    if (reg && (backward || (L != 16 && L != 32) || !reg_user_bound(pb->U, npl))) return false;
    const int cap = (reg ? 256 : 512) / L;
    if (pl.vectors_per_block < 1 || pl.vectors_per_block > cap) return false;
    std::memset(&P, 0, sizeof(P));
    P.B = pb->B; P.U = pb->U; P.W = pb->W; P.S = pb->S; P.K = pb->K; P.Q = pb->Q;
    P.box = pb->mode != OCD_MMSE;
    P.per_sweep = lambda != nullptr;
    P.Bpad = L * npl;
    P.vpb = pl.vectors_per_block;
    if (P.vpb % P.S == 0) P.maxslots = P.vpb / P.S;
    else P.maxslots = std::min(P.vpb, (P.vpb - 1) / P.S + 2);
    const int row = P.U * P.Bpad;             // float2 per slot, before padding
    P.slot_stride = row + ((row % 16 == 0) ? 8 : (16 - row % 16 + 8) % 16);
    P.xcd_remap = pl.xcd_remap ? 1 : 0;
    P.stagger = pl.stagger;
    P.Es = pb->Es; P.N0 = pb->N0;
    P.beta = pb->beta > 0.f ? pb->beta : box_edge(pb->Q) * std::sqrt(pb->Es);
    P.lam_default = pb->mode == OCD_BOX ? 0.f : pb->N0 / pb->Es;
    P.sqEs = std::sqrt(pb->Es);
    P.qscale = qam_scale(pb->Q);
    P.invU = 1.0f / (float)pb->U;
    set_divisor((unsigned)pb->S, P.divS_m, P.divS_s1, P.divS_s2);
    P.lambda = lambda;
    const long nvec = (long)pb->W * pb->S;
    P.nblocks = (int)((nvec + P.vpb - 1) / P.vpb);
    const int waves = (P.vpb * L + 63) / 64;
    threads = waves * 64;
    if (reg) {
        P.reg_uc = reg_user_bound(pb->U, npl);
        P.maxslots = 0;
        lds = 0;
        return true;
    }
    lds = lds_bytes(P, threads / L, backward, threads / 64);
    return lds <= (size_t)lds_limit_bytes();
}

// Rough occupancy model used by the heuristic: lanes doing useful work per CU.
static double plan_score(const ocd_problem *pb, const ocd_plan &pl, const Params &P, int npl,
                         int threads, size_t lds)
{
    const int lds_cu = 160 * 1024;
    const int vgpr = 4 * npl + 40;
    const int waves_simd = std::max(1, std::min(8, 512 / vgpr));
    const int blocks_lds = (int)std::max<size_t>(1, lds_cu / std::max<size_t>(lds, 1));
    const int blocks_thr = std::max(1, (4 * waves_simd * 64) / threads);
    const int blocks = std::min(blocks_lds, blocks_thr);
    double useful = (double)P.vpb * pl.lanes_per_vector / threads;     // idle groups
    double eff = (double)pb->B / P.Bpad;                               // zero padding
    return blocks * threads * useful * eff;
}

ocd_plan heuristic_plan(const ocd_problem *pb, const float *lambda, bool backward, bool allow_reg)
{
    if (allow_reg && !backward && pb->S <= 2) {
        // a channel shared by at most two vectors: nothing to reuse from LDS
        for (int L : {16, 32}) {
            ocd_plan pl = {L, 256 / L, 0, 1};
            Params P;
            int npl, threads;
            size_t lds;
            if (make_params(pb, pl, lambda, backward, P, npl, threads, lds)) return pl;
        }
    }
    int L = 4;
    while (L < 32 && L * 16 < pb->B) L *= 2;
    ocd_plan best = {L, 1, 0, 0};
    double best_score = -1;
    const int cap = 512 / L;
    int cands[160];   // at most 8 powers of two and 128 multiples of S
    int nc = 0;
    for (int v = cap; v >= 1; v /= 2) cands[nc++] = v;
    for (int m = pb->S; m <= cap; m += pb->S) cands[nc++] = m;
    for (int i = 0; i < nc; ++i) {
        const int v = cands[i];
        ocd_plan pl = {L, v, 0, 0};
        Params P;
        int npl, threads;
        size_t lds;
        if (!make_params(pb, pl, lambda, backward, P, npl, threads, lds)) continue;
        double s = plan_score(pb, pl, P, npl, threads, lds);
        if (s > best_score * 1.02 || (s > best_score * 0.98 && v > best.vectors_per_block)) {
            best_score = std::max(s, best_score);
            best = pl;
        }
    }
    return best;
}

// ------------------------------------------------------------------ plan cache

static std::mutex g_plan_mu;
static std::map<std::string, ocd_plan, std::less<>> g_plans;   // lookups take a string_view
static bool g_plans_loaded = false;

PlanKey plan_key_dir(const ocd_problem *pb, bool per_sweep, const char *dir)
{
    PlanKey k;
    std::snprintf(k.s, sizeof k.s, "%s|%s|B%d|U%d|W%d|S%d|K%d|Q%d|m%d|s%d|l%d", arch_name(), dir,
                  pb->B, pb->U, pb->W, pb->S, pb->K, pb->Q, pb->mode, pb->storage,
                  per_sweep ? 1 : 0);
    return k;
}

PlanKey plan_key(const ocd_problem *pb, bool per_sweep, bool backward)
{
    return plan_key_dir(pb, per_sweep, backward ? "bwd" : "fwd");
}

static void load_plan_file_locked()
{
    if (g_plans_loaded) return;
    g_plans_loaded = true;
    const char *path = std::getenv("OCD_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char key[256];
        ocd_plan pl = {0, 0, 0, 0, 0};
        const int n = std::sscanf(line, " {\"key\": \"%255[^\"]\", \"lanes_per_vector\": %d, "
                                        "\"vectors_per_block\": %d, \"xcd_remap\": %d, "
                                        "\"channel_in_registers\": %d, \"stagger\": %d",
                                  key, &pl.lanes_per_vector, &pl.vectors_per_block, &pl.xcd_remap,
                                  &pl.channel_in_registers, &pl.stagger);
        if (n >= 5) g_plans[key] = pl;   // files written before the stagger field: 0
    }
    std::fclose(f);
}

static void save_plan_file_locked()
{
    const char *path = std::getenv("OCD_TUNE_CACHE");
    if (!path || !*path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (auto &kv : g_plans)
        std::fprintf(f, "{\"key\": \"%s\", \"lanes_per_vector\": %d, \"vectors_per_block\": %d, "
                        "\"xcd_remap\": %d, \"channel_in_registers\": %d, \"stagger\": %d}\n",
                     kv.first.c_str(), kv.second.lanes_per_vector, kv.second.vectors_per_block,
                     kv.second.xcd_remap, kv.second.channel_in_registers, kv.second.stagger);
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

bool cached_plan(const PlanKey &key, ocd_plan &pl)
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    load_plan_file_locked();
    auto it = g_plans.find(std::string_view(key.s));
    if (it == g_plans.end()) return false;
    pl = it->second;
    return true;
}

void store_plan(const PlanKey &key, const ocd_plan &pl, bool persist)
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    load_plan_file_locked();
    g_plans[std::string(key.s)] = pl;
    if (persist) save_plan_file_locked();
}

ocd_plan choose_plan(const ocd_problem *pb, const float *lambda, bool backward)
{
    ocd_plan pl;
    if (cached_plan(plan_key(pb, lambda != nullptr, backward), pl)) {
        Params P;
        int npl, threads;
        size_t lds;
        if (make_params(pb, pl, lambda, backward, P, npl, threads, lds)) return pl;
    }
    return heuristic_plan(pb, lambda, backward, true);
}

static bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

void set_vec_ok(Params &P, const ocd_problem *pb, const void *H, const void *y)
{
    const size_t a = pb->storage == OCD_STORE_F16 ? 8 : 16;
    P.vec_ok = (pb->B % 2 == 0) && aligned(H, a) && (y == nullptr || aligned(y, a));
}

}  // namespace ocd

// ------------------------------------------------------------------ preprocessing

extern "C" ocd_status ocd_preprocess(const ocd_problem *pb, const void *H, const float *lambda,
                                     float *g, float *dinv, float *p, hipStream_t stream)
{
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    if (pb->W == 0) return OCD_OK;
    if (!H || !g || !dinv || !p) return OCD_EINVAL;
    Params P;
    std::memset(&P, 0, sizeof P);
    P.B = pb->B; P.U = pb->U; P.W = pb->W; P.S = pb->S; P.K = pb->K; P.Q = pb->Q;
    P.per_sweep = lambda != nullptr;
    P.lam_default = pb->mode == OCD_BOX ? 0.f : pb->N0 / pb->Es;
    P.lambda = lambda;
    P.H = H;
    set_vec_ok(P, pb, H, nullptr);
    hipError_t e = launch_preprocess(pb->storage == OCD_STORE_F16, P, g, dinv, p, stream);
    return e == hipSuccess ? OCD_OK : OCD_EDEVICE;
}

// ------------------------------------------------------------------ forward

namespace ocd {

ocd_status run_forward(const ocd_problem *pb, const ocd_plan &pl, const void *H, const void *y,
                       const float *lambda, const float *g, const float *dinv, const float *p,
                       float *z, float *llr, float *z_hist, hipStream_t stream)
{
    Params P;
    int npl, threads;
    size_t lds;
    if (!make_params(pb, pl, lambda, false, P, npl, threads, lds)) return OCD_EUNSUPPORTED;
    P.H = H; P.y = y;
    P.g_in = g; P.dinv_in = dinv; P.p_in = p;
    P.z = reinterpret_cast<float2 *>(z);
    P.llr = llr;
    P.z_hist = reinterpret_cast<float2 *>(z_hist);
    set_vec_ok(P, pb, H, y);
    if (pl.channel_in_registers && (!P.vec_ok || g)) {
        // the register kernel takes aligned rows of even length and fuses the
        // preprocessing: anything else runs an LDS-staged plan
        return run_forward(pb, heuristic_plan(pb, lambda, false, false), H, y, lambda, g, dinv, p,
                           z, llr, z_hist, stream);
    }
    const bool f16 = pb->storage == OCD_STORE_F16;
    hipError_t e = pl.channel_in_registers
                       ? launch_forward_reg(pl.lanes_per_vector, npl, P.reg_uc, f16, P, threads,
                                            stream)
                       : launch_forward(pl.lanes_per_vector, npl, f16, P, threads, lds, stream);
    return e == hipSuccess ? OCD_OK : OCD_EDEVICE;
}

}  // namespace ocd

extern "C" ocd_status ocd_detect(const ocd_problem *pb, const void *H, const void *y,
                                 const float *lambda, const float *g, const float *dinv,
                                 const float *p, float *z, float *llr, float *z_hist,
                                 hipStream_t stream)
{
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    const int given = (g != nullptr) + (dinv != nullptr) + (p != nullptr);
    if (given != 0 && given != 3) return OCD_EINVAL;
    if (pb->W == 0) return OCD_OK;
    if (!H || !y) return OCD_EINVAL;
    const ocd_plan pl = choose_plan(pb, lambda, false);
    return run_forward(pb, pl, H, y, lambda, g, dinv, p, z, llr, z_hist, stream);
}

// ------------------------------------------------------------------ explicit MMSE

namespace ocd {

// Launch parameters of an explicit-MMSE plan; false if the plan does not fit.
static bool make_mmse_params(const ocd_problem *pb, const ocd_plan &pl, Params &P, int &npl,
                             int &threads, size_t &lds)
{
    const int L = pl.lanes_per_vector;
    if ((L != 8 && L != 16 && L != 32) || pl.channel_in_registers != 0) return false;
    if (!make_params(pb, pl, nullptr, false, P, npl, threads, lds) || npl > 16) return false;
    lds = mmse_lds_bytes(P);
    return lds <= (size_t)lds_limit_bytes();
}

// The matrix-core kernel (plan lanes_per_vector = 0): one subcarrier per
// workgroup, U <= 8, S <= 16, B rounded up to a multiple of 4 antennas.
static bool make_mmse_mfma_params(const ocd_problem *pb, const ocd_plan &pl, Params &P,
                                  size_t &lds)
{
    if (pl.lanes_per_vector != 0 || pl.channel_in_registers != 0) return false;
    if (pb->U > 8 || pb->S > 16) return false;
    if (pl.vectors_per_block != 0 && pl.vectors_per_block != pb->S) return false;
    if (pl.stagger < 0 || pl.stagger > 16) return false;
    std::memset(&P, 0, sizeof(P));
    P.B = pb->B; P.U = pb->U; P.W = pb->W; P.S = pb->S; P.K = pb->K; P.Q = pb->Q;
    P.Bpad = (pb->B + 3) / 4 * 4;
    P.vpb = pb->S;
    P.maxslots = 1;
    P.nblocks = pb->W;
    P.xcd_remap = pl.xcd_remap ? 1 : 0;
    P.stagger = pl.stagger;
    P.Es = pb->Es; P.N0 = pb->N0;
    P.lam_default = pb->N0 / pb->Es;
    P.sqEs = std::sqrt(pb->Es);
    P.qscale = qam_scale(pb->Q);
    P.invU = 1.0f / (float)pb->U;
    set_divisor((unsigned)pb->S, P.divS_m, P.divS_s1, P.divS_s2);
    lds = mmse_mfma_lds_bytes(P.Bpad, pb->U, pb->S);
    return lds <= (size_t)lds_limit_bytes();
}

// Whole subcarriers per workgroup where they fit in 256 threads, with at most 8
// entries of a column per lane; fewer vectors while the LDS does not fit.  (The
// matrix-core form is not chosen by default: both forms are bound by the latency
// of their per-subcarrier chain, and the vector form measured faster.)
static ocd_plan mmse_heuristic_plan(const ocd_problem *pb)
{
    int L = 8;
    while (L < 32 && !(npl_for(pb->B, L) > 0 && npl_for(pb->B, L) <= 8)) L *= 2;
    const int cap = 256 / L;
    int v = pb->S <= cap ? (cap / pb->S) * pb->S : cap;
    ocd_plan pl = {L, v, 0, 0};
    Params P;
    int npl, threads;
    size_t lds;
    while (pl.vectors_per_block > 1 && !make_mmse_params(pb, pl, P, npl, threads, lds))
        pl.vectors_per_block = pl.vectors_per_block > pb->S && pl.vectors_per_block % pb->S == 0
                                   ? pl.vectors_per_block - pb->S
                                   : pl.vectors_per_block / 2;
    return pl;
}

}  // namespace ocd

extern "C" ocd_status ocd_detect_mmse(const ocd_problem *pb, const void *H, const void *y,
                                      float *z, float *llr, const ocd_plan *plan,
                                      hipStream_t stream)
{
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    if (!H || !y || (!z && !llr)) return OCD_EINVAL;
    if (pb->mode != OCD_MMSE || pb->B > 512) return OCD_EUNSUPPORTED;
    const ocd_plan pl = plan ? *plan : mmse_heuristic_plan(pb);
    Params P;
    int npl, threads;
    size_t lds;
    if (pl.lanes_per_vector == 0) {
        if (!make_mmse_mfma_params(pb, pl, P, lds)) return OCD_EUNSUPPORTED;
        if (pb->W == 0) return OCD_OK;
        P.H = H;
        P.y = y;
        P.z = reinterpret_cast<float2 *>(z);
        P.llr = llr;
        const hipError_t e = launch_mmse_mfma(pb->storage == OCD_STORE_F16, P, lds, stream);
        return e == hipSuccess ? OCD_OK : OCD_EDEVICE;
    }
    if (!make_mmse_params(pb, pl, P, npl, threads, lds)) return OCD_EUNSUPPORTED;
    if (pb->W == 0) return OCD_OK;
    P.H = H;
    P.y = y;
    P.z = reinterpret_cast<float2 *>(z);
    P.llr = llr;
    set_vec_ok(P, pb, H, y);
    const hipError_t e = launch_mmse(pl.lanes_per_vector, npl, pb->storage == OCD_STORE_F16, P,
                                     threads, lds, stream);
    return e == hipSuccess ? OCD_OK : OCD_EDEVICE;
}

extern "C" ocd_status ocd_get_plan(const ocd_problem *pb, ocd_plan *plan)
{
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    if (!plan) return OCD_EINVAL;
    *plan = choose_plan(pb, nullptr, false);
    return OCD_OK;
}

extern "C" ocd_status ocd_set_plan(const ocd_problem *pb, const ocd_plan *plan)
{
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    if (!plan) return OCD_EINVAL;
    Params P;
    int npl, threads;
    size_t lds;
    if (!make_params(pb, *plan, nullptr, false, P, npl, threads, lds)) return OCD_EUNSUPPORTED;
    store_plan(plan_key(pb, false, false), *plan, false);
    store_plan(plan_key(pb, true, false), *plan, false);
    return OCD_OK;
}

// The forward autotuner over n input sets: each candidate is timed over `repeats`
// passes through all n sets (H[i], y[i]), so that with more sets than the caches
// hold every launch reads its inputs from HBM, as a stream of distinct slots does.
static ocd_status autotune_forward(const ocd_problem *pb, int n, const void *const *H,
                                   const void *const *y, float *z, float *llr, int repeats,
                                   ocd_plan *best, hipStream_t stream)
{
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    if (n < 1 || n > 65536 || !H || !y || !z || !llr || !best) return OCD_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!H[i] || !y[i]) return OCD_EINVAL;
    if (pb->W == 0) {
        *best = heuristic_plan(pb, nullptr, false, true);
        return OCD_OK;
    }
    repeats = std::max(1, std::min(repeats, 100));
    std::vector<ocd_plan> cands;
    for (int L : {4, 8, 16, 32}) {
        const int cap = 512 / L;
        std::vector<int> vs;
        for (int v = cap; v >= 1 && v >= cap / 16; v /= 2) vs.push_back(v);
        if (pb->S > 1)   // whole subcarriers per workgroup: one LDS slot per subcarrier
            for (int m = pb->S; m <= cap && m <= 4 * pb->S; m += pb->S) vs.push_back(m);
        std::sort(vs.begin(), vs.end());
        vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
        for (int v : vs)
            for (int x : {0, 1}) {
                ocd_plan pl = {L, v, x, 0};
                Params P;
                int npl, threads;
                size_t lds;
                if (make_params(pb, pl, nullptr, false, P, npl, threads, lds)) cands.push_back(pl);
            }
    }
    for (int L : {16, 32}) {   // channel columns in registers (no LDS)
        for (int v = 256 / L; v >= 1 && v >= 64 / L; v /= 2) {
            ocd_plan pl = {L, v, 0, 1};
            Params P;
            int npl, threads;
            size_t lds;
            if (make_params(pb, pl, nullptr, false, P, npl, threads, lds)) cands.push_back(pl);
        }
    }
    if (cands.empty()) return OCD_EUNSUPPORTED;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return OCD_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return OCD_EDEVICE; }
    st = OCD_OK;
    const int launches = repeats * n;
    auto launch = [&](const ocd_plan &pl, int i) {
        return run_forward(pb, pl, H[i % n], y[i % n], nullptr, nullptr, nullptr, nullptr, z, llr,
                           nullptr, stream);
    };
    // one timed pass of a plan over the inputs in turn (ms; < 0 on a device error)
    auto time_plan = [&](const ocd_plan &pl) -> float {
        (void)hipEventRecord(e0, stream);
        for (int i = 0; i < launches && st == OCD_OK; ++i) st = launch(pl, i);
        (void)hipEventRecord(e1, stream);
        if (st != OCD_OK || hipEventSynchronize(e1) != hipSuccess) {
            st = OCD_EDEVICE;
            return -1.f;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    // The clocks settle over the first milliseconds of load: a plan timed then
    // would look slower than it is.  Run the first candidate for ~20 ms first.
    {
        float warm = 0.f;
        for (int r = 0; r < 64 && warm < 20.f && st == OCD_OK; ++r) {
            const float ms = time_plan(cands[0]);
            if (ms >= 0.f) warm += ms;
        }
    }
    // first stage: every candidate once, to rank them
    std::vector<std::pair<float, int>> ranked;
    for (size_t c = 0; c < cands.size() && st == OCD_OK; ++c) {
        st = launch(cands[c], n - 1);
        if (st != OCD_OK) break;
        const float ms = time_plan(cands[c]);
        if (ms >= 0.f) ranked.push_back({ms, (int)c});
    }
    // second stage: the fastest four, each also with staggered starts, timed in
    // three interleaved rounds; the lowest median wins.  Near-equal plans are
    // common (a few percent apart), and one timing each picks among them by noise.
    ocd_plan best_pl = cands[0];
    if (st == OCD_OK && !ranked.empty()) {
        std::sort(ranked.begin(), ranked.end());
        std::vector<ocd_plan> fin;
        for (size_t r = 0; r < ranked.size() && r < 4; ++r)
            for (int sg : {0, 1, 2, 4}) {
                ocd_plan pl = cands[ranked[r].second];
                pl.stagger = sg;
                fin.push_back(pl);
            }
        constexpr int ROUNDS = 3;
        std::vector<float> t(fin.size() * ROUNDS, 0.f);
        for (int rd = 0; rd < ROUNDS && st == OCD_OK; ++rd)
            for (size_t k = 0; k < fin.size() && st == OCD_OK; ++k) {
                // alternate the order, so that no plan is always timed right after another
                const size_t f = rd % 2 ? fin.size() - 1 - k : k;
                t[f * ROUNDS + rd] = time_plan(fin[f]);
            }
        float best_med = 1e30f;
        for (size_t f = 0; f < fin.size() && st == OCD_OK; ++f) {
            float *v = &t[f * ROUNDS];
            std::sort(v, v + ROUNDS);
            if (v[ROUNDS / 2] < best_med) { best_med = v[ROUNDS / 2]; best_pl = fin[f]; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != OCD_OK) return st;
    // the same kernels run with and without per-sweep regularisers (only the
    // preprocessing table is longer): the plan serves both
    store_plan(plan_key(pb, false, false), best_pl, true);
    store_plan(plan_key(pb, true, false), best_pl, true);
    *best = best_pl;
    return OCD_OK;
}

extern "C" ocd_status ocd_autotune(const ocd_problem *pb, const void *H, const void *y, float *z,
                                   float *llr, int repeats, ocd_plan *best, hipStream_t stream)
{
    return autotune_forward(pb, 1, &H, &y, z, llr, repeats, best, stream);
}

extern "C" ocd_status ocd_autotune_inputs(const ocd_problem *pb, int n, const void *const *H,
                                          const void *const *y, float *z, float *llr, int repeats,
                                          ocd_plan *best, hipStream_t stream)
{
    return autotune_forward(pb, n, H, y, z, llr, repeats, best, stream);
}

// ------------------------------------------------------------------ adjoint

extern "C" size_t ocd_backward_workspace_bytes(const ocd_problem *pb)
{
    if (validate(pb) != OCD_OK) return 0;
    // the completion ticket (256 bytes), then the block partials of
    // (dlambda_1..K, dbeta, loss) for the plan with the most blocks
    const long nvec = (long)pb->W * pb->S;
    return 256 + (size_t)std::max(1L, nvec) * (size_t)(pb->K + 2) * sizeof(float);
}

namespace ocd {

// dllr_or_bits: the dLoss/dLLR array or the bits of the fused cross-entropy
static ocd_status check_backward_args(const ocd_problem *pb, const void *H, const void *y,
                                      const float *z_hist, const void *dllr_or_bits,
                                      float *dlambda, float *dbeta, void *workspace,
                                      size_t workspace_bytes)
{
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    if (!dlambda || !dbeta) return OCD_EINVAL;
    if (pb->W > 0 && (!H || !y || !z_hist || !dllr_or_bits)) return OCD_EINVAL;
    if (workspace_bytes < ocd_backward_workspace_bytes(pb) || !workspace) return OCD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return OCD_EINVAL;
    return OCD_OK;
}

// dLoss/dLLR from dllr, or (dllr null) formed in the kernel from bits for the mean
// binary cross-entropy of the LLRs
static ocd_status run_backward(const ocd_problem *pb, const ocd_plan &pl, const void *H,
                               const void *y, const float *lambda, const float *z_hist,
                               const float *dllr, float *dlambda, float *dbeta, float *dy,
                               void *workspace, hipStream_t stream,
                               const unsigned char *bits = nullptr)
{
    Params P;
    int npl, threads;
    size_t lds;
    if (!make_params(pb, pl, lambda, true, P, npl, threads, lds)) return OCD_EUNSUPPORTED;
    P.H = H; P.y = y;
    P.zh_in = reinterpret_cast<const float2 *>(z_hist);
    P.dllr = dllr;
    P.bits = dllr ? nullptr : bits;
    P.inv_nbits = (float)(1.0 / ((double)pb->W * pb->S * pb->U * pb->Q));
    P.dy = reinterpret_cast<float2 *>(dy);
    // workspace: the completion ticket in the first 256 bytes, then the partials
    P.ticket = reinterpret_cast<unsigned *>(workspace);
    P.partials = reinterpret_cast<float *>(static_cast<unsigned char *>(workspace) + 256);
    P.dlambda = dlambda;
    P.dbeta = dbeta;
    set_vec_ok(P, pb, H, y);
    hipError_t e;
    if (pb->W > 0) {
        e = launch_backward(pl.lanes_per_vector, npl, pb->storage == OCD_STORE_F16, P, threads,
                            lds, stream);
    } else {
        P.nblocks = 0;   // no workgroups: zero gradients
        e = launch_reduce_partials(P, dlambda, dbeta, nullptr, stream);
    }
    return e == hipSuccess ? OCD_OK : OCD_EDEVICE;
}

}  // namespace ocd

extern "C" ocd_status ocd_detect_backward(const ocd_problem *pb, const void *H, const void *y,
                                          const float *lambda, const float *z_hist,
                                          const float *dllr, float *dlambda, float *dbeta,
                                          float *dy, void *workspace, size_t workspace_bytes,
                                          hipStream_t stream)
{
    ocd_status st = check_backward_args(pb, H, y, z_hist, dllr, dlambda, dbeta, workspace,
                                        workspace_bytes);
    if (st != OCD_OK) return st;
    return run_backward(pb, choose_plan(pb, lambda, true), H, y, lambda, z_hist, dllr, dlambda,
                        dbeta, dy, workspace, stream);
}

extern "C" ocd_status ocd_detect_backward_bce(const ocd_problem *pb, const void *H, const void *y,
                                              const float *lambda, const float *z_hist,
                                              const uint8_t *bits, float *dlambda, float *dbeta,
                                              float *dy, void *workspace, size_t workspace_bytes,
                                              hipStream_t stream)
{
    ocd_status st = check_backward_args(pb, H, y, z_hist, bits, dlambda, dbeta, workspace,
                                        workspace_bytes);
    if (st != OCD_OK) return st;
    return run_backward(pb, choose_plan(pb, lambda, true), H, y, lambda, z_hist, nullptr, dlambda,
                        dbeta, dy, workspace, stream, bits);
}

// ------------------------------------------------------------------ training step

namespace ocd {

// Parameters of a training-step launch of plan pl: the adjoint's, with each
// vector's K rows of z history in LDS as well; false if that does not fit.
static bool train_params(const ocd_problem *pb, const ocd_plan &pl, const float *lambda, Params &P,
                         int &npl, int &threads, size_t &lds)
{
    if (!make_params(pb, pl, lambda, true, P, npl, threads, lds)) return false;
    lds = lds_bytes(P, threads / pl.lanes_per_vector, true, threads / 64, true);
    return lds <= (size_t)lds_limit_bytes();
}

// The training step's plan: the one ocd_autotune_train cached for the shape, else
// the adjoint's with its vectors per workgroup halved until the z history fits.
static bool choose_train_params(const ocd_problem *pb, const float *lambda, Params &P, int &npl,
                                int &threads, size_t &lds, ocd_plan *used)
{
    ocd_plan pl;
    if (cached_plan(plan_key_dir(pb, lambda != nullptr, "trn"), pl) &&
        train_params(pb, pl, lambda, P, npl, threads, lds)) {
        if (used) *used = pl;
        return true;
    }
    pl = choose_plan(pb, lambda, true);
    for (;;) {
        if (train_params(pb, pl, lambda, P, npl, threads, lds)) {
            if (used) *used = pl;
            return true;
        }
        if (pl.vectors_per_block <= 1) return false;
        pl.vectors_per_block /= 2;
    }
}

}  // namespace ocd

extern "C" ocd_status ocd_train_plan(const ocd_problem *pb, ocd_plan *plan)
{
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    if (!plan) return OCD_EINVAL;
    Params P;
    int npl, threads;
    size_t lds;
    if (!choose_train_params(pb, nullptr, P, npl, threads, lds, plan)) return OCD_EUNSUPPORTED;
    return OCD_OK;
}

namespace ocd {

static ocd_status check_train_args(const ocd_problem *pb, const void *H, const void *y,
                                   const uint8_t *bits, float *loss, float *dlambda, float *dbeta,
                                   void *workspace, size_t workspace_bytes)
{
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    if (!loss || !dlambda || !dbeta) return OCD_EINVAL;
    if (pb->W > 0 && (!H || !y || !bits)) return OCD_EINVAL;
    if (workspace_bytes < ocd_backward_workspace_bytes(pb) || !workspace) return OCD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return OCD_EINVAL;
    return OCD_OK;
}

// One training-step launch with the parameters P of its plan (lanes per vector L,
// npl complex entries per lane).
static ocd_status run_train(const ocd_problem *pb, Params P, int L, int npl, int threads,
                            size_t lds, const void *H, const void *y, const uint8_t *bits,
                            float *z, float *llr, float *loss, float *dlambda, float *dbeta,
                            float *dy, void *workspace, hipStream_t stream)
{
    P.H = H; P.y = y;
    P.bits = bits;
    const double nbits = (double)pb->W * pb->S * pb->U * pb->Q;
    P.inv_nbits = nbits > 0 ? (float)(1.0 / nbits) : 0.f;
    P.z = reinterpret_cast<float2 *>(z);
    P.llr = llr;
    P.dy = reinterpret_cast<float2 *>(dy);
    P.ticket = reinterpret_cast<unsigned *>(workspace);
    P.partials = reinterpret_cast<float *>(static_cast<unsigned char *>(workspace) + 256);
    P.dlambda = dlambda;
    P.dbeta = dbeta;
    P.loss = loss;
    set_vec_ok(P, pb, H, y);
    hipError_t e;
    if (pb->W > 0) {
        e = launch_train(L, npl, pb->storage == OCD_STORE_F16, P, threads, lds, stream);
    } else {
        P.nblocks = 0;   // no workgroups: zero gradients and loss
        e = launch_reduce_partials(P, dlambda, dbeta, loss, stream);
    }
    return e == hipSuccess ? OCD_OK : OCD_EDEVICE;
}

}  // namespace ocd

extern "C" ocd_status ocd_detect_train_bce(const ocd_problem *pb, const void *H, const void *y,
                                           const float *lambda, const uint8_t *bits, float *z,
                                           float *llr, float *loss, float *dlambda, float *dbeta,
                                           float *dy, void *workspace, size_t workspace_bytes,
                                           hipStream_t stream)
{
    ocd_status st = check_train_args(pb, H, y, bits, loss, dlambda, dbeta, workspace,
                                     workspace_bytes);
    if (st != OCD_OK) return st;
    Params P;
    int npl, threads;
    size_t lds;
    ocd_plan pl;
    if (!choose_train_params(pb, lambda, P, npl, threads, lds, &pl)) return OCD_EUNSUPPORTED;
    P.lambda = lambda;
    return run_train(pb, P, pl.lanes_per_vector, npl, threads, lds, H, y, bits, z, llr, loss,
                     dlambda, dbeta, dy, workspace, stream);
}

extern "C" ocd_status ocd_autotune_train(const ocd_problem *pb, const void *H, const void *y,
                                         const float *lambda, const uint8_t *bits, float *loss,
                                         float *dlambda, float *dbeta, float *dy, void *workspace,
                                         size_t workspace_bytes, int repeats, ocd_plan *best,
                                         hipStream_t stream)
{
    ocd_status st = check_train_args(pb, H, y, bits, loss, dlambda, dbeta, workspace,
                                     workspace_bytes);
    if (st != OCD_OK) return st;
    if (!best) return OCD_EINVAL;
    if (pb->W == 0) {
        Params P;
        int npl, threads;
        size_t lds;
        if (!choose_train_params(pb, lambda, P, npl, threads, lds, best)) return OCD_EUNSUPPORTED;
        return OCD_OK;
    }
    repeats = std::max(1, std::min(repeats, 100));
    std::vector<ocd_plan> cands;
    for (int L : {4, 8, 16, 32}) {
        const int cap = 512 / L;
        std::vector<int> vs;
        for (int v = cap; v >= 1 && v >= cap / 16; v /= 2) vs.push_back(v);
        if (pb->S > 1)
            for (int m = pb->S; m <= cap && m <= 4 * pb->S; m += pb->S) vs.push_back(m);
        std::sort(vs.begin(), vs.end());
        vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
        for (int v : vs)
            for (int x : {0, 1}) {
                ocd_plan pl = {L, v, x, 0, 0};
                Params P;
                int npl, threads;
                size_t lds;
                if (train_params(pb, pl, lambda, P, npl, threads, lds)) cands.push_back(pl);
            }
    }
    if (cands.empty()) return OCD_EUNSUPPORTED;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return OCD_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return OCD_EDEVICE; }
    auto time_plan = [&](const ocd_plan &pl, float *ms) -> ocd_status {
        Params P;
        int npl, threads;
        size_t lds;
        if (!train_params(pb, pl, lambda, P, npl, threads, lds)) return OCD_EUNSUPPORTED;
        P.lambda = lambda;
        ocd_status s2 = run_train(pb, P, pl.lanes_per_vector, npl, threads, lds, H, y, bits,
                                  nullptr, nullptr, loss, dlambda, dbeta, dy, workspace, stream);
        if (s2 != OCD_OK) return s2;
        (void)hipEventRecord(e0, stream);
        for (int i = 0; i < repeats && s2 == OCD_OK; ++i)
            s2 = run_train(pb, P, pl.lanes_per_vector, npl, threads, lds, H, y, bits, nullptr,
                           nullptr, loss, dlambda, dbeta, dy, workspace, stream);
        (void)hipEventRecord(e1, stream);
        if (s2 != OCD_OK || hipEventSynchronize(e1) != hipSuccess) return OCD_EDEVICE;
        (void)hipEventElapsedTime(ms, e0, e1);
        return OCD_OK;
    };
    float best_ms = 1e30f;
    ocd_plan best_pl = cands[0];
    for (const ocd_plan &pl : cands) {
        float ms = 0.f;
        st = time_plan(pl, &ms);
        if (st != OCD_OK) break;
        if (ms < best_ms) { best_ms = ms; best_pl = pl; }
    }
    // second stage: the staggered staging on the fastest plan
    if (st == OCD_OK) {
        const ocd_plan base = best_pl;
        for (int sg : {1, 2, 4}) {
            ocd_plan pl = base;
            pl.stagger = sg;
            float ms = 0.f;
            st = time_plan(pl, &ms);
            if (st != OCD_OK) break;
            if (ms < best_ms) { best_ms = ms; best_pl = pl; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != OCD_OK) return st;
    store_plan(plan_key_dir(pb, false, "trn"), best_pl, true);
    store_plan(plan_key_dir(pb, true, "trn"), best_pl, true);
    *best = best_pl;
    return OCD_OK;
}

// ------------------------------------------------------------------ adjoint without allocation

// Scratch of ocd_detect_backward_bce_noalloc: the adjoint's completion counter (first
// 256 bytes) and its per-workgroup partial sums.  A file-scope device array: every GPU
// the library runs on holds its own copy, zero when the code object loads, until the
// process ends.  On the host its name stands in for the symbol and is not a device
// address: host code uses only the per-device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[OCD_NOALLOC_SCRATCH_BYTES];

namespace ocd {

static std::mutex g_scratch_mu;
static void *g_scratch_addr[MAX_DEVICES];

// Device address of the scratch on device dev (the current device), looked up once
// per device.
static ocd_status scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OCD_EDEVICE;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return OCD_OK;
}

}  // namespace ocd

extern "C" ocd_status ocd_detect_backward_bce_noalloc(const ocd_problem *pb, const void *H,
                                                      const void *y, const float *lambda,
                                                      const float *z_hist, const uint8_t *bits,
                                                      float *dlambda, float *dbeta, float *dy,
                                                      hipStream_t stream)
{
    ocd_status st = validate(pb);
    if (st != OCD_OK) return st;
    if (!dlambda || !dbeta) return OCD_EINVAL;
    if (pb->W > 0 && (!H || !y || !z_hist || !bits)) return OCD_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return OCD_EDEVICE;
    if (dev < 0 || dev >= MAX_DEVICES) return OCD_EUNSUPPORTED;
    if (stream) {
        hipDevice_t sdev = 0;
        if (hipStreamGetDevice(stream, &sdev) != hipSuccess) return OCD_EDEVICE;
        if (sdev != dev) return OCD_EINVAL;
    }
    const ocd_plan pl = choose_plan(pb, lambda, true);
    Params P;
    int npl, threads;
    size_t lds;
    if (!make_params(pb, pl, lambda, true, P, npl, threads, lds)) return OCD_EUNSUPPORTED;
    const size_t need = 256 + (size_t)P.nblocks * (size_t)(pb->K + 1) * sizeof(float);
    if (need > OCD_NOALLOC_SCRATCH_BYTES) return OCD_ESCRATCH;
    void *ws = nullptr;
    st = scratch_address(dev, &ws);
    if (st != OCD_OK) return st;
    return run_backward(pb, pl, H, y, lambda, z_hist, nullptr, dlambda, dbeta, dy, ws, stream,
                        bits);
}

extern "C" ocd_status ocd_autotune_backward(const ocd_problem *pb, const void *H, const void *y,
                                            const float *lambda, const float *z_hist,
                                            const float *dllr, float *dlambda, float *dbeta,
                                            float *dy, void *workspace, size_t workspace_bytes,
                                            int repeats, ocd_plan *best, hipStream_t stream)
{
    ocd_status st = check_backward_args(pb, H, y, z_hist, dllr, dlambda, dbeta, workspace,
                                        workspace_bytes);
    if (st != OCD_OK) return st;
    if (!best) return OCD_EINVAL;
    if (pb->W == 0) {
        *best = heuristic_plan(pb, lambda, true, false);
        return OCD_OK;
    }
    repeats = std::max(1, std::min(repeats, 100));
    std::vector<ocd_plan> cands;
    for (int L : {4, 8, 16, 32}) {
        const int cap = 512 / L;
        std::vector<int> vs;
        for (int v = cap; v >= 1 && v >= cap / 16; v /= 2) vs.push_back(v);
        if (pb->S > 1)
            for (int m = pb->S; m <= cap && m <= 4 * pb->S; m += pb->S) vs.push_back(m);
        std::sort(vs.begin(), vs.end());
        vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
        for (int v : vs)
            for (int x : {0, 1}) {
                ocd_plan pl = {L, v, x, 0};
                Params P;
                int npl, threads;
                size_t lds;
                if (make_params(pb, pl, lambda, true, P, npl, threads, lds)) cands.push_back(pl);
            }
    }
    if (cands.empty()) return OCD_EUNSUPPORTED;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return OCD_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return OCD_EDEVICE; }
    float best_ms = 1e30f;
    ocd_plan best_pl = cands[0];
    for (const ocd_plan &pl : cands) {
        st = run_backward(pb, pl, H, y, lambda, z_hist, dllr, dlambda, dbeta, dy, workspace, stream);
        if (st != OCD_OK) break;
        (void)hipEventRecord(e0, stream);
        for (int i = 0; i < repeats && st == OCD_OK; ++i)
            st = run_backward(pb, pl, H, y, lambda, z_hist, dllr, dlambda, dbeta, dy, workspace,
                              stream);
        (void)hipEventRecord(e1, stream);
        if (st != OCD_OK || hipEventSynchronize(e1) != hipSuccess) { st = OCD_EDEVICE; break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) { best_ms = ms; best_pl = pl; }
    }
    // second stage: the staggered staging on the fastest plan
    if (st == OCD_OK) {
        const ocd_plan base = best_pl;
        for (int sg : {1, 2, 4}) {
            ocd_plan pl = base;
            pl.stagger = sg;
            (void)hipEventRecord(e0, stream);
            for (int i = 0; i < repeats && st == OCD_OK; ++i)
                st = run_backward(pb, pl, H, y, lambda, z_hist, dllr, dlambda, dbeta, dy,
                                  workspace, stream);
            (void)hipEventRecord(e1, stream);
            if (st != OCD_OK || hipEventSynchronize(e1) != hipSuccess) { st = OCD_EDEVICE; break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) { best_ms = ms; best_pl = pl; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != OCD_OK) return st;
    store_plan(plan_key(pb, false, true), best_pl, true);
    store_plan(plan_key(pb, true, true), best_pl, true);
    *best = best_pl;
    return OCD_OK;
}
