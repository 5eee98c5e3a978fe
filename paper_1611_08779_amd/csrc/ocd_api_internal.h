// ocd_api_internal.h -- host helpers shared by the ABI translation units.
#pragma once

#include <string>

#include "../../include/ocd.h"
#include "ocd_internal.h"

namespace ocd {

ocd_status validate(const ocd_problem *pb);
constexpr int MAX_DEVICES = 64;
const char *arch_name();
int lds_limit_bytes();
float box_edge(int Q);
int npl_for(int B, int L);
// min_npl (a power of two <= 32, or 0): at least this many complex entries per lane,
// the antennas past B zero-padded (the batched kernel is built for a few widths only)
bool make_params(const ocd_problem *pb, const ocd_plan &pl, const float *lambda, bool backward,
                 Params &P, int &npl, int &threads, size_t &lds, int min_npl = 0);
void set_vec_ok(Params &P, const ocd_problem *pb, const void *H, const void *y);
ocd_plan heuristic_plan(const ocd_problem *pb, const float *lambda, bool backward, bool allow_reg);
ocd_plan choose_plan(const ocd_problem *pb, const float *lambda, bool backward);
// Key of the plan cache: architecture, direction and problem shape, in a fixed
// buffer (building and looking up a key never allocates).
struct PlanKey {
    char s[192];
};
PlanKey plan_key(const ocd_problem *pb, bool per_sweep, bool backward);
PlanKey plan_key_dir(const ocd_problem *pb, bool per_sweep, const char *dir);
bool cached_plan(const PlanKey &key, ocd_plan &pl);
void store_plan(const PlanKey &key, const ocd_plan &pl, bool persist);
ocd_status run_forward(const ocd_problem *pb, const ocd_plan &pl, const void *H, const void *y,
                       const float *lambda, const float *g, const float *dinv, const float *p,
                       float *z, float *llr, float *z_hist, hipStream_t stream);

}  // namespace ocd
