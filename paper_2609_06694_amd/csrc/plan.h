// Plan object and dispatch map (host only).
#pragma once

#include <string>
#include <vector>

#include "stencil.h"
#include "internal.h"

struct st_plan {
    st_problem prob;                // coeffs pointer cleared; see `dense`
    std::vector<float> dense;       // (2r+1)^ndim coefficients as given
    stk::Taps taps;                 // compact forward taps
    stk::Taps taps_t;               // compact transposed taps (offsets negated)
    stk::TapsD taps64;              // ST_F64 wave plans: the star weights in binary64
    stk::LaunchCfg cfg;
    stk::LaunchCfg adj_cfg;         // wave adjoint and gradient steps (direct-form kernel)
    int ckpt_every;
    bool iso;                       // isotropic star: one weight per distance
    bool batched;
    std::vector<st_plan*> members;  // batched plans own their members
    // Batched launch: pinned host staging for the device member table, and
    // the event of the last upload (the staging is rewritten only after it).
    mutable void* stage = nullptr;
    mutable size_t stage_cap = 0;
    mutable hipEvent_t stage_event = nullptr;
    int tune_tried = 0, tune_rejected = 0;   // last autotune: candidates, parity rejects
};

namespace stk {

// Case key of the dispatch map (Section 4.2: the map is indexed by stencil,
// shape and precision; a cell names the kernel structure that won there).
struct CaseKey {
    int ndim, shape, r, dtype, boundary, update;
    int size_class;   // 0: <= 2^18 cells, 1: <= 2^20, 2: <= 2^22, 3: <= 2^25, 4: larger
    int slab;         // longest side >= 4x the shortest: 1 march axis shortest, 2 longest, 3 neither; else 0
};

CaseKey classify(const st_problem& p);
std::string key_string(const CaseKey& k);

// Key-only update value: the reverse (adjoint and gradient) step of a wave
// case has a map cell of its own next to the forward step's.
constexpr int kKeyWaveReverse = 3;
CaseKey reverse_key(const st_problem& p);
bool adj_cfg_legal(const st_problem& p, const LaunchCfg& c);

// Default entry for a case (compiled in), then the tuning cache file and the
// in-process table written by the autotuner override it.
LaunchCfg dispatch_lookup(const CaseKey& k);
LaunchCfg default_dispatch(const CaseKey& k);
LaunchCfg variant_default(const st_problem& p, int variant);
// Coefficient fields of an ST_VARCOEF problem: one per offset of the shape.
int varcoef_taps(const st_problem& p);
void dispatch_store(const CaseKey& k, const LaunchCfg& cfg, bool persist);
bool cfg_legal(const st_problem& p, const LaunchCfg& c);
constexpr int kAutoChunk = -1;   // dispatch-map value: derive the plane chunk from the grid
// resident > 0 overrides the workgroups per CU assumed for the configuration.
int auto_zchunk(const st_problem& p, const LaunchCfg& c, int resident = 0);

void set_error(const char* fmt, ...);
// Batch depth value asking for each member's own map depth.
constexpr int kMemberDepths = -1;
// Member-table bytes of a batched launch of `steps` steps at batch depth
// kbatch (0: the plan's own).
size_t batched_meta_bytes(const st_plan* plan, int steps, int kbatch = 0);
size_t reverse_tune_bytes(const st_problem& p);   // autotune scratch for a wave plan's reverse step
size_t batch_tune_bytes(const st_plan* plan);   // autotune scratch for the batch depth
Geom geom_of(const st_problem& p);
Geom plan_geom(const st_plan* pl);

}  // namespace stk
