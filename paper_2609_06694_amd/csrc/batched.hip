// Batched launch over many independent 2D grids.
//
// All members advance one time block (k_g fused steps of member g) per
// launch: a launch covers every member's row-march workgroups, so one kernel
// fills the device with the work of many small grids instead of one launch
// per grid and block.  The blocks of a member are ordered by the launches
// themselves (one stream), so no workgroup ever waits on another.  A member
// with fewer blocks than the longest one has its workgroups exit at once in
// the remaining launches.  Each workgroup finds its member by a binary search
// over the members' first workgroup indices in a device table (member
// geometry, buffers and coefficients), written from pinned host staging.
//
// Members keep their own stencil (shape, radius, coefficients) and extent;
// they share storage type and boundary rule.  The fused depth k is one batch
// depth for all members (every launch carries every member), or, on request,
// each member's own depth from its map entry: then the deep members finish
// in fewer launches, and every launch re-divides the device among the
// members still running (a table per distinct set of running members), so
// the last launches are not left mostly idle.  Blocks ping-pong
// between the caller's output and a workspace partner so that the last
// block of every member lands in its output.
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "plan.h"
#include "ym2d_run.h"

namespace stk {

constexpr int kGroupThreads = 256;

struct GMember {
    const void* in;   // source of block 1 (u_in, or its workspace copy)
    void* out;        // caller output: receives the last block
    void* ws;         // ping-pong partner
    int nx, ny;
    int k;            // fused steps per block (window geometry)
    int L;            // blocks: ceil(steps / k)
    int ow, ych, strips;
    int first;        // first workgroup of this member in every launch
    int shape, r;
    Taps taps;
};

template <typename T, int BC, int RY, int R, int SHAPE>
__device__ void grouped_member(const GMember& m, int round, int steps, int local, acc_t<T>* lds) {
    const int kl = min(m.k, steps - round * m.k);
    // Block j = round + 1 writes out if (L - j) is even, else the partner.
    const int j = round + 1;
    T* dst = (T*)(((m.L - j) % 2 == 0) ? m.out : m.ws);
    const T* src = (const T*)(j == 1 ? m.in : (((m.L - j + 1) % 2 == 0) ? m.out : m.ws));
    ym2d_run<R, SHAPE, T, BC, kGroupThreads, RY, 2>(src, dst, m.nx, m.ny, m.k, kl, m.ow, m.ych,
                                                    m.strips, local, m.taps, lds);
}

template <typename T, int BC, int RY>
__global__ __launch_bounds__(kGroupThreads) void grouped_kernel(const GMember* __restrict__ ms, int nm,
                                                                int round, int steps) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    acc_t<T>* lds = reinterpret_cast<acc_t<T>*>(lds_raw);   // member rings in the arithmetic type
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = nm - 1;   // last member whose first workgroup is <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ms[mid].first <= b) lo = mid;
        else hi = mid - 1;
    }
    const GMember& m = ms[lo];
    if (round >= m.L) return;   // uniform: this member has finished
    const int local = b - m.first;
    if (m.shape == kStar) {
        switch (m.r) {
            case 1: grouped_member<T, BC, RY, 1, kStar>(m, round, steps, local, lds); break;
            case 2: grouped_member<T, BC, RY, 2, kStar>(m, round, steps, local, lds); break;
            case 3: grouped_member<T, BC, RY, 3, kStar>(m, round, steps, local, lds); break;
            case 4: grouped_member<T, BC, RY, 4, kStar>(m, round, steps, local, lds); break;
        }
    } else {
        switch (m.r) {
            case 1: grouped_member<T, BC, RY, 1, kBox>(m, round, steps, local, lds); break;
            case 2: grouped_member<T, BC, RY, 2, kBox>(m, round, steps, local, lds); break;
        }
    }
}

template <typename T, int BC, int RY>
static hipError_t launch_round(const GMember* d_members, int nm, int round, int steps, int grid,
                               size_t lds, hipStream_t s) {
    if (lds > 64 * 1024) {
        hipError_t e = allow_large_lds<grouped_kernel<T, BC, RY>>();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((grouped_kernel<T, BC, RY>), dim3(grid), dim3(kGroupThreads), lds, s, d_members, nm,
                       round, steps);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_round_t(int bc, int ry, const GMember* d, int nm, int round, int steps,
                                 int grid, size_t lds, hipStream_t s) {
    if (bc == kPeriodic)
        return ry == 8 ? launch_round<T, kPeriodic, 8>(d, nm, round, steps, grid, lds, s)
                       : launch_round<T, kPeriodic, 4>(d, nm, round, steps, grid, lds, s);
    return ry == 8 ? launch_round<T, kZero, 8>(d, nm, round, steps, grid, lds, s)
                   : launch_round<T, kZero, 4>(d, nm, round, steps, grid, lds, s);
}

}  // namespace stk

using namespace stk;

namespace {

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of one storage value and of one ring value (the arithmetic type:
// f64 for f64 storage, else f32).
int storage_bytes(int dtype) { return dtype == ST_F16 ? 2 : (dtype == ST_F64 ? 8 : 4); }
int ring_bytes(int dtype) { return dtype == ST_F64 ? 8 : 4; }

size_t member_grid_bytes(const st_plan* m) {
    return (size_t)m->prob.n[0] * m->prob.n[1] * storage_bytes(m->prob.dtype);
}

// Fused depth of member m in a grouped launch: the batch depth (kbatch =
// kMemberDepths: the member's own map depth), within the limits of a
// 256-column window (at least 64 output columns) and of LDS.
int member_depth(const st_plan* m, int kbatch) {
    const int r = m->prob.radius;
    if (kbatch == kMemberDepths) kbatch = m->cfg.tsteps;
    int k = std::min(16, std::max(1, kbatch));
    while (k > 1 && (kGroupThreads - 2 * k * r < kWave ||
                     ring_bytes(m->prob.dtype) * k * ym2d_ring_rows(4, r) * (kGroupThreads + 2 * r) > ym2d_max_lds_bytes()))
        --k;
    return k;
}

struct Layout {
    std::vector<GMember> members;   // pointers filled at apply time
    int rounds = 0, grid = 0, ry = 8;
    size_t lds = 0;
};

// Relative cost of one cell of member b in a grouped launch: its stencil's
// taps plus a fixed share for the loads, stores, ring traffic and
// addressing of a cell, times the window's recompute (the fused stages run
// on all kGroupThreads columns to keep ow).  The fixed share is measured:
// on the 64-grid mixed workload (k = 3) shares by cells alone ran at
// 614-620 GCells/s, and a fixed share of 6, 12, 15, 18, 24 and 36 taps at
// about 655, 695, 713, 712, 675 and 670.
constexpr double kCellOverhead = 15.0;

double member_cost(const GMember& b) {
    const int taps = b.shape == kStar ? 4 * b.r + 1 : (2 * b.r + 1) * (2 * b.r + 1);
    return (taps + kCellOverhead) * (double)kGroupThreads / b.ow;
}

// Geometry of the grouped launches from launch `round` on: chunks sized so
// that every member still running gets workgroups in proportion to its
// cells times their cost, about eight per CU in total (two and four per CU
// measured 40 % and 5 % slower on the 64-grid workload); finished members
// get none.  Weighting by cost keeps the workgroups of a launch of similar
// length: each XCD runs a contiguous range of them, and a range heavy in
// wide stencils would otherwise finish last.  The row
// count per iteration and the LDS reservation cover every member, so all
// launches share one kernel.
Layout layout(const st_plan* plan, int steps, int cus, int round = 0) {
    Layout lay;
    const int nm = (int)plan->members.size();
    int need8 = 0;
    for (int g = 0; g < nm; ++g) {
        const st_plan* m = plan->members[g];
        GMember b;
        memset(&b, 0, sizeof b);
        b.nx = (int)m->prob.n[0];
        b.ny = (int)m->prob.n[1];
        b.r = m->prob.radius;
        b.shape = m->prob.shape;
        b.k = member_depth(m, plan->cfg.tsteps);
        b.L = steps > 0 ? (steps + b.k - 1) / b.k : 0;
        b.ow = kGroupThreads - 2 * b.k * b.r;
        b.strips = (b.nx + b.ow - 1) / b.ow;
        b.taps = m->taps;
        lay.rounds = std::max(lay.rounds, b.L);
        if (ring_bytes(m->prob.dtype) * b.k * ym2d_ring_rows(8, b.r) * (kGroupThreads + 2 * b.r) > 64 * 1024) need8 = 1;
        lay.members.push_back(b);
    }
    double total = 0;
    for (const GMember& b : lay.members)
        if (b.L > round) total += (double)b.nx * b.ny * member_cost(b);
    const double target = 8.0 * cus;
    // Eight input rows per iteration unless a member's rings would outgrow
    // 64 KiB; the launch reserves the largest member's rings.
    lay.ry = need8 ? 4 : 8;
    // With the row count known, each chunk fills its last march iteration;
    // the workgroup ranges follow.
    lay.grid = 0;
    for (GMember& b : lay.members) {
        const double share = target * ((double)b.nx * b.ny * member_cost(b) / std::max(1.0, total));
        const int chunks = std::max(1, (int)(share / b.strips + 0.5));
        int ych = (b.ny + chunks - 1) / chunks;
        ych = std::max(ych, std::max(16, 4 * b.k * b.r));
        b.ych = ym2d_fill_chunk(std::min(ych, b.ny), b.k * b.r, lay.ry, b.ny);
        b.first = lay.grid;
        if (b.L > round) lay.grid += b.strips * ((b.ny + b.ych - 1) / b.ych);
        lay.lds = std::max(lay.lds, (size_t)ring_bytes(plan->prob.dtype) * b.k * ym2d_ring_rows(lay.ry, b.r) *
                                        (kGroupThreads + 2 * b.r));
    }
    return lay;
}

// Launches at which the set of running members changes (0 first): each
// starts a new member table.
std::vector<int> table_starts(const st_plan* plan, int steps, int kbatch) {
    std::vector<int> ends;   // distinct block counts
    for (const st_plan* m : plan->members) {
        const int k = member_depth(m, kbatch);
        ends.push_back(steps > 0 ? (steps + k - 1) / k : 0);
    }
    std::sort(ends.begin(), ends.end());
    ends.erase(std::unique(ends.begin(), ends.end()), ends.end());
    std::vector<int> starts{0};
    for (int e : ends)
        if (e > 0 && e < ends.back()) starts.push_back(e);
    return starts;
}

// The whole launch schedule of a batched apply, built on the host before
// any device work: one member table per distinct set of running members,
// every table carrying the members' buffers.
struct Schedule {
    std::vector<int> starts;    // first launch of each table
    std::vector<Layout> tabs;   // tabs[i].members: geometry and buffers of table i
    std::vector<int> copy_in;   // members whose input is first copied to their partner (ws)
    int rounds = 0;
};

// Builds the schedule for buffers u_in / u_out (per member) and the
// workspace base ws (partner grids first), then checks it: every buffer
// set, and in every table the running members' workgroup ranges tile
// [0, grid) in order with at least one workgroup each.  Returns NULL, or
// what is wrong.
const char* build_schedule(const st_plan* plan, int steps, int cus, const void* const* u_in,
                           void* const* u_out, char* ws, Schedule& sc) {
    const int nm = (int)plan->members.size();
    sc.starts = table_starts(plan, steps, plan->cfg.tsteps);
    sc.tabs.clear();
    sc.copy_in.clear();
    for (int start : sc.starts) sc.tabs.push_back(layout(plan, steps, cus, start));
    sc.rounds = sc.tabs[0].rounds;
    size_t off = 0;
    for (int g = 0; g < nm; ++g) {
        const GMember& b0 = sc.tabs[0].members[g];
        void* partner = ws + off;
        off += align256(member_grid_bytes(plan->members[g]));
        // In place with an odd block count: block 1 would write the grid it
        // reads, so it reads a copy in the partner instead (block 2 writes
        // the partner only after block 1's launch has completed).
        const bool copy = u_in[g] == u_out[g] && (b0.L % 2) == 1;
        if (copy) sc.copy_in.push_back(g);
        for (Layout& t : sc.tabs) {
            GMember& b = t.members[g];
            b.in = copy ? partner : u_in[g];
            b.out = u_out[g];
            b.ws = partner;
        }
    }
    for (size_t i = 0; i < sc.tabs.size(); ++i) {
        const Layout& t = sc.tabs[i];
        int next = 0;
        for (int g = 0; g < nm; ++g) {
            const GMember& b = t.members[g];
            if (!b.in || !b.out || !b.ws) return "a member table entry has no buffer";
            if (b.first != next) return "member workgroup ranges are not contiguous";
            if (b.L <= sc.starts[i]) continue;   // finished: no workgroups
            if (b.k < 1 || b.ow < kWave || b.strips < 1 || b.ych < 1) return "member geometry out of range";
            next += b.strips * ((b.ny + b.ych - 1) / b.ych);
        }
        if (next != t.grid || t.grid < 1) return "launch size does not match the member ranges";
        if (t.ry != sc.tabs[0].ry || t.lds != sc.tabs[0].lds) return "tables disagree on the launch shape";
    }
    return nullptr;
}

}  // namespace

namespace stk {

size_t batched_meta_bytes(const st_plan* plan, int steps, int kbatch) {
    if (kbatch == 0) kbatch = plan->cfg.tsteps;
    return align256(sizeof(GMember) * plan->members.size() * table_starts(plan, steps, kbatch).size());
}

}  // namespace stk

#define B_FAIL(code, ...)             \
    do {                              \
        stk::set_error(__VA_ARGS__);  \
        return (code);                \
    } while (0)

#define B_HIP(expr)                                                                       \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) B_FAIL(ST_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

extern "C" {

st_status stencil_plan_batched(const st_problem* problems, int32_t count, const st_plan_opts* opts,
                               st_plan** out) {
    stk::set_error("%s", "");
    if (!out) B_FAIL(ST_EINVAL, "out is NULL");
    *out = nullptr;
    if (!problems || count < 1) B_FAIL(ST_EINVAL, "need at least one problem");
    st_plan* pl = new (std::nothrow) st_plan();
    if (!pl) B_FAIL(ST_ENOMEM, "out of host memory");
    pl->batched = true;
    pl->ckpt_every = 0;
    memset(&pl->cfg, 0, sizeof pl->cfg);
    pl->cfg.variant = ST_VARIANT_YM2D;
    pl->cfg.tile_x = kGroupThreads;
    // Three fused steps measured fastest for the 64-grid workload (k = 1, 2,
    // 4: 47 %, 5 %, 32 % slower; deeper rings of wide stencils cut occupancy).
    // opts->tsteps = -1 (kMemberDepths): each member's own map depth.
    if (opts && opts->tsteps < kMemberDepths) {
        delete pl;
        B_FAIL(ST_EINVAL, "batched tsteps must be >= -1");
    }
    pl->cfg.tsteps = (opts && (opts->tsteps > 0 || opts->tsteps == kMemberDepths)) ? opts->tsteps : 3;
    // Member plans carry the stencils; the batch depth is not theirs to check.
    st_plan_opts mopts;
    if (opts) {
        mopts = *opts;
        mopts.tsteps = 0;
    }
    for (int i = 0; i < count; ++i) {
        const st_problem& p = problems[i];
        if (p.ndim != 2 || p.update != ST_LINEAR) {
            stencil_plan_destroy(pl);
            B_FAIL(ST_EUNSUPPORTED, "batched member %d: only 2D linear sweeps are batched", i);
        }
        if (p.dtype != problems[0].dtype || p.boundary != problems[0].boundary) {
            stencil_plan_destroy(pl);
            B_FAIL(ST_EINVAL, "batched members must share dtype and boundary (member %d)", i);
        }
        st_plan* m = nullptr;
        st_status s = stencil_plan(&p, opts ? &mopts : nullptr, &m);
        if (s != ST_OK) {
            stencil_plan_destroy(pl);
            return s;
        }
        pl->members.push_back(m);
    }
    pl->prob = pl->members[0]->prob;
    *out = pl;
    return ST_OK;
}

st_status stencil_apply_batched(const st_plan* plan, const void* const* u_in, void* const* u_out,
                                int32_t steps, void* workspace, size_t ws_bytes, void* stream) {
    stk::set_error("%s", "");
    if (!plan || !plan->batched) B_FAIL(ST_EINVAL, "not a batched plan");
    if (!u_in || !u_out) B_FAIL(ST_EINVAL, "pointer arrays are NULL");
    if (steps < 0) B_FAIL(ST_EINVAL, "steps must be >= 0");
    const int nm = (int)plan->members.size();
    for (int g = 0; g < nm; ++g)
        if (!u_in[g] || !u_out[g]) B_FAIL(ST_EINVAL, "member %d has a NULL grid pointer", g);
    hipStream_t s = (hipStream_t)stream;
    if (steps == 0) {
        for (int g = 0; g < nm; ++g)
            if (u_in[g] != u_out[g])
                B_HIP(hipMemcpyAsync(u_out[g], u_in[g], member_grid_bytes(plan->members[g]),
                                     hipMemcpyDeviceToDevice, s));
        return ST_OK;
    }
    const size_t need = stencil_workspace_bytes(plan, steps, 0);
    if (!workspace || ws_bytes < need) B_FAIL(ST_EWORKSPACE, "workspace of %zu bytes needed", need);

    int dev = 0, cus = 0;
    B_HIP(hipGetDevice(&dev));
    B_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    Schedule sc;
    char* ws = (char*)workspace;
    const char* bad = build_schedule(plan, steps, std::max(1, cus), u_in, u_out, ws, sc);
    if (bad) B_FAIL(ST_EINVAL, "batched schedule: %s", bad);
    const Layout& lay = sc.tabs[0];
    if (lay.lds > (size_t)ym2d_max_lds_bytes()) B_FAIL(ST_EUNSUPPORTED, "member rings exceed LDS");
    size_t grids = 0;
    for (int g = 0; g < nm; ++g) grids += align256(member_grid_bytes(plan->members[g]));
    GMember* d_members = (GMember*)(ws + grids);
    for (int g : sc.copy_in)
        B_HIP(hipMemcpyAsync(sc.tabs[0].members[g].ws, u_in[g], member_grid_bytes(plan->members[g]),
                             hipMemcpyDeviceToDevice, s));

    // Upload the member tables from plan-owned pinned staging; the previous
    // upload must have left the staging before it is rewritten.
    const size_t tb = sizeof(GMember) * nm;
    const size_t mb = tb * sc.tabs.size();
    if (!plan->stage_event) B_HIP(hipEventCreateWithFlags(&plan->stage_event, hipEventDisableTiming));
    else B_HIP(hipEventSynchronize(plan->stage_event));
    if (plan->stage_cap < mb) {
        if (plan->stage) B_HIP(hipHostFree(plan->stage));
        plan->stage = nullptr;
        plan->stage_cap = 0;
        B_HIP(hipHostMalloc(&plan->stage, mb, hipHostMallocDefault));
        plan->stage_cap = mb;
    }
    for (size_t i = 0; i < sc.tabs.size(); ++i)
        memcpy((char*)plan->stage + i * tb, sc.tabs[i].members.data(), tb);
    B_HIP(hipMemcpyAsync(d_members, plan->stage, mb, hipMemcpyHostToDevice, s));
    B_HIP(hipEventRecord(plan->stage_event, s));

    const int bc = plan->prob.boundary;
    size_t ti = 0;
    for (int round = 0; round < sc.rounds; ++round) {
        while (ti + 1 < sc.starts.size() && sc.starts[ti + 1] <= round) ++ti;
        const GMember* tab = d_members + ti * nm;
        const int grid = sc.tabs[ti].grid;
        const int dt = plan->prob.dtype;
        hipError_t e = dt == ST_F16   ? launch_round_t<_Float16>(bc, lay.ry, tab, nm, round, steps, grid, lay.lds, s)
                       : dt == ST_F64 ? launch_round_t<double>(bc, lay.ry, tab, nm, round, steps, grid, lay.lds, s)
                                      : launch_round_t<float>(bc, lay.ry, tab, nm, round, steps, grid, lay.lds, s);
        if (e != hipSuccess) B_FAIL(ST_EHIP, "batched launch %d failed: %s", round, hipGetErrorString(e));
    }
    return ST_OK;
}

st_status stencil_plan_describe_batched(const st_plan* plan, int32_t steps, int32_t cus, int32_t* launches,
                                        int32_t* tables, int64_t* workgroups) {
    stk::set_error("%s", "");
    if (!plan || !plan->batched) B_FAIL(ST_EINVAL, "not a batched plan");
    if (steps < 1) B_FAIL(ST_EINVAL, "steps must be >= 1");
    if (cus < 0) B_FAIL(ST_EINVAL, "cus must be >= 0");
    if (cus == 0) {
        int dev = 0;
        B_HIP(hipGetDevice(&dev));
        B_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    // Stand-in buffer addresses (never dereferenced): distinct inputs and
    // outputs, workspace partners after them.
    const int nm = (int)plan->members.size();
    std::vector<const void*> in(nm);
    std::vector<void*> out(nm);
    for (int g = 0; g < nm; ++g) {
        in[g] = (const void*)(uintptr_t)(((uint64_t)2 * g + 1) << 32);
        out[g] = (void*)(uintptr_t)(((uint64_t)2 * g + 2) << 32);
    }
    Schedule sc;
    const char* bad = build_schedule(plan, steps, std::max(1, (int)cus), in.data(), out.data(),
                                     (char*)(uintptr_t)((uint64_t)(2 * nm + 2) << 32), sc);
    if (bad) B_FAIL(ST_EINVAL, "batched schedule: %s", bad);
    int64_t wg = 0;
    size_t ti = 0;
    for (int round = 0; round < sc.rounds; ++round) {
        while (ti + 1 < sc.starts.size() && sc.starts[ti + 1] <= round) ++ti;
        wg += sc.tabs[ti].grid;
    }
    if (launches) *launches = sc.rounds;
    if (tables) *tables = (int32_t)sc.tabs.size();
    if (workgroups) *workgroups = wg;
    return ST_OK;
}

}  // extern "C"
