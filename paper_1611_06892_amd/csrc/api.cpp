// C ABI of libbidiag (declarations and contracts in include/bidiag.h).
//
// A plan holds the task graph of one (m, n, nb, tree, variant) reduction and
// the execution order of its work units, built on the host at creation, with
// a host copy of everything the device reads (page-locked when a device is
// present).  Execution copies that graph into the caller's workspace with an
// asynchronous copy on the caller's stream and enqueues either one persistent
// scheduler launch or one launch per topological level after it: the library
// allocates no device memory and keeps no device state between calls.
#include "../../include/bidiag.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <queue>
#include <tuple>
#include <vector>

#include "adjoint.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace {

// Host bytes that a launch copies into the caller's workspace.  Page-locked
// when a device is present, so that the copy is an asynchronous DMA on the
// caller's stream; plain memory on a host without one (plans are also built
// and inspected there).
struct HostBlob {
    char* p = nullptr;
    size_t bytes = 0;
    bool pinned = false;
    HostBlob() = default;
    HostBlob(const HostBlob&) = delete;
    HostBlob& operator=(const HostBlob&) = delete;
    bool alloc(size_t b) {
        release();
        bytes = b;
        const size_t n = std::max<size_t>(b, 8);
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0 &&
            hipHostMalloc((void**)&p, n, hipHostMallocDefault) == hipSuccess) {
            pinned = true;
        } else {
            (void)hipGetLastError();
            p = (char*)std::malloc(n);
            pinned = false;
        }
        if (p) std::memset(p, 0, n);
        return p != nullptr;
    }
    void release() {
        if (!p) return;
        if (pinned) (void)hipHostFree(p);
        else std::free(p);
        p = nullptr;
        bytes = 0;
    }
    ~HostBlob() { release(); }
};

}  // namespace

struct bb_plan {
    int64_t m = 0, n = 0;
    int32_t nmats = 1;                       // matrices of the graph (batched plans)
    std::vector<int64_t> gidx, dims;         // batched: batch index and (m, n) per matrix
    int nb = 0, tree = 0, variant = 0, prec = 0;
    bb_opts opts{};
    bb::Graph g;
    int ns = 0;                              // update strip width
    std::vector<int32_t> nparts, ndeps, succ_off, succ_idx;
    std::vector<int32_t> units_ticket;       // (task, part) pairs, list-scheduling order
    std::vector<int32_t> units_prio;         // persistent scheduler: (task, part) pairs by priority
    std::vector<int32_t> units_level;        // (task, part) pairs sorted by level
    std::vector<int32_t> level_off;          // units_level offsets per level
    double cp = 0.0, total = 0.0;
    double makespan = 0.0;                   // length of the list schedule (cost-model units)
    // Panel scratch (nb = 256): one area per workgroup of a persistent
    // launch, or per panel unit of the widest level (levels put panels first).
    int64_t pscr_slots = 0;
    bool apply_graph = false;                // applies Q or P (bb_apply_q/p), no panels
    // m < n (Section 3.6): the graph reduces A^T, whose tile (i, j) is tile
    // (j, i) of A seen transposed; the device tasks swap the tile
    // coordinates and flip the transpose flag, so A's storage is used as is.
    bool transposed = false;
    // Host copy of the graph the device reads, uploaded into the workspace
    // by every execution: tasks, initial dependency counts, successors, the
    // unit order of the chosen schedule, batched descriptors' sources.
    HostBlob blob;
    size_t off_tasks = 0, off_ndeps = 0, off_succ_off = 0, off_succ_idx = 0, off_units = 0;
    size_t off_gidx = 0, off_dims = 0, off_recoff = 0;
    // Batched plans: per local matrix, its tile size (NB_MIXED plans), the
    // first global slot of its records and their offset in the group's
    // record area (doubles); vt_doubles: that area's size.
    std::vector<int32_t> mat_nb;
    std::vector<int32_t> slot_base;
    std::vector<int64_t> recoff;
    int64_t vt_doubles = -1;
    std::atomic<uint32_t> used_devices{0};   // devices an upload was enqueued on (bit mask)
    std::once_flag ev_once;
    hipError_t ev_err = hipSuccess;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::atomic<bool> timed{false};
    // Plans that apply Q, Q^T, P or P^T with this plan's records, by
    // (side, transpose, tile columns of C).
    std::map<std::tuple<int, int, int64_t>, bb_plan*> apply;
    std::mutex apply_mu;
    // adjoint: operation list and its host copy
    std::mutex adj_mu;
    bbk::AdjointOps* adj = nullptr;
    HostBlob adj_blob;
};

// A batch: one plan (union graph) per tile size, run one after the other.
struct bb_batch {
    int64_t count = 0;
    int prec = 0;
    bb_opts opts{};
    std::vector<int64_t> m, n;
    std::vector<int32_t> nb, tree, variant;
    struct Group {
        int nb = 0;
        bb_plan* plan = nullptr;
        size_t vt_off = 0, ws_off = 0;   // byte offsets of the group's records / workspace
    };
    std::vector<Group> groups;
    std::vector<int64_t> rec_off;        // per matrix: byte offset of its first record in vt
    std::vector<int64_t> nrec;           // per matrix: number of records
    size_t vt_bytes = 0, ws_bytes = 0;
    std::once_flag ev_once;
    hipError_t ev_err = hipSuccess;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::atomic<bool> timed{false};
    ~bb_batch();
};

namespace {

#include "tuned_table.inc"

// Table 1, then the same update weights for the Q-applying kinds.
const double kUnit[bb::NKINDS] = {4.0, 6.0, 2.0, 6.0, 12.0, 6.0, 6.0, 12.0, 6.0};

// Execution-cost model used to order work on the GPU (relative latency of one
// task with its column strips run side by side).  Unlike Table 1, whose unit
// is flops, it reflects that a panel is a chain of nb dependent Householder
// steps while an update is throughput-bound MFMA work.  Measured on MI355X in
// loaded runs, in units of 10 us:
//  - nb <= 128 (nb = 128): GEQRT / TSQRT / TTQRT panels ~100 / 135 / 120 us,
//    UNMQR / TSMQR / TTMQR tile updates ~41 / 60 / 53 us;
//  - nb = 256: panels ~397 / 506 / 353 us, updates (two 128-column halves
//    side by side) ~104 / 176 / 116 us.
const double kGpuCost[bb::NKINDS] = {10.0, 13.5, 12.0, 4.1, 6.0, 5.3, 4.1, 6.0, 5.3};
const double kGpuCost256[bb::NKINDS] = {39.7, 50.6, 35.3, 10.4, 17.6, 11.6, 10.4, 17.6, 11.6};

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Host validation of a schedule: predecessors precede each task in program
// order and in ticket order, and the dependency counts match the graph.
bool validate(const bb_plan& P) {
    const size_t nt = P.g.tasks.size();
    const size_t nu = P.units_ticket.size() / 2;
    std::vector<int64_t> first(nt, -1), last(nt, -1);
    for (size_t u = 0; u < nu; ++u) {
        int t = P.units_ticket[2 * u];
        if (t < 0 || (size_t)t >= nt) return false;
        if (first[t] < 0) first[t] = (int64_t)u;
        last[t] = (int64_t)u;
    }
    for (size_t t = 0; t < nt; ++t) {
        if (first[t] < 0) return false;
        int32_t nd = 0;
        for (int32_t pr : P.g.pred[t]) {
            if (pr < 0 || (size_t)pr >= t) return false;
            if (last[pr] >= first[t]) return false;
            nd += P.nparts[pr];
        }
        if (nd != P.ndeps[t]) return false;
    }
    return true;
}

// Cost of task t in the GPU cost model.  In a launch that mixes tile sizes a
// task is weighted by (nb / 128)^1.5: small tiles are latency bound, so their
// time falls more slowly than their flops (nb^3).
double task_cost(const bb_plan& P, int t) {
    const bb::Task& x = P.g.tasks[t];
    double c = (P.nb == 256 ? kGpuCost256 : kGpuCost)[x.kind];
    if (!P.mat_nb.empty()) c *= std::pow(P.mat_nb[x.mat] / 128.0, 1.5);
    return c;
}

int build_schedule(bb_plan& P) {
    const bb::Graph& g = P.g;
    const int nt = (int)g.tasks.size();
    // one strip per update below nb = 128 (every task of a mixed launch)
    P.ns = P.nb == bbk::NB_MIXED ? 128 : bbk::strip_width(P.nb);
    const int nb = P.nb == bbk::NB_MIXED ? 128 : P.nb;
    P.nparts.assign(nt, 1);
    for (int t = 0; t < nt; ++t)
        if (!bb::is_panel(g.tasks[t].kind)) P.nparts[t] = (nb + P.ns - 1) / P.ns;
    P.ndeps.assign(nt, 0);
    std::vector<int32_t> cnt(nt + 1, 0);
    for (int t = 0; t < nt; ++t) {
        for (int32_t pr : g.pred[t]) {
            P.ndeps[t] += P.nparts[pr];
            cnt[pr + 1]++;
        }
    }
    P.succ_off.assign(nt + 1, 0);
    for (int t = 0; t < nt; ++t) P.succ_off[t + 1] = P.succ_off[t] + cnt[t + 1];
    P.succ_idx.assign(P.succ_off[nt], 0);
    std::vector<int32_t> fill(P.succ_off.begin(), P.succ_off.end() - 1);
    for (int t = 0; t < nt; ++t)
        for (int32_t pr : g.pred[t]) P.succ_idx[fill[pr]++] = t;

    // Priorities: bottom level (longest path from the task to the end under
    // the GPU cost model).
    std::vector<double> blevel(nt, 0.0);
    for (int t = nt - 1; t >= 0; --t) {
        double b = 0.0;
        for (int s = P.succ_off[t]; s < P.succ_off[t + 1]; ++s) b = std::max(b, blevel[P.succ_idx[s]]);
        blevel[t] = b + task_cost(P, t);
    }
    // Plain bottom levels for both variants: ranking R-BiDiag's second phase
    // above QR(p,q) measured slightly slower for tall and square inputs.
    const std::vector<double>& prio = blevel;
    P.cp = bb::critical_path(g, kUnit);
    P.total = 0.0;
    for (int t = 0; t < nt; ++t) P.total += kUnit[g.tasks[t].kind];

    // Ticket order: list scheduling of the units on W workers, highest bottom
    // level first; the order in which units start is the ticket order.
    const int W = std::max(1, P.opts.workgroups);
    typedef std::tuple<double, int, int> RK;   // (-priority, task, part)
    std::priority_queue<RK, std::vector<RK>, std::greater<RK>> ready;
    typedef std::tuple<double, int> EV;        // (finish time, task)
    std::priority_queue<EV, std::vector<EV>, std::greater<EV>> running;
    std::vector<int32_t> indeg(nt), left(nt);
    for (int t = 0; t < nt; ++t) {
        indeg[t] = (int32_t)g.pred[t].size();
        left[t] = P.nparts[t];
        if (indeg[t] == 0)
            for (int q = 0; q < P.nparts[t]; ++q) ready.emplace(-prio[t], t, q);
    }
    P.units_ticket.clear();
    double now = 0.0;
    int busy = 0;
    while (!ready.empty() || !running.empty()) {
        while (busy < W && !ready.empty()) {
            RK r = ready.top();
            ready.pop();
            int t = std::get<1>(r);
            P.units_ticket.push_back(t);
            P.units_ticket.push_back(std::get<2>(r));
            running.emplace(now + task_cost(P, t), t);
            busy++;
        }
        if (running.empty()) break;
        EV e = running.top();
        running.pop();
        now = std::get<0>(e);
        busy--;
        int t = std::get<1>(e);
        if (--left[t] == 0) {
            for (int s = P.succ_off[t]; s < P.succ_off[t + 1]; ++s) {
                int v = P.succ_idx[s];
                if (--indeg[v] == 0)
                    for (int q = 0; q < P.nparts[v]; ++q) ready.emplace(-prio[v], v, q);
            }
        }
    }

    P.makespan = now;

    // The persistent scheduler claims units in this simulated start order
    // (topological: a unit starts after its predecessors finished).
    P.units_prio = P.units_ticket;

    // Levels: longest path, in tasks, from a source.
    std::vector<int32_t> level(nt, 0);
    int nlev = 0;
    for (int t = 0; t < nt; ++t) {
        int l = 0;
        for (int32_t pr : g.pred[t]) l = std::max(l, level[pr] + 1);
        level[t] = l;
        nlev = std::max(nlev, l + 1);
    }
    const size_t nu = P.units_ticket.size() / 2;
    P.level_off.assign(nlev + 1, 0);
    for (size_t u = 0; u < nu; ++u) P.level_off[level[P.units_ticket[2 * u]] + 1]++;
    for (int l = 0; l < nlev; ++l) P.level_off[l + 1] += P.level_off[l];
    P.units_level.assign(2 * nu, 0);
    // Within a level the panels come first, so that a panel's block index
    // is also its scratch slot.
    std::vector<int32_t> lf(P.level_off.begin(), P.level_off.end() - 1);
    std::vector<int32_t> npan(nlev, 0);
    for (int pass = 0; pass < 2; ++pass)
        for (size_t u = 0; u < nu; ++u) {
            int t = P.units_ticket[2 * u];
            if (bb::is_panel(g.tasks[t].kind) != (pass == 0)) continue;
            if (pass == 0) npan[level[t]]++;
            int pos = lf[level[t]]++;
            P.units_level[2 * pos] = t;
            P.units_level[2 * pos + 1] = P.units_ticket[2 * u + 1];
        }
    P.pscr_slots = 0;
    if (bbk::panel_scratch_doubles(P.nb) > 0 && !P.apply_graph) {
        int32_t widest = 0;
        for (int32_t c : npan) widest = std::max(widest, c);
        P.pscr_slots = P.opts.sched == BB_SCHED_PERSISTENT ? std::max(1, P.opts.workgroups) : widest;
    }
    return validate(P) ? BB_OK : BB_EDAG;
}

// Workspace: control words, the launch's matrix descriptors, one dependency
// counter per task, the trace (BB_FLAG_TRACE), the copy of the graph, then
// the panels' scratch (nb = 256).
size_t ws_mats_off() { return round_up(sizeof(int32_t) * bbk::CTRL_WORDS, 256); }
size_t ws_deps_off(const bb_plan& P) {
    return ws_mats_off() + round_up(sizeof(bbk::MatDesc) * (size_t)P.nmats, 256);
}
size_t ws_trace_off(const bb_plan& P) {
    return ws_deps_off(P) + round_up(sizeof(int32_t) * P.g.tasks.size(), 256);
}
size_t ws_blob_off(const bb_plan& P) {
    size_t b = ws_trace_off(P);
    if (P.opts.flags & BB_FLAG_TRACE) b += round_up(4 * sizeof(int64_t) * (P.units_ticket.size() / 2), 256);
    return b;
}
size_t ws_pscr_off(const bb_plan& P) { return ws_blob_off(P) + round_up(P.blob.bytes, 256); }
size_t ws_bytes_of(const bb_plan& P) {
    return ws_pscr_off(P) + (size_t)P.pscr_slots * (size_t)bbk::panel_scratch_doubles(P.nb) * sizeof(double);
}

size_t vt_bytes_of(const bb_plan& P) {
    if (P.vt_doubles >= 0) return (size_t)P.vt_doubles * sizeof(double);
    return (size_t)P.g.nslots * (size_t)bbk::record_doubles(P.nb) * sizeof(double);
}

// Lay out the device's view of the graph in the plan's host blob: tasks,
// initial dependency counts, successor lists, the units of the plan's
// schedule (priority order or levels) and, for batches, the per-matrix
// sources of the descriptors.  Called once, when the plan is built.
int build_blob(bb_plan& P) {
    const size_t nt = P.g.tasks.size();
    const std::vector<int32_t>& units = P.opts.sched == BB_SCHED_PERSISTENT ? P.units_prio : P.units_level;
    size_t off = 0;
    P.off_tasks = off; off = round_up(off + nt * sizeof(bbk::DevTask), 256);
    P.off_ndeps = off; off = round_up(off + nt * 4, 256);
    P.off_succ_off = off; off = round_up(off + P.succ_off.size() * 4, 256);
    P.off_succ_idx = off; off = round_up(off + std::max<size_t>(1, P.succ_idx.size()) * 4, 256);
    P.off_units = off; off = round_up(off + units.size() * 4, 256);
    P.off_gidx = off; off = round_up(off + P.gidx.size() * 8, 256);
    P.off_dims = off; off = round_up(off + P.dims.size() * 8, 256);
    P.off_recoff = off; off = round_up(off + P.recoff.size() * 8, 256);
    if (!P.blob.alloc(off)) return BB_ENOMEM;
    char* h = P.blob.p;
    bbk::DevTask* dt = (bbk::DevTask*)(h + P.off_tasks);
    for (size_t t = 0; t < nt; ++t) {
        const bb::Task& s = P.g.tasks[t];
        // slot within the task's matrix; tile-size code in trans >> 1
        const int32_t slot = s.slot - (P.slot_base.empty() ? 0 : P.slot_base[s.mat]);
        int32_t code = 0;
        if (!P.mat_nb.empty()) code = P.mat_nb[s.mat] == 32 ? 0 : P.mat_nb[s.mat] == 64 ? 1 : 2;
        dt[t] = P.transposed ? bbk::DevTask{s.kind, (s.trans ^ 1) | (code << 1), s.c1, s.r1, s.c2, s.r2, slot, s.mat}
                             : bbk::DevTask{s.kind, s.trans | (code << 1), s.r1, s.c1, s.r2, s.c2, slot, s.mat};
    }
    auto put32 = [&](size_t o, const std::vector<int32_t>& v) {
        if (!v.empty()) std::memcpy(h + o, v.data(), v.size() * 4);
    };
    auto put64 = [&](size_t o, const std::vector<int64_t>& v) {
        if (!v.empty()) std::memcpy(h + o, v.data(), v.size() * 8);
    };
    put32(P.off_ndeps, P.ndeps);
    put32(P.off_succ_off, P.succ_off);
    put32(P.off_succ_idx, P.succ_idx);
    put32(P.off_units, units);
    put64(P.off_gidx, P.gidx);
    put64(P.off_dims, P.dims);
    put64(P.off_recoff, P.recoff);
    return BB_OK;
}

// Enqueue the copy of the plan's graph into workspace ws (stream-ordered).
int upload_graph(bb_plan& P, void* ws, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return BB_EHIP;
    if (dev < 32) P.used_devices.fetch_or(1u << dev);
    if (hipMemcpyAsync((char*)ws + ws_blob_off(P), P.blob.p, P.blob.bytes, hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return BB_EHIP;
    return BB_OK;
}

int device_attr(hipDeviceAttribute_t attr, int fallback) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, attr, dev) != hipSuccess || v <= 0)
        return fallback;
    return v;
}

// The kernel family a plan runs: its arithmetic for reductions, the
// application kernels for the graphs that apply Q or P.
int kernel_prec(const bb_plan& P) { return P.apply_graph ? bbk::PREC_APPLY : P.prec; }

int plan_events(bb_plan& P) {
    std::call_once(P.ev_once, [&P] {
        if (hipEventCreate(&P.ev0) != hipSuccess || hipEventCreate(&P.ev1) != hipSuccess)
            P.ev_err = hipErrorInvalidValue;
    });
    return P.ev_err == hipSuccess ? BB_OK : BB_EHIP;
}

// Enqueue one run of plan P (arguments already validated, graph already
// uploaded into ws on this stream).  d0: the only matrix of a single-matrix
// plan; NULL when the descriptors of a batched plan are already in the
// workspace.
int launch_kernels(bb_plan& P, const bbk::MatDesc* d0, void* vt, void* ws, hipStream_t s,
                   bool allow_timing = true) {
    bbk::KArgs a{};
    if (d0) {
        a.single = *d0;
        a.single.rec = (double*)vt;
        a.mats = nullptr;
    } else {
        a.mats = (const bbk::MatDesc*)((char*)ws + ws_mats_off());
    }
    char* blob = (char*)ws + ws_blob_off(P);
    a.tasks = (const bbk::DevTask*)(blob + P.off_tasks);
    a.nunits = (int32_t)(P.units_ticket.size() / 2);
    a.units = (const int2*)(blob + P.off_units);
    a.succ_off = (const int32_t*)(blob + P.off_succ_off);
    a.succ_idx = (const int32_t*)(blob + P.off_succ_idx);
    a.ctrl = (int32_t*)ws;
    a.deps = (int32_t*)((char*)ws + ws_deps_off(P));
    const double khz = (double)device_attr(hipDeviceAttributeWallClockRate, 100000);
    a.watchdog_ticks = (int64_t)(P.opts.watchdog_s * khz * 1000.0);
    a.trace = (P.opts.flags & BB_FLAG_TRACE) ? (int64_t*)((char*)ws + ws_trace_off(P)) : nullptr;
    a.pscratch = P.pscr_slots > 0 ? (double*)((char*)ws + ws_pscr_off(P)) : nullptr;

    const bool timed = allow_timing && (P.opts.flags & BB_FLAG_TIMING) != 0;
    if (timed && plan_events(P) != BB_OK) return BB_EHIP;
    const bool persistent = P.opts.sched == BB_SCHED_PERSISTENT;
    if (bbk::launch_init(a, (const int32_t*)(blob + P.off_ndeps), (int32_t)P.g.tasks.size(), s) != hipSuccess)
        return BB_EHIP;
    if (timed && hipEventRecord(P.ev0, s) != hipSuccess) return BB_EHIP;
    if (a.nunits > 0) {
        if (persistent) {
            const int cus = device_attr(hipDeviceAttributeMultiprocessorCount, P.opts.workgroups);
            int wg = std::min(P.opts.workgroups, cus);
            wg = std::max(1, std::min(wg, a.nunits));
            if (bbk::launch_persistent(P.nb, kernel_prec(P), a, wg, s) != hipSuccess) return BB_EHIP;
        } else {
            for (size_t l = 0; l + 1 < P.level_off.size(); ++l) {
                int32_t b = P.level_off[l], e = P.level_off[l + 1];
                if (bbk::launch_level(P.nb, kernel_prec(P), a, b, e - b, s) != hipSuccess) return BB_EHIP;
            }
        }
    }
    if (timed && hipEventRecord(P.ev1, s) != hipSuccess) return BB_EHIP;
    if (allow_timing) P.timed = timed;
    return BB_OK;
}

int launch_plan(bb_plan& P, const bbk::MatDesc* d0, void* vt, void* ws, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    int rc = upload_graph(P, ws, s);
    if (rc != BB_OK) return rc;
    return launch_kernels(P, d0, vt, ws, s);
}

// Finish a plan whose graph is built: schedule, then the host copy of what
// the device reads.
int finish_plan(bb_plan& P) {
    int rc = build_schedule(P);
    if (rc != BB_OK) return rc;
    return build_blob(P);
}

// The plan applying side (0: Q, 1: P), transposed or not, to ncols columns.
int get_apply(bb_plan* P, int side, int transpose, int64_t ncols, bb_plan** out) {
    const int64_t jc = (ncols + P->nb - 1) / P->nb;
    if (jc > (1 << 20)) return BB_ENOTSUP;
    std::lock_guard<std::mutex> lk(P->apply_mu);
    auto key = std::make_tuple(side, transpose, jc);
    auto it = P->apply.find(key);
    if (it != P->apply.end()) {
        *out = it->second;
        return BB_OK;
    }
    bb_plan* Q = new (std::nothrow) bb_plan();
    if (!Q) return BB_ENOMEM;
    Q->m = side == 0 ? P->m : P->n;
    Q->n = jc * P->nb;
    Q->nb = P->nb;
    Q->tree = P->tree;
    Q->variant = P->variant;
    Q->prec = BB_F64;
    Q->apply_graph = true;
    Q->opts = P->opts;
    try {
        // For a transposed plan, Q of A is P of A^T and the other way round.
        bb::build_apply_graph(P->g, P->transposed ? 1 - side : side, transpose, (int)jc, Q->g);
        int rc = finish_plan(*Q);
        if (rc != BB_OK) {
            delete Q;
            return rc;
        }
    } catch (const std::bad_alloc&) {
        delete Q;
        return BB_ENOMEM;
    }
    P->apply[key] = Q;
    *out = Q;
    return BB_OK;
}

bb_opts resolved_opts(const bb_opts* o) {
    bb_opts r{};
    if (o) r = *o;
    if (r.workgroups <= 0) {
        r.workgroups = 0;   // resolved to the CU count at first execution
    }
    if (!(r.gamma > 0.0)) r.gamma = 2.0;
    if (!(r.watchdog_s > 0.0)) r.watchdog_s = 30.0;
    if (!(r.delta > 0.0)) r.delta = 5.0;
    return r;
}

int default_workgroups() {
    // Number of compute units of the current device if one is visible, else
    // the MI355X count.  Only used for planning; no device work is enqueued.
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        return cus;
    return 256;
}

// The one-shot entry points keep a bounded number of recently used plans
// (least recently used out first).  A call holds its plan through a shared
// pointer, so a plan evicted (or dropped by bb_cache_clear) while another
// thread executes it is destroyed only after that call returns.  The caches
// are never destroyed themselves: plans left in them at exit are not torn
// down after the HIP runtime.
template <class Key, class T>
struct PlanCache {
    std::mutex mu;
    size_t cap;
    std::list<std::pair<Key, std::shared_ptr<T>>> items;   // most recently used first
    explicit PlanCache(size_t c) : cap(c) {}
    std::shared_ptr<T> find(const Key& k) {
        std::lock_guard<std::mutex> lk(mu);
        for (auto it = items.begin(); it != items.end(); ++it)
            if (it->first == k) {
                items.splice(items.begin(), items, it);
                return items.front().second;
            }
        return nullptr;
    }
    // Returns the cached plan for k: v, or one another thread inserted first.
    std::shared_ptr<T> insert(const Key& k, std::shared_ptr<T> v) {
        std::vector<std::shared_ptr<T>> dropped;   // destroyed outside the lock
        std::lock_guard<std::mutex> lk(mu);
        for (auto& kv : items)
            if (kv.first == k) return kv.second;
        items.emplace_front(k, v);
        while (items.size() > cap) {
            dropped.push_back(items.back().second);
            items.pop_back();
        }
        return v;
    }
    void clear() {
        std::list<std::pair<Key, std::shared_ptr<T>>> old;
        {
            std::lock_guard<std::mutex> lk(mu);
            old.swap(items);
        }
    }
};

constexpr size_t kPlanCacheSize = 16, kBatchCacheSize = 4;

PlanCache<std::vector<double>, bb_plan>& plan_cache() {
    static auto* c = new PlanCache<std::vector<double>, bb_plan>(kPlanCacheSize);
    return *c;
}

PlanCache<std::vector<int64_t>, bb_batch>& batch_cache() {
    static auto* c = new PlanCache<std::vector<int64_t>, bb_batch>(kBatchCacheSize);
    return *c;
}

std::vector<double> cache_key(int64_t m, int64_t n, int nb, int tree, int variant, int prec,
                              const bb_opts& o) {
    return {(double)m, (double)n, (double)nb, (double)tree, (double)variant, (double)prec,
            (double)o.workgroups, o.gamma, (double)o.auto_a, (double)o.sched, o.watchdog_s,
            (double)o.flags, (double)o.switch_step, o.delta};
}

// Wait until no copy enqueued from a plan's host memory can still be in
// flight: every device the plan uploaded on is synchronized.
void quiesce(bb_plan& P) {
    const uint32_t mask = P.used_devices.load();
    if (!mask) return;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return;
    for (int d = 0; d < 32; ++d)
        if (mask & (1u << d)) {
            if (d != cur && hipSetDevice(d) != hipSuccess) continue;
            (void)hipDeviceSynchronize();
        }
    (void)hipSetDevice(cur);
}

}  // namespace

bb_batch::~bb_batch() {
    for (Group& g : groups) bb_plan_destroy(g.plan);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
}

extern "C" {

int bb_plan_create(bb_plan** plan, int64_t m, int64_t n, int nb, int tree, int variant, int prec,
                   const bb_opts* opts) {
    if (!plan) return -1;
    *plan = nullptr;
    if (m < 1) return -2;
    if (n < 1) return -3;
    if (nb < 1) return -4;
    if (tree < BB_FLATTS || tree > BB_AUTO) return -5;
    if (variant < BB_BIDIAG || variant > BB_THREESTEP) return -6;
    if (prec != BB_F64 && prec != BB_F64_UPD_F32 && prec != BB_F64_UPD_SPLIT32) return -7;
    if (!bbk::nb_supported(nb)) return BB_ENOTSUP;
    bb_opts o = resolved_opts(opts);
    if (o.sched != BB_SCHED_PERSISTENT && o.sched != BB_SCHED_LEVELS) return -8;
    if (o.workgroups <= 0) o.workgroups = default_workgroups();
    // tile grid of the matrix the graph reduces: A, or A^T when m < n
    const bool tr = m < n;
    int64_t p = ((tr ? n : m) + nb - 1) / nb, q = ((tr ? m : n) + nb - 1) / nb;
    if (p > (1 << 20) || q > (1 << 16)) return BB_ENOTSUP;
    bb_plan* P = new (std::nothrow) bb_plan();
    if (!P) return BB_ENOMEM;
    P->m = m; P->n = n; P->nb = nb; P->tree = tree; P->variant = variant; P->prec = prec;
    P->transposed = tr;
    P->opts = o;
    bb::PlanOptions po;
    po.tree = tree;
    po.variant = variant;
    po.workgroups = o.workgroups;
    po.gamma = o.gamma;
    po.auto_a = o.auto_a;
    po.switch_step = o.switch_step > 0 ? o.switch_step : -1;
    po.delta = o.delta;
    try {
        std::string err = bb::build_graph((int)p, (int)q, po, P->g);
        if (!err.empty()) {
            delete P;
            return BB_EDAG;
        }
        // Static race check of the generated graph before anything runs.
        {
            const size_t nt = P->g.tasks.size();
            std::vector<int32_t> tk(8 * nt), off(nt + 1, 0), idx;
            for (size_t t = 0; t < nt; ++t) {
                const bb::Task& x = P->g.tasks[t];
                int32_t v[8] = {x.kind, x.trans, x.r1, x.c1, x.r2, x.c2, x.slot, x.step};
                std::copy(v, v + 8, tk.begin() + 8 * t);
                for (int32_t pr : P->g.pred[t]) idx.push_back(pr);
                off[t + 1] = (int32_t)idx.size();
            }
            if (!bb::check_graph((int)p, (int)q, (int64_t)nt, tk.data(), off.data(), idx.data()).empty()) {
                delete P;
                return BB_EDAG;
            }
        }
        int rc = finish_plan(*P);
        if (rc != BB_OK) {
            delete P;
            return rc;
        }
    } catch (const std::bad_alloc&) {
        delete P;
        return BB_ENOMEM;
    } catch (...) {
        delete P;
        return BB_EDAG;
    }
    *plan = P;
    return BB_OK;
}

void bb_plan_destroy(bb_plan* P) {
    if (!P) return;
    quiesce(*P);
    for (auto& kv : P->apply) bb_plan_destroy(kv.second);
    delete P->adj;
    if (P->ev0) (void)hipEventDestroy(P->ev0);
    if (P->ev1) (void)hipEventDestroy(P->ev1);
    delete P;
}

int bb_choose(int64_t m, int64_t n, int nb, const bb_opts* opts, int* tree, int* variant, double* estimate) {
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (nb < 1) return -3;
    if (!tree) return -5;
    if (!variant) return -6;
    if (!bbk::nb_supported(nb)) return BB_ENOTSUP;
    bb_opts o = resolved_opts(opts);
    if (o.workgroups <= 0) o.workgroups = default_workgroups();
    const bool tr = m < n;
    const int64_t p = ((tr ? n : m) + nb - 1) / nb, q = ((tr ? m : n) + nb - 1) / nb;
    if (p > (1 << 20) || q > (1 << 16)) return BB_ENOTSUP;
    double best = -1.0;
    try {
        for (int v : {BB_BIDIAG, BB_RBIDIAG, BB_THREESTEP}) {
            if (v == BB_THREESTEP) {
                const int s = bb::three_step_switch((int)p, (int)q, o.delta);
                if (s == 0 || s == (int)q) continue;     // the same graph as R-BiDiag or BiDiag
            }
            for (int t : {BB_GREEDY, BB_AUTO}) {
                bb_plan P;
                P.m = m; P.n = n; P.nb = nb; P.tree = t; P.variant = v; P.prec = BB_F64; P.opts = o;
                bb::PlanOptions po;
                po.tree = t;
                po.variant = v;
                po.workgroups = o.workgroups;
                po.gamma = o.gamma;
                po.auto_a = o.auto_a;
                po.switch_step = -1;
                po.delta = o.delta;
                if (!bb::build_graph((int)p, (int)q, po, P.g).empty()) return BB_EDAG;
                if (build_schedule(P) != BB_OK) return BB_EDAG;
                if (best < 0.0 || P.makespan < best) {
                    best = P.makespan;
                    *tree = t;
                    *variant = v;
                }
            }
        }
    } catch (const std::bad_alloc&) {
        return BB_ENOMEM;
    }
    if (estimate) *estimate = best;
    return BB_OK;
}

void bb_cache_clear(void) {
    plan_cache().clear();
    batch_cache().clear();
}

int bb_plan_workspace(const bb_plan* P, size_t* vt_bytes, size_t* ws_bytes) {
    if (!P) return -1;
    if (vt_bytes) *vt_bytes = vt_bytes_of(*P);
    if (ws_bytes) *ws_bytes = ws_bytes_of(*P);
    return BB_OK;
}

int bb_plan_get_stats(const bb_plan* P, bb_plan_stats* s) {
    if (!P) return -1;
    if (!s) return -2;
    std::memset(s, 0, sizeof(*s));
    s->p = P->g.p;
    s->q = P->g.q;
    s->nb = P->nb;
    s->ntasks = (int64_t)P->g.tasks.size();
    s->nunits = (int64_t)P->units_ticket.size() / 2;
    s->nslots = P->g.nslots;
    s->nlevels = (int64_t)P->level_off.size() - 1;
    for (const bb::Task& t : P->g.tasks) s->count_by_kind[t.kind]++;
    s->critical_path = P->cp;
    s->total_weight = P->total;
    return BB_OK;
}

int bb_plan_export(const bb_plan* P, int32_t* tasks, int32_t* pred_off, int32_t* pred_idx,
                   int64_t* npred) {
    if (!P) return -1;
    int64_t np = 0;
    for (const auto& v : P->g.pred) np += (int64_t)v.size();
    if (npred) *npred = np;
    if (tasks) {
        for (size_t t = 0; t < P->g.tasks.size(); ++t) {
            const bb::Task& s = P->g.tasks[t];
            int32_t* o = tasks + 8 * t;
            o[0] = s.kind; o[1] = s.trans; o[2] = s.r1; o[3] = s.c1;
            o[4] = s.r2; o[5] = s.c2; o[6] = s.slot; o[7] = s.step;
        }
    }
    if (pred_off && pred_idx) {
        int64_t k = 0;
        for (size_t t = 0; t < P->g.tasks.size(); ++t) {
            pred_off[t] = (int32_t)k;
            for (int32_t pr : P->g.pred[t]) pred_idx[k++] = pr;
        }
        pred_off[P->g.tasks.size()] = (int32_t)k;
    }
    return BB_OK;
}

int bb_execute(bb_plan* P, void* A, int64_t lda, void* vt, size_t vt_bytes, void* ws,
               size_t ws_bytes, void* stream) {
    if (!P) return -1;
    if (!A) return -2;
    if (lda < std::max<int64_t>(1, P->m)) return -3;
    if (!vt) return -4;
    if (vt_bytes < vt_bytes_of(*P)) return BB_EWORKSPACE;
    if (!ws) return -6;
    if (ws_bytes < ws_bytes_of(*P)) return BB_EWORKSPACE;
    const bbk::MatDesc d0{(double*)A, lda, P->m, P->n};
    return launch_plan(*P, &d0, vt, ws, stream);
}

int bb_execute_noalloc(bb_plan* P, void* A, int64_t lda, void* vt, size_t vt_bytes, void* stream) {
    if (!P) return -1;
    if (!A) return -2;
    if (lda < std::max<int64_t>(1, P->m)) return -3;
    if (!vt) return -4;
    if (vt_bytes < vt_bytes_of(*P)) return BB_EWORKSPACE;
    if (ws_bytes_of(*P) > (size_t)BB_NOALLOC_WS_MAX) return BB_EWORKSPACE;
    void* ws = nullptr;
    size_t cap = 0;
    if (bbk::noalloc_scratch(&ws, &cap) != hipSuccess) return BB_EHIP;
    if (ws_bytes_of(*P) > cap) return BB_EWORKSPACE;
    const bbk::MatDesc d0{(double*)A, lda, P->m, P->n};
    hipStream_t s = (hipStream_t)stream;
    int rc = upload_graph(*P, ws, s);
    if (rc != BB_OK) return rc;
    return launch_kernels(*P, &d0, vt, ws, s, /*allow_timing=*/false);
}

int bb_apply_workspace(bb_plan* P, int side, int transpose, int64_t ncols, size_t* ws_bytes) {
    if (!P) return -1;
    if (side != 0 && side != 1) return -2;
    if (transpose != 0 && transpose != 1) return -3;
    if (ncols < 0) return -4;
    if (!ws_bytes) return -5;
    if (ncols == 0) {
        *ws_bytes = 0;
        return BB_OK;
    }
    bb_plan* Q = nullptr;
    int rc = get_apply(P, side, transpose, ncols, &Q);
    if (rc != BB_OK) return rc;
    *ws_bytes = ws_bytes_of(*Q);
    return BB_OK;
}

static int apply_side(bb_plan* P, int side, int transpose, const void* vt, size_t vt_bytes, void* C,
                      int64_t ldc, int64_t ncols, void* ws, size_t ws_bytes, void* stream) {
    if (!P) return -1;
    if (transpose != 0 && transpose != 1) return -2;
    if (!vt) return -3;
    if (vt_bytes < vt_bytes_of(*P)) return BB_EWORKSPACE;
    const int64_t rows = side == 0 ? P->m : P->n;
    if (ncols < 0) return -7;
    if (ncols == 0) return BB_OK;
    if (!C) return -5;
    if (ldc < std::max<int64_t>(1, rows)) return -6;
    if (!ws) return -8;
    bb_plan* Q = nullptr;
    int rc = get_apply(P, side, transpose, ncols, &Q);
    if (rc != BB_OK) return rc;
    if (ws_bytes < ws_bytes_of(*Q)) return BB_EWORKSPACE;
    // exact column count: the last tile column is masked
    const bbk::MatDesc d0{(double*)C, ldc, rows, ncols};
    return launch_plan(*Q, &d0, const_cast<void*>(vt), ws, stream);
}

int bb_apply_q(bb_plan* P, int transpose, const void* vt, size_t vt_bytes, void* C, int64_t ldc,
               int64_t ncols, void* ws, size_t ws_bytes, void* stream) {
    return apply_side(P, 0, transpose, vt, vt_bytes, C, ldc, ncols, ws, ws_bytes, stream);
}

int bb_apply_p(bb_plan* P, int transpose, const void* vt, size_t vt_bytes, void* C, int64_t ldc,
               int64_t ncols, void* ws, size_t ws_bytes, void* stream) {
    return apply_side(P, 1, transpose, vt, vt_bytes, C, ldc, ncols, ws, ws_bytes, stream);
}

namespace {

// Workspace of the adjoint: G, G^T (n x n), the Omega and Psi bar grids
// (npad x npad), scratch (npad x 3nb), the inverted diagonal blocks, the copy
// of the operation list, then the state of the two applications (P, then Q),
// each in its own region so that both error words survive the call.
struct AdjLayout {
    size_t g, gt, om, ps, tmp, inv, ops, apply_p, apply_q, total;
};

// Builds (once) the adjoint's operation list and its host copy.
int adjoint_ops(bb_plan* P, const bbk::AdjointOps** out) {
    std::lock_guard<std::mutex> lk(P->adj_mu);
    if (!P->adj) {
        try {
            std::unique_ptr<bbk::AdjointOps> ops(new bbk::AdjointOps());
            bbk::build_adjoint_ops(P->m, P->n, P->nb, *ops);
            const size_t bytes = ops->ops.size() * sizeof(bbk::AOp);
            if (!P->adj_blob.alloc(bytes)) return BB_ENOMEM;
            if (bytes) std::memcpy(P->adj_blob.p, ops->ops.data(), bytes);
            P->adj = ops.release();
        } catch (const std::bad_alloc&) {
            return BB_ENOMEM;
        }
    }
    *out = P->adj;
    return BB_OK;
}

int adjoint_layout(bb_plan* P, AdjLayout& L) {
    const int64_t n = P->n, nb = P->nb;
    const int64_t npad = (n + nb - 1) / nb * nb;
    bb_plan *Qp = nullptr, *Pp = nullptr;
    const bbk::AdjointOps* ops = nullptr;
    int rc = get_apply(P, 1, 0, n, &Pp);
    if (rc != BB_OK) return rc;
    rc = get_apply(P, 0, 0, n, &Qp);
    if (rc != BB_OK) return rc;
    rc = adjoint_ops(P, &ops);
    if (rc != BB_OK) return rc;
    size_t off = 0;
    L.g = off; off = round_up(off + sizeof(double) * n * n, 256);
    L.gt = off; off = round_up(off + sizeof(double) * n * n, 256);
    L.om = off; off = round_up(off + sizeof(double) * npad * npad, 256);
    L.ps = off; off = round_up(off + sizeof(double) * npad * npad, 256);
    L.tmp = off; off = round_up(off + sizeof(double) * npad * 3 * nb, 256);
    L.inv = off; off = round_up(off + sizeof(double) * npad * 2 * nb, 256);
    L.ops = off; off = round_up(off + P->adj_blob.bytes, 256);
    L.apply_p = off; off = round_up(off + ws_bytes_of(*Pp), 256);
    L.apply_q = off; off = round_up(off + ws_bytes_of(*Qp), 256);
    L.total = off;
    return BB_OK;
}

}  // namespace

int bb_adjoint_workspace(bb_plan* P, size_t* ws_bytes) {
    if (!P) return -1;
    if (!ws_bytes) return -2;
    AdjLayout L;
    int rc = adjoint_layout(P, L);
    if (rc != BB_OK) return rc;
    *ws_bytes = L.total;
    return BB_OK;
}

int bidiag_band_adjoint(bb_plan* P, const void* B, int64_t ldb, const void* W, int64_t ldw, const void* vt,
                        size_t vt_bytes, void* Abar, int64_t ldabar, void* ws, size_t ws_bytes, void* stream) {
    if (!P) return -1;
    if (!B) return -2;
    if (ldb < std::max<int64_t>(1, P->m)) return -3;
    if (!W) return -4;
    if (ldw < std::max<int64_t>(1, P->n)) return -5;
    if (!vt) return -6;
    if (vt_bytes < vt_bytes_of(*P)) return BB_EWORKSPACE;
    if (!Abar) return -8;
    if (ldabar < std::max<int64_t>(1, P->m)) return -9;
    if (!ws) return -10;
    if (P->variant == BB_QRONLY) return BB_ENOTSUP;
    if (P->nb > 128) return BB_ENOTSUP;     // the sweep's block solves cover nb <= 128
    if (P->transposed) return BB_ENOTSUP;
    AdjLayout L;
    int rc = adjoint_layout(P, L);
    if (rc != BB_OK) return rc;
    if (ws_bytes < L.total) return BB_EWORKSPACE;
    const bbk::AdjointOps* opsp = nullptr;
    if ((rc = adjoint_ops(P, &opsp)) != BB_OK) return rc;
    const bbk::AdjointOps& ops = *opsp;
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)ws;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return BB_EHIP;
    if (dev < 32) P->used_devices.fetch_or(1u << dev);
    if (hipMemcpyAsync(w + L.ops, P->adj_blob.p, P->adj_blob.bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return BB_EHIP;
    const int64_t n = P->n, npad = ops.npad;
    bbk::AArgs a{};
    a.buf[bbk::AB_B] = {(double*)B, ldb};
    a.buf[bbk::AB_W] = {(double*)W, ldw};
    a.buf[bbk::AB_G] = {(double*)(w + L.g), n};
    a.buf[bbk::AB_GT] = {(double*)(w + L.gt), n};
    a.buf[bbk::AB_OM] = {(double*)(w + L.om), npad};
    a.buf[bbk::AB_PS] = {(double*)(w + L.ps), npad};
    a.buf[bbk::AB_TMP] = {(double*)(w + L.tmp), npad};
    a.buf[bbk::AB_ABAR] = {(double*)Abar, ldabar};
    a.buf[bbk::AB_INV] = {(double*)(w + L.inv), npad};
    const bbk::AOp* dops = (const bbk::AOp*)(w + L.ops);
    auto run_stages = [&](int32_t s0, int32_t s1) -> int {
        for (int32_t st = s0; st < s1; ++st) {
            const int32_t o0 = ops.stage_off[st], o1 = ops.stage_off[st + 1];
            if (bbk::launch_adjoint_stage(a, dops, o0, o1, ops.ops[o0].kind, ops.stage_m[st], ops.stage_n[st], s) !=
                hipSuccess)
                return BB_EHIP;
        }
        return BB_OK;
    };
    const int32_t nst = (int32_t)ops.stage_off.size() - 1;
    rc = run_stages(0, ops.finish_stage);
    if (rc != BB_OK) return rc;
    bb_plan *Pp = nullptr, *Qp = nullptr;
    if ((rc = get_apply(P, 1, 0, n, &Pp)) != BB_OK) return rc;
    if ((rc = get_apply(P, 0, 0, n, &Qp)) != BB_OK) return rc;
    const bbk::MatDesc dP{(double*)(w + L.gt), n, n, n};
    if ((rc = launch_plan(*Pp, &dP, const_cast<void*>(vt), w + L.apply_p, stream)) != BB_OK) return rc;
    rc = run_stages(ops.finish_stage, nst);
    if (rc != BB_OK) return rc;
    const bbk::MatDesc dQ{(double*)Abar, ldabar, P->m, n};
    return launch_plan(*Qp, &dQ, const_cast<void*>(vt), w + L.apply_q, stream);
}

int bb_adjoint_poll_error(bb_plan* P, const void* ws, void* stream, int* device_status) {
    if (!P) return -1;
    if (!ws) return -2;
    if (!device_status) return -4;
    AdjLayout L;
    int rc = adjoint_layout(P, L);
    if (rc != BB_OK) return rc;
    *device_status = 0;
    for (size_t off : {L.apply_p, L.apply_q}) {
        int st = 0;
        rc = bb_poll_error((const char*)ws + off, stream, &st);
        if (rc != BB_OK) return rc;
        if (st != 0) {
            *device_status = st;
            break;
        }
    }
    return BB_OK;
}

int bb_plan_trace(bb_plan* P, size_t* offset, int64_t* nunits, double* tick_hz, int32_t* units) {
    if (!P) return -1;
    if (!(P->opts.flags & BB_FLAG_TRACE)) return BB_ENOTSUP;
    if (offset) *offset = ws_trace_off(*P);
    if (nunits) *nunits = (int64_t)(P->units_ticket.size() / 2);
    if (tick_hz) *tick_hz = 1000.0 * (double)device_attr(hipDeviceAttributeWallClockRate, 100000);
    if (units) std::copy(P->units_prio.begin(), P->units_prio.end(), units);
    return BB_OK;
}

int bb_plan_last_kernel_ms(bb_plan* P, double* ms) {
    if (!P) return -1;
    if (!ms) return -2;
    if (!P->timed || !P->ev0) return BB_ENOTSUP;
    if (hipEventSynchronize(P->ev1) != hipSuccess) return BB_EHIP;
    float f = 0.f;
    if (hipEventElapsedTime(&f, P->ev0, P->ev1) != hipSuccess) return BB_EHIP;
    *ms = (double)f;
    return BB_OK;
}

namespace {

// The cached plan of the one-shot entry points for these arguments, built
// on first use.  Returns BB_OK or bb_plan_create's code.
int cached_plan(int64_t m, int64_t n, int nb, int tree, int variant, int prec, const bb_opts& o,
                std::shared_ptr<bb_plan>& out) {
    std::vector<double> key = cache_key(m, n, nb, tree, variant, prec, o);
    out = plan_cache().find(key);
    if (out) return BB_OK;
    bb_plan* P = nullptr;
    int rc = bb_plan_create(&P, m, n, nb, tree, variant, prec, &o);
    if (rc != BB_OK) return rc;
    try {
        out = plan_cache().insert(key, std::shared_ptr<bb_plan>(P, bb_plan_destroy));
    } catch (const std::bad_alloc&) {
        return BB_ENOMEM;
    }
    return BB_OK;
}

}  // namespace

int bb_query(int64_t m, int64_t n, int nb, int tree, int variant, int prec, const bb_opts* opts,
             size_t* vt_bytes, size_t* ws_bytes) {
    std::shared_ptr<bb_plan> P;
    int rc = cached_plan(m, n, nb, tree, variant, prec, resolved_opts(opts), P);
    if (rc != BB_OK) return rc;
    bb_plan_workspace(P.get(), vt_bytes, ws_bytes);
    return BB_OK;
}

int bidiag_band(void* A, int64_t m, int64_t n, int64_t lda, int nb, int tree, int variant, int prec,
                void* vt, size_t vt_bytes, void* ws, size_t ws_bytes, const bb_opts* opts,
                void* stream) {
    if (!A) return -1;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (!vt) return -9;
    if (!ws) return -11;
    std::shared_ptr<bb_plan> P;
    int rc = cached_plan(m, n, nb, tree, variant, prec, resolved_opts(opts), P);
    if (rc != BB_OK) {
        // map plan-creation argument numbers onto this entry point's
        if (rc < 0) {
            static const int remap[9] = {0, 0, -2, -3, -5, -6, -7, -8, -13};
            return rc >= -8 ? remap[-rc] : rc;
        }
        return rc;
    }
    rc = bb_execute(P.get(), A, lda, vt, vt_bytes, ws, ws_bytes, stream);
    if (rc == -3) return -4;
    if (rc == -4) return -9;
    if (rc == -6) return -11;
    return rc;
}

int bb_poll_error(const void* ws, void* stream, int* device_status) {
    if (!device_status) return -3;
    if (!ws) {
        // the workspace of bb_execute_noalloc on the current device
        void* p = nullptr;
        size_t cap = 0;
        if (bbk::noalloc_scratch(&p, &cap) != hipSuccess) return BB_EHIP;
        ws = p;
    }
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return BB_EHIP;
    int32_t e = 0;
    if (hipMemcpy(&e, (const char*)ws + sizeof(int32_t) * bbk::CTRL_ERROR, sizeof(int32_t),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return BB_EHIP;
    *device_status = e;
    return BB_OK;
}

int bb_graph_check(int p, int q, int64_t ntasks, const int32_t* tasks, const int32_t* pred_off,
                   const int32_t* pred_idx) {
    if (q < 1 || p < q) return -1;
    if (ntasks < 0) return -3;
    if (ntasks > 0 && (!tasks || !pred_off || (!pred_idx && pred_off[ntasks] > 0))) return -4;
    try {
        return bb::check_graph(p, q, ntasks, tasks, pred_off, pred_idx).empty() ? BB_OK : BB_EDAG;
    } catch (...) {
        return BB_ENOMEM;
    }
}

int bb_plan_auto_domains(const bb_plan* P, int32_t* a, int64_t* nsteps) {
    if (!P) return -1;
    if (nsteps) *nsteps = (int64_t)P->g.auto_a_used.size();
    if (a)
        for (size_t k = 0; k < P->g.auto_a_used.size(); ++k) a[k] = P->g.auto_a_used[k];
    return BB_OK;
}

double bb_critical_path(int p, int q, int tree, int variant, int auto_a, int workgroups,
                        double gamma) {
    if (q < 1 || p < q) return -1.0;
    bb::PlanOptions po;
    po.tree = tree;
    po.variant = variant;
    po.auto_a = auto_a;
    po.workgroups = workgroups > 0 ? workgroups : 256;
    po.gamma = gamma > 0.0 ? gamma : 2.0;
    bb::Graph g;
    try {
        if (!bb::build_graph(p, q, po, g).empty()) return -1.0;
    } catch (...) {
        return -1.0;
    }
    return bb::critical_path(g, bb::kTable1Weights);
}

int bb_tuned_config(int64_t m, int64_t n, int prec, int* nb, int* tree, int* variant) {
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (prec != BB_F64 && prec != BB_F64_UPD_F32 && prec != BB_F64_UPD_SPLIT32) return -3;
    if (!nb || !tree || !variant) return -4;
    if (m < n) return BB_ENOTSUP;
    const int64_t r = (1000 * n + m - 1) / m;      // ceil(1000 n / m), in (0, 1000]
    const int* best = kTunedTable[0];
    for (const auto& row : kTunedTable) {
        if (m >= row[0] && m < row[1] && r > row[2] && r <= row[3]) {
            best = row;
            break;
        }
    }
    *nb = best[4];
    *tree = best[5];
    *variant = best[6];
    return BB_OK;
}

int bb_batch_create(bb_batch** batch, int64_t count, const int64_t* m, const int64_t* n, const int* nb,
                    const int* tree, const int* variant, int prec, const bb_opts* opts) {
    if (!batch) return -1;
    *batch = nullptr;
    if (count < 0 || count > (1 << 24)) return -2;
    if (count > 0 && !m) return -3;
    if (count > 0 && !n) return -4;
    if (prec != BB_F64 && prec != BB_F64_UPD_F32 && prec != BB_F64_UPD_SPLIT32) return -8;
    bb_opts o = resolved_opts(opts);
    if (o.sched != BB_SCHED_PERSISTENT && o.sched != BB_SCHED_LEVELS) return -9;
    if (o.workgroups <= 0) o.workgroups = default_workgroups();
    bb_batch* B = new (std::nothrow) bb_batch();
    if (!B) return BB_ENOMEM;
    B->count = count;
    B->prec = prec;
    B->opts = o;
    try {
        B->m.assign(m, m + count);
        B->n.assign(n, n + count);
        B->nb.resize(count);
        B->tree.resize(count);
        B->variant.resize(count);
        for (int64_t i = 0; i < count; ++i) {
            if (B->m[i] < 1 || B->n[i] < 1) { delete B; return -3; }
            if (B->m[i] < B->n[i]) { delete B; return BB_ENOTSUP; }
            if (!nb || nb[i] == 0) {
                bb_tuned_config(B->m[i], B->n[i], prec, &B->nb[i], &B->tree[i], &B->variant[i]);
            } else {
                B->nb[i] = nb[i];
                B->tree[i] = tree ? tree[i] : BB_GREEDY;
                B->variant[i] = variant ? variant[i] : BB_BIDIAG;
            }
            if (!bbk::nb_supported(B->nb[i])) { delete B; return BB_ENOTSUP; }
            if (B->tree[i] < BB_FLATTS || B->tree[i] > BB_AUTO) { delete B; return -6; }
            if (B->variant[i] < BB_BIDIAG || B->variant[i] > BB_THREESTEP) { delete B; return -7; }
            if ((B->m[i] + B->nb[i] - 1) / B->nb[i] > (1 << 20)) { delete B; return BB_ENOTSUP; }
        }
        B->rec_off.assign(count, 0);
        B->nrec.assign(count, 0);
        const size_t wsg = 256;
        // Tile sizes 32 .. 128 share one launch when the batch holds more
        // than one of them (tasks carry their size); nb = 256 runs apart.
        std::vector<std::vector<int>> sets;
        {
            bool has[4] = {false, false, false, false};
            for (int64_t i = 0; i < count; ++i)
                has[B->nb[i] == 32 ? 0 : B->nb[i] == 64 ? 1 : B->nb[i] == 128 ? 2 : 3] = true;
            const int small = (int)has[0] + (int)has[1] + (int)has[2];
            if (small > 1) sets.push_back({32, 64, 128});
            else
                for (int k = 0; k < 3; ++k)
                    if (has[k]) sets.push_back({32 << k});
            if (has[3]) sets.push_back({256});
        }
        for (const std::vector<int>& set : sets) {
            std::vector<int64_t> idx;
            for (int64_t i = 0; i < count; ++i)
                if (std::find(set.begin(), set.end(), B->nb[i]) != set.end()) idx.push_back(i);
            bb_plan* P = new bb_plan();
            bb_batch::Group grp;
            grp.nb = set.size() > 1 ? bbk::NB_MIXED : set[0];
            grp.plan = P;
            B->groups.push_back(grp);       // owned by B from here on
            P->nb = grp.nb;
            P->prec = prec;
            P->opts = o;
            P->nmats = (int32_t)idx.size();
            P->gidx = idx;
            P->dims.resize(2 * idx.size());
            P->slot_base.resize(idx.size());
            P->recoff.resize(idx.size());
            if (P->nb == bbk::NB_MIXED) P->mat_nb.resize(idx.size());
            int64_t rec_doubles = 0;
            for (size_t li = 0; li < idx.size(); ++li) {
                const int64_t i = idx[li];
                const int tile = B->nb[i];
                P->dims[2 * li] = B->m[i];
                P->dims[2 * li + 1] = B->n[i];
                bb::PlanOptions po;
                po.tree = B->tree[i];
                po.variant = B->variant[i];
                po.workgroups = o.workgroups;
                po.gamma = o.gamma;
                po.auto_a = o.auto_a;
                po.switch_step = o.switch_step > 0 ? o.switch_step : -1;
                po.delta = o.delta;
                const int p = (int)((B->m[i] + tile - 1) / tile), q = (int)((B->n[i] + tile - 1) / tile);
                bb::Graph gi;
                if (!bb::build_graph(p, q, po, gi).empty()) { delete B; return BB_EDAG; }
                {
                    const size_t nt = gi.tasks.size();
                    std::vector<int32_t> tk(8 * nt), off(nt + 1, 0), pidx;
                    for (size_t t = 0; t < nt; ++t) {
                        const bb::Task& x = gi.tasks[t];
                        int32_t v[8] = {x.kind, x.trans, x.r1, x.c1, x.r2, x.c2, x.slot, x.step};
                        std::copy(v, v + 8, tk.begin() + 8 * t);
                        for (int32_t pr : gi.pred[t]) pidx.push_back(pr);
                        off[t + 1] = (int32_t)pidx.size();
                    }
                    if (!bb::check_graph(p, q, (int64_t)nt, tk.data(), off.data(), pidx.data()).empty()) {
                        delete B;
                        return BB_EDAG;
                    }
                }
                B->nrec[i] = gi.nslots;
                B->rec_off[i] = rec_doubles * (int64_t)sizeof(double);   // within the group
                P->slot_base[li] = P->g.nslots;
                P->recoff[li] = rec_doubles;
                if (!P->mat_nb.empty()) P->mat_nb[li] = tile;
                rec_doubles += (int64_t)gi.nslots * bbk::record_doubles(tile);
                bb::append_graph(P->g, gi, (int32_t)li);
                if (P->g.tasks.size() > (size_t)INT32_MAX / 2) { delete B; return BB_ENOTSUP; }
            }
            P->vt_doubles = rec_doubles;
            int rc = finish_plan(*P);
            if (rc != BB_OK) { delete B; return rc; }
        }
        size_t vt_off = 0, ws_off = 0;
        for (bb_batch::Group& grp : B->groups) {
            grp.vt_off = vt_off;
            grp.ws_off = ws_off;
            vt_off = round_up(vt_off + vt_bytes_of(*grp.plan), 256);
            ws_off = round_up(ws_off + ws_bytes_of(*grp.plan), wsg);
            for (size_t li = 0; li < grp.plan->gidx.size(); ++li)
                B->rec_off[grp.plan->gidx[li]] += (int64_t)grp.vt_off;
        }
        B->vt_bytes = vt_off;
        B->ws_bytes = ws_off;
    } catch (const std::bad_alloc&) {
        delete B;
        return BB_ENOMEM;
    } catch (...) {
        delete B;
        return BB_EDAG;
    }
    *batch = B;
    return BB_OK;
}

void bb_batch_destroy(bb_batch* B) { delete B; }

int bb_batch_workspace(const bb_batch* B, size_t* vt_bytes, size_t* ws_bytes) {
    if (!B) return -1;
    if (vt_bytes) *vt_bytes = B->vt_bytes;
    if (ws_bytes) *ws_bytes = B->ws_bytes;
    return BB_OK;
}

int bb_batch_info(const bb_batch* B, int64_t i, int* nb, int* tree, int* variant, int64_t* rec_offset,
                  int64_t* nrec) {
    if (!B) return -1;
    if (i < 0 || i >= B->count) return -2;
    if (nb) *nb = B->nb[i];
    if (tree) *tree = B->tree[i];
    if (variant) *variant = B->variant[i];
    if (rec_offset) *rec_offset = B->rec_off[i];
    if (nrec) *nrec = B->nrec[i];
    return BB_OK;
}

int bb_batch_execute(bb_batch* B, double* const* A, const int64_t* lda, void* vt, size_t vt_bytes,
                     void* ws, size_t ws_bytes, void* stream) {
    if (!B) return -1;
    if (B->count == 0) return BB_OK;
    if (!A) return -2;
    if (!lda) return -3;
    if (!vt) return -4;
    if (vt_bytes < B->vt_bytes) return BB_EWORKSPACE;
    if (!ws) return -6;
    if (ws_bytes < B->ws_bytes) return BB_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const bool timed = (B->opts.flags & BB_FLAG_TIMING) != 0;
    if (timed) {
        std::call_once(B->ev_once, [B] {
            if (hipEventCreate(&B->ev0) != hipSuccess || hipEventCreate(&B->ev1) != hipSuccess)
                B->ev_err = hipErrorInvalidValue;
        });
        if (B->ev_err != hipSuccess) return BB_EHIP;
    }
    // Every group's graph and descriptors first, so that the timed region
    // holds the reduction kernels only.
    for (bb_batch::Group& grp : B->groups) {
        bb_plan& P = *grp.plan;
        char* w = (char*)ws + grp.ws_off;
        int rc = upload_graph(P, w, s);
        if (rc != BB_OK) return rc;
        char* blob = w + ws_blob_off(P);
        if (bbk::launch_batch_desc((bbk::MatDesc*)(w + ws_mats_off()), P.nmats,
                                   (const int64_t*)(blob + P.off_gidx), (const int64_t*)(blob + P.off_dims),
                                   (const int64_t*)(blob + P.off_recoff), A, lda, (double*)((char*)vt + grp.vt_off),
                                   s) != hipSuccess)
            return BB_EHIP;
    }
    if (timed && hipEventRecord(B->ev0, s) != hipSuccess) return BB_EHIP;
    for (bb_batch::Group& grp : B->groups) {
        int rc = launch_kernels(*grp.plan, nullptr, (char*)vt + grp.vt_off, (char*)ws + grp.ws_off, s);
        if (rc != BB_OK) return rc;
    }
    if (timed && hipEventRecord(B->ev1, s) != hipSuccess) return BB_EHIP;
    B->timed = timed;
    return BB_OK;
}

int bb_batch_last_kernel_ms(bb_batch* B, double* ms) {
    if (!B) return -1;
    if (!ms) return -2;
    if (!B->timed || !B->ev0) return BB_ENOTSUP;
    if (hipEventSynchronize(B->ev1) != hipSuccess) return BB_EHIP;
    float f = 0.f;
    if (hipEventElapsedTime(&f, B->ev0, B->ev1) != hipSuccess) return BB_EHIP;
    *ms = (double)f;
    return BB_OK;
}

int bb_batch_poll_error(const bb_batch* B, const void* ws, void* stream, int* device_status) {
    if (!B) return -1;
    if (!ws) return -2;
    if (!device_status) return -4;
    *device_status = 0;
    for (const bb_batch::Group& grp : B->groups) {
        int st = 0;
        int rc = bb_poll_error((const char*)ws + grp.ws_off, stream, &st);
        if (rc != BB_OK) return rc;
        if (st != 0) {
            *device_status = st;
            break;
        }
    }
    return BB_OK;
}

int bb_query_batched(int64_t count, const int64_t* m, const int64_t* n, const int* nb, const int* tree,
                     const int* variant, int prec, const bb_opts* opts, size_t* vt_bytes, size_t* ws_bytes) {
    bb_batch* B = nullptr;
    int rc = bb_batch_create(&B, count, m, n, nb, tree, variant, prec, opts);
    if (rc != BB_OK) return rc < 0 ? rc + 1 : rc;
    bb_batch_workspace(B, vt_bytes, ws_bytes);
    bb_batch_destroy(B);
    return BB_OK;
}

int bidiag_band_batched(double* const* A, const int64_t* lda, int64_t count, const int64_t* m,
                        const int64_t* n, const int* nb, const int* tree, const int* variant, int prec,
                        void* vt, size_t vt_bytes, void* ws, size_t ws_bytes, const bb_opts* opts,
                        void* stream) {
    if (count < 0) return -3;
    if (count == 0) return BB_OK;
    if (!A) return -1;
    if (!lda) return -2;
    if (!m) return -4;
    if (!n) return -5;
    bb_opts o = resolved_opts(opts);
    std::vector<int64_t> key;
    try {
        key.reserve(5 * (size_t)count + 8);
        key.push_back(prec);
        key.push_back(o.workgroups);
        key.push_back((int64_t)(o.gamma * 1e6));
        key.push_back(o.auto_a);
        key.push_back(o.sched);
        key.push_back((int64_t)(o.watchdog_s * 1e3));
        key.push_back(o.flags);
        key.push_back(o.switch_step);
        key.push_back((int64_t)(o.delta * 1e6));
        for (int64_t i = 0; i < count; ++i) {
            key.push_back(m[i]);
            key.push_back(n[i]);
            key.push_back(nb ? nb[i] : 0);
            key.push_back(tree ? tree[i] : -1);
            key.push_back(variant ? variant[i] : -1);
        }
    } catch (const std::bad_alloc&) {
        return BB_ENOMEM;
    }
    std::shared_ptr<bb_batch> B = batch_cache().find(key);
    if (!B) {
        bb_batch* b = nullptr;
        int rc = bb_batch_create(&b, count, m, n, nb, tree, variant, prec, &o);
        if (rc != BB_OK) {
            if (rc < 0) {
                // bb_batch_create numbering -> this entry point's
                static const int remap[10] = {0, 0, -3, -4, -5, -6, -7, -8, -9, -14};
                return rc >= -9 ? remap[-rc] : rc;
            }
            return rc;
        }
        try {
            B = batch_cache().insert(key, std::shared_ptr<bb_batch>(b, bb_batch_destroy));
        } catch (const std::bad_alloc&) {
            return BB_ENOMEM;
        }
    }
    int rc = bb_batch_execute(B.get(), A, lda, vt, vt_bytes, ws, ws_bytes, stream);
    switch (rc) {
    case -2: return -1;
    case -3: return -2;
    case -4: return -10;
    case -6: return -12;
    default: return rc;
    }
}

const char* bb_strerror(int code) {
    if (code < 0) return "invalid argument";
    switch (code) {
    case BB_OK: return "success";
    case BB_ENOTSUP: return "unsupported request";
    case BB_EHIP: return "HIP runtime error";
    case BB_ETIMEOUT: return "device scheduler watchdog expired";
    case BB_EDAG: return "task graph failed validation";
    case BB_ENOMEM: return "out of memory";
    case BB_EWORKSPACE: return "workspace too small";
    default: return "unknown error";
    }
}

}  // extern "C"
