// gfx950 kernels of the tiled band bidiagonalization.
//
// Every task of the graph is one tile kernel of Table 1 (Section 3.2):
//   panel  : GEQRT (factor a square tile into a triangle), TSQRT (zero a square
//            tile below a triangle), TTQRT (zero a triangle below a triangle);
//   update : UNMQR, TSMQR, TTMQR (apply those reflectors to a trailing tile or
//            tile pair).
// LQ steps use the same kernels on transposed tiles (Section 3.4, Algorithm 4):
// each task carries a transpose flag and all arithmetic is written in a
// "logical" frame where logical element (r, c) of a tile is physical element
// (r, c) for QR steps and (c, r) for LQ steps.
//
// Reflector convention (the LAPACK/PLASMA kernels the paper builds on): for
// x = (alpha, x_tail), beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta,
// v = (1, x_tail/(alpha - beta)); tau = 0 when x_tail == 0.  The k reflectors
// of a panel are kept in compact WY form Q = H_1 ... H_k = I - V T V^T with T
// upper triangular, and an update applies Q^T: C <- C - V T^T V^T C.
//
// One workgroup of 512 threads (8 wave64, two per SIMD) executes one work
// unit.  Panels are blocked by 16 columns (a register-resident leaf on four
// waves plus MFMA trailing updates on all eight); updates apply the 16-column
// blocks of a panel's reflectors with FP64 MFMA (v_mfma_f64_16x16x4) to
// register-resident 16-column slices of the trailing tile(s), one slice per
// wave.  Two waves per SIMD let one wave's MFMA chain run while the other
// waits on a dependency.
#include <mutex>
#include <type_traits>

#include "../../include/bidiag.h"
#include "kernels.hpp"

namespace bbk {

namespace {

constexpr int NT = 512;          // threads per workgroup
typedef double d4 __attribute__((ext_vector_type(4)));

enum : int { K_GEQRT = 0, K_TSQRT = 1, K_TTQRT = 2, K_UNMQR = 3, K_TSMQR = 4, K_TTMQR = 5, K_HQ = 3 };

template <int NB>
struct Shape {
    static constexpr int MT = NB / 16;                 // 16 x 16 tiles per tile side
    static constexpr int LDL = NB + 1;                 // LDS stride of the leaf (odd: conflict-free)
    // doubles used by a panel: leaf buffer(s) (two at nb = 256), then the
    // reflector broadcast, taus, G, T_b and R1's diagonal entries
    // (nb = 256: two leaf buffers, the block's reflector ring, taus, G, two
    // T_b and the role counters)
    static constexpr int PANEL = NB > 128 ? 32 * LDL + 16 * NB + 16 + 256 + 512 + 2048 + 4
                                          : 16 * LDL + 2 * NB + 16 + 768;
    static constexpr int UPDATE = 2 * (16 * LDL + 256);           // ... and by an update
    static constexpr int LDS = PANEL > UPDATE ? PANEL : UPDATE;
};

// Keeps the scheduler from hoisting loads of later 16-row steps of a fully
// unrolled product above this point (bounds register pressure).
#define SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)

// Workgroup barrier that orders LDS only.  The tile kernels exchange data
// between waves through LDS alone; their global stores (outputs) are not read
// back by the same workgroup, so barriers need not wait for them.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Global store of a task output.  CO (coherent outputs) selects agent-scope
// stores, which are made coherent across the L2s of all XCDs as they
// complete; the persistent scheduler uses them so that finishing a task needs
// only a wait for its stores instead of an L2 write-back.
// Matrix tiles and records are global memory.  Accessing them through
// global-address-space pointers (not generic ones) keeps them off the LDS
// counter, so LDS waits in the products do not also wait for global loads.
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ gdouble* gptr(double* p) { return (gdouble*)p; }

template <bool CO>
__device__ __forceinline__ void gstore(double* p, double v) {
    gdouble* q = gptr(p);
    if (CO) __hip_atomic_store(q, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *q = v;
}

// A tile seen in the logical frame.  vr/vc: logical rows/columns that exist in
// the matrix (the rest of the nb x nb tile is zero padding, never accessed).
struct TileView {
    double* base;
    int64_t ld;
    int trans, vr, vc;
    __device__ __forceinline__ double* ptr(int r, int c) const {
        return trans ? base + c + (int64_t)r * ld : base + r + (int64_t)c * ld;
    }
    __device__ __forceinline__ double get(int r, int c) const {
        return (r < vr && c < vc) ? *gptr(ptr(r, c)) : 0.0;
    }
    template <bool CO>
    __device__ __forceinline__ void put(int r, int c, double v) const {
        if (r < vr && c < vc) gstore<CO>(ptr(r, c), v);
    }
};

// Descriptor of the task's matrix.  A single-matrix launch carries it in the
// kernel arguments.  A batched launch reads it from the workspace, where an
// earlier kernel of the stream wrote it: the loads are agent-scope atomics,
// so no cache level can serve a value left there by an earlier launch that
// used the same workspace.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ MatDesc mat_desc(const KArgs& a, int mat) {
    if (a.mats == nullptr) return a.single;
    const uint64_t* w = reinterpret_cast<const uint64_t*>(a.mats + mat);
    uint64_t f[5];
#pragma unroll
    for (int k = 0; k < 5; ++k)
        f[k] = uniform64(__hip_atomic_load(w + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    MatDesc d;
    d.A = reinterpret_cast<double*>(f[0]);
    d.lda = (int64_t)f[1];
    d.m = (int64_t)f[2];
    d.n = (int64_t)f[3];
    d.rec = reinterpret_cast<double*>(f[4]);
    return d;
}

// The V/T record of a task (slot within its matrix's records).
template <int NB>
__device__ __forceinline__ double* record(const MatDesc& d, const DevTask& tk) {
    return d.rec + (int64_t)tk.slot * (int64_t)(NB * NB + 16 * NB);
}

__device__ __forceinline__ TileView view(const MatDesc& d, const DevTask& tk, int pr, int pc, int nb) {
    const int trans = tk.trans & 1;
    TileView t;
    t.base = d.A + (int64_t)pr * nb + (int64_t)pc * nb * d.lda;
    t.ld = d.lda;
    t.trans = trans;
    int prow = (int)min((int64_t)nb, d.m - (int64_t)pr * nb);
    int pcol = (int)min((int64_t)nb, d.n - (int64_t)pc * nb);
    t.vr = trans ? pcol : prow;
    t.vc = trans ? prow : pcol;
    return t;
}

// Register ("accumulator") layout of a 16-column slice of a tile, shared by
// every MFMA of this file: element r (0..3) of lane l of row tile i holds
// logical (16 i + 4 r + l/16, c0 + l%16).  That is the result layout of
// v_mfma_f64_16x16x4, and element r of row tile i is also exactly the second
// operand of the k-step covering rows 16 i + 4 r .. 16 i + 4 r + 3, so a slice
// held this way feeds the next product without any data movement.
template <int MT>
__device__ __forceinline__ void load_slice(const TileView& t, int c0, d4 (&x)[MT]) {
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[i][r] = t.get(16 * i + 4 * r + g, c0 + j);
}

template <bool CO, int MT>
__device__ __forceinline__ void store_slice(const TileView& t, int c0, const d4 (&x)[MT]) {
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) t.put<CO>(16 * i + 4 * r + g, c0 + j, x[i][r]);
}

__device__ __forceinline__ d4 load16(const TileView& t, int r0, int c0) {
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    d4 x;
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = t.get(r0 + 4 * r + g, c0 + j);
    return x;
}

template <bool CO>
__device__ __forceinline__ void store16(const TileView& t, int r0, int c0, d4 x) {
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) t.put<CO>(r0 + 4 * r + g, c0 + j, x[r]);
}

// Whole-vector accesses of 32 bytes (global memory).
typedef __attribute__((address_space(1))) d4 gd4;
__device__ __forceinline__ d4 load_d4(const double* p) { return *(const gd4*)p; }
__device__ __forceinline__ void store_d4(double* p, d4 v) { *(gd4*)p = v; }

// Reads of one V/T record through a buffer descriptor: every load of a
// product shares one per-lane byte offset and adds a wave-uniform constant,
// so unrolled products need no per-load address registers.  Reads past the
// record's end return zero.
struct Rec {
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ Rec(const double* base, int nb) {
        rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0,
                                                 (int)(8 * (nb * nb + 16 * nb)), 0x00020000);
    }
    __device__ __forceinline__ double ld(int voff, int soff) const {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff, soff, 0));
    }
};

// Cross-lane move inside rows of 16 lanes (DPP), on both halves of a double.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}

// Sum over the 16 lanes of a DPP row (lanes l with equal l/16): swap with
// lane^1 and lane^2 (quad permutes), then with the mirrored lane in the half
// row and in the row.  Every lane ends with the same bits (each step adds two
// equal partial sums in either order).  All 16 lanes of the row must be active.
__device__ __forceinline__ double sum16(double v) {
    v += dpp<0xB1>(v);     // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);     // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);    // row_half_mirror
    v += dpp<0x140>(v);    // row_mirror
    return v;
}

// sqrt(t) and 1/x for positive normal t and nonzero normal x, from the
// hardware approximations (v_rsq_f64, v_rcp_f64):
//  - sqrt: one step of Goldschmidt's coupled iteration for s ~ sqrt(t) and
//    h ~ 1/(2 sqrt(t)) (residual e = 1/2 - h s, then s += s e, h += h e),
//    followed by two Newton-Raphson corrections s += h (t - s^2);
//  - 1/x: two Newton-Raphson steps r += r (1 - x r).
// Both end within an ulp, without the special-value and scaling paths of the
// IEEE library forms, which the Householder steps never need.
__device__ __forceinline__ double refined_sqrt(double t) {
    const double r = __builtin_amdgcn_rsq(t);
    double s = t * r, h = 0.5 * r;
    const double e = fma(-h, s, 0.5);
    s = fma(s, e, s);
    h = fma(h, e, h);
    double d = fma(-s, s, t);
    s = fma(d, h, s);
    d = fma(-s, s, t);
    return fma(d, h, s);
}

__device__ __forceinline__ double refined_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Value of lane `src` (wave-uniform) of a double.
__device__ __forceinline__ double readlane64(double v, int src) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}

// The unit a workgroup of the persistent scheduler finished last, whose
// output stores may still be in flight.  The next unit retires it once its own
// first loads are issued, so that the store drain and the load latency
// overlap: every wave waits for all of its memory operations, then thread 0
// counts the unit as done.
struct Prev {
    int task;                      // -1: nothing to retire
    int ticket;
    uint64_t wait, run, end;       // trace times of the finished unit
};

__device__ __forceinline__ int aload(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0, after the unit's outputs are complete: count down the
// successors' dependency counters, then count the unit as done.
__device__ __forceinline__ void complete_unit(const KArgs& a, int task) {
    const int s0 = a.succ_off[task], s1 = a.succ_off[task + 1];
    for (int e = s0; e < s1; ++e)
        __hip_atomic_fetch_add(&a.deps[a.succ_idx[e]], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&a.ctrl[CTRL_DONE], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by all 64 lanes of wave 0 (the results are the same in every lane).
// take_ticket: the next priority position, or -1 when all are taken.
// unit_ready: whether that unit's task has no unfinished predecessor now.
// wait_unit: wait until it has none; returns the ticket, or -1 to stop.
__device__ __forceinline__ int take_ticket(const KArgs& a, int lane) {
    int u = 0;
    if (lane == 0)
        u = __hip_atomic_fetch_add(&a.ctrl[CTRL_HEAD], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    u = __builtin_amdgcn_readfirstlane(u);
    return u >= a.nunits ? -1 : u;
}

__device__ __forceinline__ bool unit_ready(const KArgs& a, int u, int lane) {
    const int task = __builtin_amdgcn_readfirstlane(a.units[u].x);
    int d = 0;
    if (lane == 0) d = aload(&a.deps[task]);
    return __builtin_amdgcn_readfirstlane(d) <= 0;
}

__device__ __forceinline__ int wait_unit(const KArgs& a, int u, int lane) {
    const int task = __builtin_amdgcn_readfirstlane(a.units[u].x);
    const uint64_t t0 = wall_clock64();
    for (;;) {
        int d = 0, err = 0;
        if (lane == 0) {
            d = aload(&a.deps[task]);
            if (d > 0) err = aload(&a.ctrl[CTRL_ERROR]);
        }
        d = __builtin_amdgcn_readfirstlane(d);
        if (d <= 0) return u;
        if (__builtin_amdgcn_readfirstlane(err) != 0) return -1;
        if ((int64_t)(wall_clock64() - t0) > a.watchdog_ticks) {
            if (lane == 0) __hip_atomic_store(&a.ctrl[CTRL_ERROR], 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return -1;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Scheduler words in LDS (persistent kernel): the next ticket, whether its
// unit was ready when taken, and the wall-clock time it was taken at.
enum : int { SCH_TICKET = 0, SCH_READY = 1, SCH_TIME = 2, SCH_WORDS = 4 };

// Wave 0 takes the next ticket and checks its unit once.  An update kernel
// does this before its final stores: a wait for the returned values then
// does not also wait for those stores (one in-order counter covers loads and
// stores), and the next unit's loads can be issued while they drain.
__device__ __forceinline__ void take_next(const KArgs& a, int* sch) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const uint64_t tw = wall_clock64();
        const int u = take_ticket(a, lane);
        const bool ready = u >= 0 && unit_ready(a, u, lane);
        if (lane == 0) {
            sch[SCH_TICKET] = u;
            sch[SCH_READY] = ready;
            *(uint64_t*)(sch + SCH_TIME) = tw;
        }
    }
}

__device__ __forceinline__ void retire(const KArgs& a, Prev& p) {
    if (p.task < 0) return;        // uniform
    __builtin_amdgcn_s_waitcnt(0);
    lds_barrier();
    if (threadIdx.x == 0) {
        if (a.trace != nullptr) {
            int64_t* tr = a.trace + 4 * (int64_t)p.ticket;
            tr[0] = (int64_t)p.wait;
            tr[1] = (int64_t)p.run;
            tr[2] = (int64_t)p.end;
            tr[3] = blockIdx.x;
        }
        complete_unit(a, p.task);
    }
    p.task = -1;
}

// ---------------------------------------------------------------------------
// Application of the first NBLK 16-column blocks of a panel record to a
// 16-column slice per wave (the body of UNMQR/TSMQR/TTMQR, Table 1).  Wave
// w's slice c2 (logical columns c0 .. c0 + 15 of C2, all NB rows, in the
// MFMA result layout) is already in registers; block b+1 of the record is
// fetched from memory while block b is applied, then staged in LDS for all
// eight waves:
//   W = C1(block-row b) + V_b^T C2     (UNMQR: no C1)
//   W = T_b^T W
//   C1(block-row b) -= W,   C2 -= V_b W
// which is Q^T [C1; C2] for Q = Q_0 Q_1 ... (Section 3.2).  Zero 16 x 16
// blocks of V are skipped: V is unit lower triangular after GEQRT and upper
// triangular after TTQRT.  HQ applies Q itself (used to form Q C and P C
// from the records): the blocks in reverse order, each with T_b instead of
// T_b^T.  The previous unit of the workgroup is retired once the first
// record block's loads are issued.
// ---------------------------------------------------------------------------
template <int NB, int NBLK, int KIND, bool CO, bool HQ>
__device__ __forceinline__ void apply_blocks(const Rec& rec, const TileView& T1, int c0, bool active,
                                             d4* c2, double* lds, const KArgs& a, Prev& prev) {
    constexpr int MT = NB / 16;
    constexpr int LDV = NB + 1;
    constexpr int BUF = 16 * LDV + 256;       // V_b (NB x 16, stride LDV) then T_b^T (16 x 16)
    constexpr int PRE = 16 * NB / NT + 1;     // staged doubles per thread and block
    constexpr bool HASC1 = KIND != K_UNMQR;
    const int tid = threadIdx.x, lane = tid & 63, j = lane & 15, g = lane >> 4;

    // Block b of the record: V(:, 16b..16b+15) is contiguous (column-major),
    // T_b^T follows the nb x nb matrix.  Thread t stages elements t + NT k of
    // V_b and element t of T_b^T (t < 256).
    auto fetch = [&](int b, double (&pre)[PRE]) {
#pragma unroll
        for (int k = 0; k < PRE - 1; ++k) pre[k] = rec.ld(8 * (tid + NT * k), 8 * (16 * b * NB));
        pre[PRE - 1] = tid < 256 ? rec.ld(8 * tid, 8 * (NB * NB + 256 * b)) : 0.0;
    };
    auto stage = [&](int buffer, const double (&pre)[PRE]) {
        double* buf = lds + buffer * BUF;
#pragma unroll
        for (int k = 0; k < PRE - 1; ++k) {
            const int e = tid + NT * k;
            buf[(e % NB) + (e / NB) * LDV] = pre[k];
        }
        if (tid < 256) buf[16 * LDV + tid] = pre[PRE - 1];
    };
    auto blk = [](int step) { return HQ ? NBLK - 1 - step : step; };

    double pre[PRE];
    fetch(blk(0), pre);
    retire(a, prev);
    stage(0, pre);
    d4 C1n = {0.0, 0.0, 0.0, 0.0};
    if (HASC1 && active) C1n = load16(T1, 16 * blk(0), c0);
    lds_barrier();
#pragma unroll
    for (int st = 0; st < NBLK; ++st) {
        const int b = blk(st);
        const double* Vs = lds + (st & 1) * BUF;
        const double* Ts = Vs + 16 * LDV;
        if (st + 1 < NBLK) fetch(blk(st + 1), pre);
        const d4 C1b = C1n;
        if (HASC1 && active && st + 1 < NBLK) C1n = load16(T1, 16 * blk(st + 1), c0);
        if (active) {
            // Two accumulators halve the dependent-MFMA chain of W.
            d4 Wp[2] = {C1b, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                if (KIND == K_UNMQR && i < b) continue;
                if (KIND == K_TTMQR && i > b) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Wp[r & 1] = mfma(Vs[(16 * i + 4 * r + g) + j * LDV], c2[i][r], Wp[r & 1]);
                // at nb = 256 the slice takes half the registers: keep the
                // operand loads of later row tiles from being hoisted
                if (MT > 8 && (i & 1)) SCHED_FENCE();
            }
            const d4 W = Wp[0] + Wp[1];
            d4 W2 = {0.0, 0.0, 0.0, 0.0};
            // Ts holds T_b^T column-major: T_b(k, i) at i + 16 k.
#pragma unroll
            for (int r = 0; r < 4; ++r)
                W2 = mfma(-(HQ ? Ts[(4 * r + g) + 16 * j] : Ts[j + 16 * (4 * r + g)]), W[r], W2);
            // W2 holds -T_b^T W: negating the 4 T operands spares negating
            // the V operands of the update below.
            if (HASC1) store16<CO>(T1, 16 * b, c0, C1b + W2);
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                if (KIND == K_UNMQR && i < b) continue;
                if (KIND == K_TTMQR && i > b) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) c2[i] = mfma(Vs[(16 * i + j) + (4 * r + g) * LDV], W2[r], c2[i]);
                if (MT > 8 && (i & 1)) SCHED_FENCE();
            }
        }
        if (st + 1 < NBLK) stage((st + 1) & 1, pre);
        lds_barrier();
    }
}

// ---------------------------------------------------------------------------
// Panel kernels: GEQRT, TSQRT, TTQRT (Table 1), blocked by 16 columns.
//
// GEQRT factors the tile X = T1 (R overwrites its upper triangle, zeros below).
// TSQRT / TTQRT factor [R1; X2] with R1 = T1 upper triangular and X2 = T2
// square (TS) or upper triangular (TT): R1 is updated in place and X2 zeroed.
// The reflector of column c is u_c = e_c + (tail below the diagonal) for
// GEQRT and u_c = [e_c ; v2_c] for TS/TT; V stores the tails (with the unit
// diagonal made explicit for GEQRT), which are full for TS and upper
// triangular for TT.
//
// Columns are processed in blocks of 16 (the paper's inner blocking ib):
//  1. leaf: the 16 columns of block b are factored one column at a time by
//     the 256 threads of waves 0-3 (thread (c, q) holds rows q, q+16, ... of
//     leaf column c in registers; one barrier per column).  The dot products of each new
//     reflector with the finished ones give G_b = U_b^T U_b, from which
//     T_b (16 x 16 upper, Q_b = I - U_b T_b U_b^T) follows by the forward
//     recurrence T(c,c) = tau_c, T(0:c-1,c) = -tau_c T(0:c-1,0:c-1) G(0:c-1,c).
//     Waves 4-7, idle in the leaf, form T_b meanwhile, one column behind it.
//  2. trailing: Q_b^T is applied to the column tiles right of the block with
//     three 16-wide MFMA products (W = U_b^T X, W = T_b^T W, X -= U_b W).
// Record (FP64): V (nb x nb, column-major), then the nb/16 blocks T_b^T
// (16 x 16 column-major) -- the same blocked compact-WY form the update
// kernels apply.
// ---------------------------------------------------------------------------

// Step cc of the forward recurrence for T_b on waves 4-7: thread
// (i, l) = (tid/16 - 16, tid%16) holds T(i, l); column cc is formed once
// G(:, cc) is complete.
__device__ __forceinline__ void t_step(double& til, int cc, const double* taus, const double* Gs, int lj, int lq) {
    const int ti = lj - 16;
    const double tcv = taus[cc];
    const double gv = Gs[lq + 16 * cc];
    const double sm = sum16((lq >= ti && lq < cc) ? til * gv : 0.0);
    const double tic = cc < ti ? 0.0 : (cc == ti ? tcv : -tcv * sm);
    if (lq == cc) til = tic;
}

// The 16 columns of leaf block B (one barrier per column).  lw selects the
// role: the leaf waves factor (x: their leaf slots, r1: PAIR's R1 entry),
// the other waves form T_b one column behind (til).  The column loop is
// instantiated per block index B, which fixes at compile time where each
// register slot s (rows lq + 16 s) lies relative to the block's diagonal
// rows 16 B .. 16 B + 15: only slot B straddles the diagonal and needs
// per-lane masks.  Slots that can hold no reflector entry (above the
// diagonal block for GEQRT, below it for the triangle of TTQRT) are left out
// of every step.
template <int NB, int KIND, int B>
__device__ __forceinline__ void leaf_columns(bool lw, double (&x)[NB / 16], double& r1, double& til, double* vbuf,
                                             double* taus, double* Gs, int lj, int lq) {
    constexpr int SR = NB / 16;
    constexpr bool PAIR = KIND != K_GEQRT;
    constexpr bool TT = KIND == K_TTQRT;
    constexpr int S0 = PAIR ? 0 : B;        // live slots [S0, S1)
    constexpr int S1 = TT ? B + 1 : SR;
    constexpr int NL = S1 - S0;
    for (int c = 0; c < 16; ++c) {
        double* vb = vbuf + (c & 1) * NB;
        if (lw && lj == c) {
            // Reflector entry in slot s: rows below the diagonal (GEQRT),
            // the whole tile (TSQRT) or rows up to it (TTQRT).
            auto tail = [&](int s) {
                if (!PAIR) return s > B || lq > c;
                if (TT) return s < B || lq <= c;
                return true;
            };
            // sum of squares in up to four partial sums
            constexpr int NQ = NL < 4 ? NL : 4;
            double q[NQ], al = 0.0;
#pragma unroll
            for (int k = 0; k < NQ; ++k) q[k] = 0.0;
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int s = S0 + k;
                if (tail(s)) q[k % NQ] = fma(x[s], x[s], q[k % NQ]);
            }
            if (!PAIR && lq == c) al = x[B];
#pragma unroll
            for (int h = 1; h < NQ; h *= 2)
#pragma unroll
                for (int k = 0; k + h < NQ; k += 2 * h) q[k] += q[k + h];
            if (PAIR && lq == c) al = r1;
            const double ss = sum16(q[0]);
            // alpha sits in the lane with row phase c of this column's 16
            // lanes (lane 16 (c % 4) + c of the wave): read it there.
            al = readlane64(al, 16 * (c & 3) + c);
            double tau = 0.0, beta = al, scale = 0.0;
            if (ss != 0.0) {
                // tau = (beta - al) / beta and scale = 1 / (al - beta) from
                // one reciprocal: with d = al - beta, 1 / (beta d) gives
                // tau = -d^2 / (beta d) and scale = beta / (beta d).
                const double nrm = refined_sqrt(fma(al, al, ss));
                beta = al >= 0.0 ? -nrm : nrm;
                const double d = al - beta;
                const double inv = refined_rcp(beta * d);
                tau = -(d * d) * inv;
                scale = beta * inv;
            }
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int s = S0 + k;
                double vv;
                if (!PAIR && s == B) {
                    const bool t = lq > c, dg = lq == c;
                    if (t) x[s] *= scale;
                    if (dg) x[s] = beta;
                    vv = t ? x[s] : (dg ? 1.0 : 0.0);
                } else if (TT && s == B) {
                    const bool t = lq <= c;
                    if (t) x[s] *= scale;
                    vv = t ? x[s] : 0.0;
                } else {
                    x[s] *= scale;
                    vv = x[s];
                }
                vb[lq + 16 * s] = vv;
            }
            if (PAIR && lq == c) r1 = beta;
            if (lq == 0) taus[c] = tau;
        }
        lds_barrier();
        if (!lw) {
            // G(:, c-1) was completed before this barrier
            if (c > 0) t_step(til, c - 1, taus, Gs, lj, lq);
        } else {
            // the reflector and tau_c are read together (one LDS latency)
            const double tc = taus[c];
            double vv[SR];
#pragma unroll
            for (int k = 0; k < NL; ++k) vv[S0 + k] = vb[lq + 16 * (S0 + k)];
            // tau_c is needed only after the dot product's reduction; holding
            // it here keeps its read in the same batch as the reflector's
            // instead of after the reduction.
            asm volatile("" ::"v"(tc));
            // tau_c = 0 (H_c = I) needs no branch: it zeroes the update and
            // every T entry that G(:, c) feeds.
            if (lj != c) {
                double dp[2] = {0.0, 0.0};
#pragma unroll
                for (int k = 0; k < NL; ++k) dp[k & 1] = fma(vv[S0 + k], x[S0 + k], dp[k & 1]);
                double d = dp[0] + dp[1];
                if (PAIR && lj > c && lq == c) d += r1;     // e_c meets row c of R1
                d = sum16(d);
                if (lj > c) {
                    const double wv = tc * d;
#pragma unroll
                    for (int k = 0; k < NL; ++k) x[S0 + k] -= wv * vv[S0 + k];
                    if (PAIR && lq == c) r1 -= wv;
                } else if (lq == 0) {
                    Gs[lj + 16 * c] = d;            // u_lj . u_c
                }
            }
        }
    }
}

// Dispatch of leaf block b (runtime) to its instantiation, for the blocks
// BASE .. BASE + COUNT - 1 (COUNT <= 8).
template <int NB, int KIND, int BASE, int COUNT>
__device__ __forceinline__ void leaf_block(int b, bool lw, double (&x)[NB / 16], double& r1, double& til,
                                           double* vbuf, double* taus, double* Gs, int lj, int lq) {
    constexpr int MT = NB / 16;
    auto go = [&](auto bc) {
        constexpr int B = decltype(bc)::value;
        if constexpr (B < MT && B < BASE + COUNT) leaf_columns<NB, KIND, B>(lw, x, r1, til, vbuf, taus, Gs, lj, lq);
    };
    if (b < BASE || b >= BASE + COUNT) return;      // uniform
    switch (b - BASE) {
        case 0: go(std::integral_constant<int, BASE + 0>{}); break;
        case 1: go(std::integral_constant<int, BASE + 1>{}); break;
        case 2: go(std::integral_constant<int, BASE + 2>{}); break;
        case 3: go(std::integral_constant<int, BASE + 3>{}); break;
        case 4: go(std::integral_constant<int, BASE + 4>{}); break;
        case 5: go(std::integral_constant<int, BASE + 5>{}); break;
        case 6: go(std::integral_constant<int, BASE + 6>{}); break;
        default: go(std::integral_constant<int, BASE + 7>{}); break;
    }
}

// Panel for nb <= 128: the whole tile is register-resident, column tile J
// on wave J for the whole kernel; all eight waves apply the trailing
// products.
template <int NB, int KIND, bool CO>
__device__ __forceinline__ void panel_resident(const KArgs& a, const DevTask& tk, double* lds, Prev& prev) {
    using S = Shape<NB>;
    constexpr int MT = S::MT, LDL = S::LDL;
    static_assert(MT <= 8, "one column tile per wave");
    constexpr int SR = NB / 16;             // leaf rows per thread
    constexpr bool PAIR = KIND != K_GEQRT;
    constexpr bool TT = KIND == K_TTQRT;
    double* Lf = lds;                       // leaf: NB x 16, stride LDL
    double* vbuf = Lf + 16 * LDL;           // 2 x NB: broadcast of the current reflector
    double* taus = vbuf + 2 * NB;           // 16
    double* Gs = taus + 16;                 // G(l, c) at l + 16 c
    double* TbT = Gs + 256;                 // T(k, i) at i + 16 k
    double* R1s = TbT + 256;                // PAIR: R1(16b + lq, 16b + lj) of the next block, per leaf thread
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, j = lane & 15, g = lane >> 4;
    const int lj = tid >> 4, lq = tid & 15; // leaf column, row phase
    const bool lw = tid < 256;              // waves 0-3 run the leaf, waves 4-7 form T_b
    const bool own = w < MT;                // the wave holds column tile w

    const MatDesc md = mat_desc(a, tk.mat);
    const TileView T1 = view(md, tk, tk.r1, tk.c1, NB);
    const TileView TX = PAIR ? view(md, tk, tk.r2, tk.c2, NB) : T1;
    double* rec = record<NB>(md, tk);
    double* gV = rec;
    double* gTt = rec + NB * NB;

    d4 xt[MT];
    if (own) load_slice<MT>(TX, 16 * w, xt);
    // R1's row block b is changed by no block before b (the reflectors of
    // block b' touch rows of block b' only), so the diagonal entries the leaf
    // of block b + 1 starts from are read during block b, before that block's
    // stores: with one in-order counter for loads and stores, a load issued
    // after the stores would also wait for them.  Each leaf thread keeps its
    // own entry in LDS until it is needed.
    if (PAIR && lw) R1s[tid] = T1.get(lq, lj);
    retire(a, prev);

    for (int b = 0; b < MT; ++b) {
        // Column tile b goes to the leaf buffer.
        if (w == b) {
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) Lf[(16 * i + 4 * r + g) + j * LDL] = xt[i][r];
        }
        if (lw) Gs[tid] = 0.0;
        lds_barrier();

        // 1. Leaf (waves 0-3), T_b one column behind (waves 4-7).
        double x[SR];
        double r1 = 0.0, til = 0.0;
        if (lw) {
#pragma unroll
            for (int s = 0; s < SR; ++s) x[s] = Lf[(lq + 16 * s) + lj * LDL];
            if (PAIR) r1 = R1s[tid];
        }
        leaf_block<NB, KIND, 0, MT>(b, lw, x, r1, til, vbuf, taus, Gs, lj, lq);
        // Loads ahead of the leaf outputs' stores: the next block's diagonal
        // entry of R1 and this block's rows of R1 in the trailing tiles.
        double r1n = 0.0;
        if (PAIR && lw && b + 1 < MT) r1n = T1.get(16 * (b + 1) + lq, 16 * (b + 1) + lj);
        const bool act = own && w > b;
        d4 R1b = {0.0, 0.0, 0.0, 0.0}, W;
        if (PAIR && act) R1b = load16(T1, 16 * b, 16 * w);
        // Leaf outputs, each thread on the leaf slots it read: explicit U_b
        // into the leaf buffer and the record, R (GEQRT) or zeros (TS/TT)
        // into the matrix.
        if (lw) {
            const int col = 16 * b + lj;
#pragma unroll
            for (int s = 0; s < SR; ++s) {
                const int row = lq + 16 * s;
                double vv;
                if (PAIR) vv = (TT && row > col) ? 0.0 : x[s];
                else vv = row > col ? x[s] : (row == col ? 1.0 : 0.0);
                Lf[row + lj * LDL] = vv;
                gstore<CO>(gV + row + (int64_t)col * NB, vv);
                TX.put<CO>(row, col, PAIR ? 0.0 : (row <= col ? x[s] : 0.0));
            }
            if (PAIR) T1.put<CO>(16 * b + lq, 16 * b + lj, r1);
            if (PAIR && b + 1 < MT) R1s[tid] = r1n;
        }
        lds_barrier();

        // 2. Trailing update of the column tiles right of block b:
        // W = R1 + U_b^T X, then W = T_b^T W, then X -= U_b W.
        W = R1b;
        double la[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) la[r] = Lf[(4 * r + g) + j * LDL];
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            double ln[4];
            if (i + 1 < MT) {
#pragma unroll
                for (int r = 0; r < 4; ++r) ln[r] = Lf[(16 * (i + 1) + 4 * r + g) + j * LDL];
            }
            const bool rows = (PAIR || i >= b) && (!TT || i <= b);
            if (act && rows) {
#pragma unroll
                for (int r = 0; r < 4; ++r) W = mfma(la[r], xt[i][r], W);
            }
            SCHED_FENCE();
            if (i + 1 < MT) {
#pragma unroll
                for (int r = 0; r < 4; ++r) la[r] = ln[r];
            }
        }
        if (!lw) {
            t_step(til, 15, taus, Gs, lj, lq);
            TbT[lq + 16 * (lj - 16)] = til;     // T(i, l)
            gstore<CO>(gTt + 256 * b + (tid - 256), til);
        }
        lds_barrier();
        if (act) {
            d4 W2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 4; ++r) W2 = mfma(TbT[j + 16 * (4 * r + g)], W[r], W2);
            if (PAIR) store16<CO>(T1, 16 * b, 16 * w, R1b - W2);
            W = W2;
        }
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            if (!PAIR && i < b) continue;
            if (TT && i > b) continue;
            double lu[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) lu[r] = -Lf[(16 * i + j) + (4 * r + g) * LDL];
            if (act) {
#pragma unroll
                for (int r = 0; r < 4; ++r) xt[i] = mfma(lu[r], W[r], xt[i]);
            }
            SCHED_FENCE();
        }
        lds_barrier();
    }
}

// Synchronization inside one workgroup through LDS words, for code where the
// waves of the workgroup follow different paths (no workgroup barrier).
// wait_geq: wait until *f >= target; false once the watchdog has expired
// (the error word is then set and the caller gives up).  post: make this
// wave's earlier LDS writes visible, then add 1 to *f.
__device__ __forceinline__ bool wait_geq(const int* f, int target, const KArgs& a) {
    uint64_t t0 = 0;
    for (int spin = 0;; ++spin) {
        const int v = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (v >= target) break;
        __builtin_amdgcn_s_sleep(1);        // leave issue slots to the working waves
        // the clock (a scalar memory read) only every 128 polls
        if ((spin & 127) == 0) {
            const uint64_t t = wall_clock64();
            if (spin == 0) {
                t0 = t;
            } else if ((int64_t)(t - t0) > a.watchdog_ticks) {
                if ((threadIdx.x & 63) == 0)
                    __hip_atomic_store(&a.ctrl[CTRL_ERROR], 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    return true;
}

__device__ __forceinline__ void post(int* f) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_add(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Panel for nb = 256 (16 column tiles of 256 x 16, each taking half of a
// wave's registers, so no tile can stay resident next to the leaf).  The
// waves split into two roles that run side by side and meet only through
// LDS counters:
//  - leaf role (waves 0-3): factors block b from the LDS copy of column
//    tile b.  Columns are handed on through a per-column counter instead of
//    a workgroup barrier; the 16 reflectors of the block stay in an LDS ring.
//    Then it writes U_b (explicit), the record's V, and R or zeros.
//  - tile role (waves 4-7): forms T_b from the dot products (each 16-lane row
//    of T on its own), then applies Q_b^T first to tile b + 1, which it hands
//    to the next leaf through LDS (look-ahead), and then to the other tiles
//    right of b, which it streams from and back to memory.  Tile J always
//    goes to wave 4 + J % 4, so every lane reads back only what it stored.
// The leaf of block b + 1 therefore runs while the tile role is still
// applying block b to tiles b + 2 ... 15.
template <int NB, int KIND, bool CO>
__device__ __forceinline__ void panel_split(const KArgs& a, const DevTask& tk, double* lds, Prev& prev) {
    using S = Shape<NB>;
    constexpr int MT = S::MT, LDL = S::LDL;
    constexpr int SR = NB / 16;
    constexpr bool PAIR = KIND != K_GEQRT;
    constexpr bool TT = KIND == K_TTQRT;
    double* buf0 = lds;                     // column tile of the leaf, by block parity: NB x 16, stride LDL
    double* vring = lds + 32 * LDL;         // the 16 reflectors of the current block, NB each
    double* taus = vring + 16 * NB;
    double* Gs = taus + 16;                 // G(l, c) at l + 16 c
    double* TbT0 = Gs + 256;                // T_b (T(k, i) at i + 16 k), by block parity
    double* Wpart = TbT0 + 512;             // the four tile waves' partial W, by tile parity
    int* flags = (int*)(Wpart + 2 * 1024);  // counters
    static_assert(32 * LDL + 16 * NB + 16 + 256 + 512 + 2048 + 4 <= S::LDS, "LDS layout");
    enum { F_COL = 0, F_LEAF = 1, F_TB = 2, F_TILE = 3, F_WA = 4, F_WORDS = 8 };
    const int tid = threadIdx.x, lane = tid & 63, j = lane & 15, g = lane >> 4;
    const int lj = tid >> 4, lq = tid & 15;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);

    const MatDesc md = mat_desc(a, tk.mat);
    const TileView T1 = view(md, tk, tk.r1, tk.c1, NB);
    const TileView TX = PAIR ? view(md, tk, tk.r2, tk.c2, NB) : T1;
    double* rec = record<NB>(md, tk);
    double* gV = rec;
    double* gTt = rec + NB * NB;

    // column tile 0 into the first leaf buffer; counters to zero
#pragma unroll
    for (int k = 0; k < NB * 16 / NT; ++k) {
        const int e = tid + NT * k, r = e % NB, c = e / NB;
        buf0[r + c * LDL] = TX.get(r, c);
    }
    if (tid < F_WORDS) flags[tid] = 0;
    retire(a, prev);                        // (a workgroup barrier)
    lds_barrier();

    if (w < 4) {
        // ---- leaf role -------------------------------------------------
        double r1 = PAIR ? T1.get(lq, lj) : 0.0;
        for (int b = 0; b < MT; ++b) {
            if (!wait_geq(&flags[F_TILE], b, a)) break;         // column tile b is in its buffer
            double* Lf = buf0 + (b & 1) * 16 * LDL;
            double x[SR];
#pragma unroll
            for (int s = 0; s < SR; ++s) x[s] = Lf[(lq + 16 * s) + lj * LDL];
            bool ok = true;
            auto leaf = [&](auto bc) {
                constexpr int B = decltype(bc)::value;
                constexpr int S0 = PAIR ? 0 : B;        // live slots [S0, S1)
                constexpr int S1 = TT ? B + 1 : SR;
                constexpr int NL = S1 - S0;
                for (int c = 0; c < 16 && ok; ++c) {
                    double* vb = vring + c * NB;
                    if (lj == c) {
                        auto tail = [&](int s) {
                            if (!PAIR) return s > B || lq > c;
                            if (TT) return s < B || lq <= c;
                            return true;
                        };
                        constexpr int NQ = NL < 4 ? NL : 4;
                        double q[NQ], al = 0.0;
#pragma unroll
                        for (int k = 0; k < NQ; ++k) q[k] = 0.0;
#pragma unroll
                        for (int k = 0; k < NL; ++k) {
                            const int s = S0 + k;
                            if (tail(s)) q[k % NQ] = fma(x[s], x[s], q[k % NQ]);
                        }
                        if (!PAIR && lq == c) al = x[B];
#pragma unroll
                        for (int h = 1; h < NQ; h *= 2)
#pragma unroll
                            for (int k = 0; k + h < NQ; k += 2 * h) q[k] += q[k + h];
                        if (PAIR && lq == c) al = r1;
                        const double ss = sum16(q[0]);
                        al = readlane64(al, 16 * (c & 3) + c);
                        double tau = 0.0, beta = al, scale = 0.0;
                        if (ss != 0.0) {
                            const double nrm = refined_sqrt(fma(al, al, ss));
                            beta = al >= 0.0 ? -nrm : nrm;
                            const double d = al - beta;
                            const double inv = refined_rcp(beta * d);
                            tau = -(d * d) * inv;
                            scale = beta * inv;
                        }
#pragma unroll
                        for (int k = 0; k < NL; ++k) {
                            const int s = S0 + k;
                            double vv;
                            if (!PAIR && s == B) {
                                const bool t = lq > c, dg = lq == c;
                                if (t) x[s] *= scale;
                                if (dg) x[s] = beta;
                                vv = t ? x[s] : (dg ? 1.0 : 0.0);
                            } else if (TT && s == B) {
                                const bool t = lq <= c;
                                if (t) x[s] *= scale;
                                vv = t ? x[s] : 0.0;
                            } else {
                                x[s] *= scale;
                                vv = x[s];
                            }
                            vb[lq + 16 * s] = vv;
                        }
                        if (PAIR && lq == c) r1 = beta;
                        if (lq == 0) taus[c] = tau;
                    }
                    if (w == (c >> 2)) post(&flags[F_COL]);            // the owner wave
                    if (!wait_geq(&flags[F_COL], 16 * b + c + 1, a)) { ok = false; break; }
                    if (lj != c) {
                        const double tc = taus[c];
                        double vv[SR];
#pragma unroll
                        for (int k = 0; k < NL; ++k) vv[S0 + k] = vb[lq + 16 * (S0 + k)];
                        double dp[2] = {0.0, 0.0};
#pragma unroll
                        for (int k = 0; k < NL; ++k) dp[k & 1] = fma(vv[S0 + k], x[S0 + k], dp[k & 1]);
                        double d = dp[0] + dp[1];
                        if (PAIR && lj > c && lq == c) d += r1;     // e_c meets row c of R1
                        d = sum16(d);
                        if (lj > c) {
                            const double wv = tc * d;
#pragma unroll
                            for (int k = 0; k < NL; ++k) x[S0 + k] -= wv * vv[S0 + k];
                            if (PAIR && lq == c) r1 -= wv;
                        } else if (lq == 0) {
                            Gs[lj + 16 * c] = d;            // u_lj . u_c
                        }
                    }
                }
            };
            switch (b) {
#define BB_LEAF_CASE(K) case K: leaf(std::integral_constant<int, K>{}); break;
                BB_LEAF_CASE(0) BB_LEAF_CASE(1) BB_LEAF_CASE(2) BB_LEAF_CASE(3)
                BB_LEAF_CASE(4) BB_LEAF_CASE(5) BB_LEAF_CASE(6) BB_LEAF_CASE(7)
                BB_LEAF_CASE(8) BB_LEAF_CASE(9) BB_LEAF_CASE(10) BB_LEAF_CASE(11)
                BB_LEAF_CASE(12) BB_LEAF_CASE(13) BB_LEAF_CASE(14)
                default: leaf(std::integral_constant<int, 15>{}); break;
#undef BB_LEAF_CASE
            }
            if (!ok) break;
            // R1's next diagonal entry: no block before b + 1 changes it
            double r1n = 0.0;
            if (PAIR && b + 1 < MT) r1n = T1.get(16 * (b + 1) + lq, 16 * (b + 1) + lj);
            const int col = 16 * b + lj;
#pragma unroll
            for (int s = 0; s < SR; ++s) {
                const int row = lq + 16 * s;
                double vv;
                if (PAIR) vv = (TT && row > col) ? 0.0 : x[s];
                else vv = row > col ? x[s] : (row == col ? 1.0 : 0.0);
                Lf[row + lj * LDL] = vv;
                gstore<CO>(gV + row + (int64_t)col * NB, vv);
                TX.put<CO>(row, col, PAIR ? 0.0 : (row <= col ? x[s] : 0.0));
            }
            if (PAIR) T1.put<CO>(16 * b + lq, 16 * b + lj, r1);
            r1 = r1n;
            post(&flags[F_LEAF]);                                   // U_b, taus, G complete
        }
    } else {
        // ---- tile role -------------------------------------------------
        // Tile J belongs to wave 4 + J % 4 for the whole panel, which applies
        // Q_b^T to it alone (W = R1 + U_b^T X over all rows, W = T_b^T W,
        // X -= U_b W): no partial sums between waves.  Only the row tiles a
        // block changes are loaded, updated and stored (all of them for TS;
        // those at or below block b for GEQRT, at or above it in TTQRT's
        // triangle), except for tile b + 1, which its owner hands to the next
        // leaf whole, through LDS.  Between blocks the tiles wait in the
        // panel's scratch (this workgroup's alone, each lane's values side by
        // side, whole-line stores); a row tile comes from the matrix the first
        // time a block changes it or the leaf needs it.  The next tile is
        // loaded as soon as the current one is stored.
        const int u = w - 4;
        const int ti = lj - 16;             // this thread's row of T_b (and l = lq)
        bool ok = true;
        double* scr = a.pscratch + (int64_t)blockIdx.x * panel_scratch_doubles(NB) + 4 * lane;
        auto scr_at = [&](int J, int i) { return scr + (J * MT + i) * 256; };
        auto active = [&](int i, int bb) { return PAIR ? (!TT || i <= bb) : i >= bb; };
        // block in which row tile i is first changed
        auto first = [&](int i) { return TT ? i : 0; };
        d4 x[MT], R1b = {0.0, 0.0, 0.0, 0.0};
        // tile J as block bb needs it
        auto fetch = [&](int J, int bb) {
            const bool whole = J == bb + 1;
            if (PAIR) R1b = load16(T1, 16 * bb, 16 * J);
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                if (!whole && !active(i, bb)) continue;
                if (bb > first(i)) x[i] = load_d4(scr_at(J, i));
                else x[i] = load16(TX, 16 * i, 16 * J);
            }
        };
        // this wave's first tile after block bb (MT if none)
        auto next_tile = [&](int bb) { return bb + 1 + ((u - (bb + 1)) % 4 + 4) % 4; };
        int Jn = next_tile(0);
        if (Jn < MT) fetch(Jn, 0);
        for (int b = 0; b < MT && ok; ++b) {
            if (!wait_geq(&flags[F_LEAF], 4 * (b + 1), a)) break;
            const double* U = buf0 + (b & 1) * 16 * LDL;
            double* TbT = TbT0 + (b & 1) * 256;
            // T_b by the forward recurrence (each 16-lane row of T on its
            // own), from G and tau read once
            double gcol[16], tcol[16];
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) {
                gcol[cc] = Gs[lq + 16 * cc];
                tcol[cc] = taus[cc];
            }
            double til = 0.0;
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) {
                const double sm = sum16((lq >= ti && lq < cc) ? til * gcol[cc] : 0.0);
                const double tic = cc < ti ? 0.0 : (cc == ti ? tcol[cc] : -tcol[cc] * sm);
                if (lq == cc) til = tic;
            }
            TbT[lq + 16 * ti] = til;
            gstore<CO>(gTt + 256 * b + (tid - 256), til);
            post(&flags[F_TB]);
            if (!wait_geq(&flags[F_TB], 4 * (b + 1), a)) break;

#pragma unroll 1
            for (int J = Jn; J < MT; J += 4) {
                asm volatile("" ::: "memory");
                const bool whole = J == b + 1;
                d4 Wk[2] = {R1b, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    if (!active(i, b)) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        Wk[i & 1] = mfma(U[(16 * i + 4 * r + g) + j * LDL], x[i][r], Wk[i & 1]);
                }
                const d4 W = Wk[0] + Wk[1];
                d4 W2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int r = 0; r < 4; ++r) W2 = mfma(TbT[j + 16 * (4 * r + g)], W[r], W2);
                if (PAIR) store16<CO>(T1, 16 * b, 16 * J, R1b - W2);
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    if (!active(i, b)) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        x[i] = mfma(-U[(16 * i + j) + (4 * r + g) * LDL], W2[r], x[i]);
                }
                if (whole) {
                    double* Ln = buf0 + ((b + 1) & 1) * 16 * LDL;
#pragma unroll
                    for (int i = 0; i < MT; ++i)
#pragma unroll
                        for (int r = 0; r < 4; ++r) Ln[(16 * i + 4 * r + g) + j * LDL] = x[i][r];
                    post(&flags[F_TILE]);                           // the next leaf may start
                } else {
#pragma unroll
                    for (int i = 0; i < MT; ++i)
                        if (active(i, b)) store_d4(scr_at(J, i), x[i]);
                }
                // the next tile: this block's, else the next block's first
                const int Jnext = J + 4 < MT ? J + 4 : next_tile(b + 1);
                if (Jnext < MT) fetch(Jnext, J + 4 < MT ? b : b + 1);
            }
            Jn = next_tile(b + 1);      // fetched above, after the block's last tile
        }
    }
    lds_barrier();
}

template <int NB, int KIND, bool CO>
__device__ __forceinline__ void panel(const KArgs& a, const DevTask& tk, double* lds, Prev& prev) {
    if constexpr (NB <= 128) panel_resident<NB, KIND, CO>(a, tk, lds, prev);
    else panel_split<NB, KIND, CO>(a, tk, lds, prev);
}

// ---------------------------------------------------------------------------
// Update kernels: UNMQR, TSMQR, TTMQR (Table 1) on a strip of the trailing
// tile (or tile pair): the whole tile for nb <= 128, a 128-column half for
// nb = 256.  Wave w owns the 16 logical columns c0 = part * NS + 16 w ..
// c0 + 15 of C2 (and C1); waves past the tile's width only stage and
// synchronize.  All nb/16 blocks of the record are applied (apply_blocks).
// ---------------------------------------------------------------------------
template <int NB, int KIND, bool CO, bool HQ>
__device__ __forceinline__ void update(const KArgs& a, const DevTask& tk, int part, double* lds, Prev& prev,
                                       int* sch) {
    constexpr int MT = NB / 16;
    constexpr int NS = NB < 128 ? NB : 128;  // strip width: one 16-column slice per wave
    constexpr bool HASC1 = KIND != K_UNMQR;
    const int tid = threadIdx.x, w = tid >> 6;
    const int c0 = part * NS + 16 * w;
    const MatDesc md = mat_desc(a, tk.mat);
    const TileView T2 = view(md, tk, tk.r2, tk.c2, NB);
    const TileView T1 = HASC1 ? view(md, tk, tk.r1, tk.c1, NB) : T2;
    // Waves without columns still take part in staging and barriers.
    const bool active = 16 * w < NS && c0 < T2.vc;
    const Rec rec(record<NB>(md, tk), NB);

    d4 c2[MT];
    if (active) load_slice<MT>(T2, c0, c2);
    apply_blocks<NB, MT, KIND, CO, HQ>(rec, T1, c0, active, &c2[0], lds, a, prev);
    if (sch != nullptr) take_next(a, sch);
    if (active) store_slice<CO, MT>(T2, c0, c2);
}

// ---------------------------------------------------------------------------
// Updates on FP32 MFMA (v_mfma_f32_16x16x4f32), for the precision variants:
// the V/T block operands and the C operands are rounded to FP32 (RNE), each
// product accumulates in FP32, and its result is added into the FP64 tiles.
// SPLIT: every operand x is also carried as x_lo = fp32(x - x_hi) and a
// product A B is taken as A_hi B_hi + A_hi B_lo + A_lo B_hi, accumulated in
// FP32 over 16-row chunks and in FP64 across chunks.  Panels, V and T stay
// FP64 in either case.
//
// The FP32 instruction returns element r of lane l at row 4(l/16) + r (the
// FP64 one at row 4r + l/16).  Slices are therefore held in that layout, and
// the k-step r of a 16-row block takes the rows {4g + r : g = 0..3}: lane l
// supplies row 4(l/16) + r of its column, which is its own element r.
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int MT>
__device__ __forceinline__ void load_slice_r4(const TileView& t, int c0, d4 (&x)[MT]) {
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[i][r] = t.get(16 * i + 4 * g + r, c0 + j);
}

template <bool CO, int MT>
__device__ __forceinline__ void store_slice_r4(const TileView& t, int c0, const d4 (&x)[MT]) {
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) t.put<CO>(16 * i + 4 * g + r, c0 + j, x[i][r]);
}

__device__ __forceinline__ d4 load16_r4(const TileView& t, int r0, int c0) {
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    d4 x;
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = t.get(r0 + 4 * g + r, c0 + j);
    return x;
}

template <bool CO>
__device__ __forceinline__ void store16_r4(const TileView& t, int r0, int c0, d4 x) {
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) t.put<CO>(r0 + 4 * g + r, c0 + j, x[r]);
}

__device__ __forceinline__ float lo32(double x, float hi) { return (float)(x - (double)hi); }

template <int NB, int KIND, bool CO, bool SPLIT>
__device__ __forceinline__ void update32(const KArgs& a, const DevTask& tk, int part, double* lds, Prev& prev,
                                         int* sch) {
    constexpr int MT = NB / 16;
    constexpr int NS = NB < 128 ? NB : 128;  // strip width: one 16-column slice per wave
    constexpr int LDV = NB + 1;
    constexpr int PL = 16 * LDV + 256;        // floats per plane: V_b (NB x 16) then T_b^T
    constexpr int BUF = (SPLIT ? 2 : 1) * PL; // hi plane [, lo plane]
    constexpr int PRE = 16 * NB / NT + 1;
    constexpr bool HASC1 = KIND != K_UNMQR;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, j = lane & 15, g = lane >> 4;
    const int c0 = part * NS + 16 * w;
    const MatDesc md = mat_desc(a, tk.mat);
    const TileView T2 = view(md, tk, tk.r2, tk.c2, NB);
    const TileView T1 = HASC1 ? view(md, tk, tk.r1, tk.c1, NB) : T2;
    const bool active = 16 * w < NS && c0 < T2.vc;
    const Rec rec(record<NB>(md, tk), NB);
    float* fl = reinterpret_cast<float*>(lds);

    auto fetch = [&](int b, double (&pre)[PRE]) {
#pragma unroll
        for (int k = 0; k < PRE - 1; ++k) pre[k] = rec.ld(8 * (tid + NT * k), 8 * (16 * b * NB));
        pre[PRE - 1] = tid < 256 ? rec.ld(8 * tid, 8 * (NB * NB + 256 * b)) : 0.0;
    };
    auto stage = [&](int b, const double (&pre)[PRE]) {
        float* hi = fl + (b & 1) * BUF;
        float* lo = hi + PL;
#pragma unroll
        for (int k = 0; k < PRE - 1; ++k) {
            const int e = tid + NT * k;
            const int at = (e % NB) + (e / NB) * LDV;
            const float h = (float)pre[k];
            hi[at] = h;
            if (SPLIT) lo[at] = lo32(pre[k], h);
        }
        if (tid < 256) {
            const float h = (float)pre[PRE - 1];
            hi[16 * LDV + tid] = h;
            if (SPLIT) lo[16 * LDV + tid] = lo32(pre[PRE - 1], h);
        }
    };
    // Product of a (16 x 4) A-fragment pair with a B-fragment given in FP64.
    auto prod = [&](float ah, float al, double bv, f4 acc) {
        const float bh = (float)bv;
        acc = mfma32(ah, bh, acc);
        if (SPLIT) {
            acc = mfma32(ah, lo32(bv, bh), acc);
            acc = mfma32(al, bh, acc);
        }
        return acc;
    };

    d4 c2[MT];
    if (active) load_slice_r4<MT>(T2, c0, c2);
    double pre[PRE];
    fetch(0, pre);
    retire(a, prev);
    stage(0, pre);
    d4 C1n = {0.0, 0.0, 0.0, 0.0};
    if (HASC1 && active) C1n = load16_r4(T1, 0, c0);
    lds_barrier();
#pragma unroll
    for (int b = 0; b < MT; ++b) {
        const float* Vh = fl + (b & 1) * BUF;
        const float* Vl = Vh + PL;
        const float* Th = Vh + 16 * LDV;
        const float* Tl = Vl + 16 * LDV;
        if (b + 1 < MT) fetch(b + 1, pre);
        const d4 C1b = C1n;
        if (HASC1 && active && b + 1 < MT) C1n = load16_r4(T1, 16 * (b + 1), c0);
        if (active) {
            // W = C1_b + V_b^T C2, FP64 across 16-row chunks.
            d4 W = C1b;
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                if (KIND == K_UNMQR && i < b) continue;
                if (KIND == K_TTMQR && i > b) continue;
                f4 ch = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int at = (16 * i + 4 * g + r) + j * LDV;
                    ch = prod(Vh[at], SPLIT ? Vl[at] : 0.f, c2[i][r], ch);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) W[r] += (double)ch[r];
            }
            // W2 = T_b^T W
            f4 w2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int at = j + 16 * (4 * g + r);
                w2 = prod(Th[at], SPLIT ? Tl[at] : 0.f, W[r], w2);
            }
            d4 W2;
#pragma unroll
            for (int r = 0; r < 4; ++r) W2[r] = (double)w2[r];
            if (HASC1) store16_r4<CO>(T1, 16 * b, c0, C1b - W2);
            // C2 -= V_b W2
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                if (KIND == K_UNMQR && i < b) continue;
                if (KIND == K_TTMQR && i > b) continue;
                f4 ch = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int at = (16 * i + j) + (4 * g + r) * LDV;
                    ch = prod(-Vh[at], SPLIT ? -Vl[at] : 0.f, W2[r], ch);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) c2[i][r] += (double)ch[r];
            }
        }
        if (b + 1 < MT) stage(b + 1, pre);
        lds_barrier();
    }
    if (sch != nullptr) take_next(a, sch);
    if (active) store_slice_r4<CO, MT>(T2, c0, c2);
}

// PREC: 0 = FP64 updates, 2 = FP32-MFMA updates, 3 = split-FP32 updates
// (reductions: panels and updates); PREC_APPLY = the applications of Q and
// P from finished records (FP64 updates of both directions, no panels).
// Reductions and applications are separate kernels, so that neither carries
// the register demand of the other's code.
template <int NB, bool CO, int PREC>
__device__ __forceinline__ void run_unit(const KArgs& a, int task, int part, double* lds, Prev& prev, int* sch) {
    const DevTask tk = a.tasks[task];      // task is wave-uniform: scalar loads
    if constexpr (PREC == PREC_APPLY) {
        switch (tk.kind) {
        case K_UNMQR: update<NB, K_UNMQR, CO, false>(a, tk, part, lds, prev, sch); break;
        case K_TSMQR: update<NB, K_TSMQR, CO, false>(a, tk, part, lds, prev, sch); break;
        case K_TTMQR: update<NB, K_TTMQR, CO, false>(a, tk, part, lds, prev, sch); break;
        case K_UNMQR + K_HQ: update<NB, K_UNMQR, CO, true>(a, tk, part, lds, prev, sch); break;
        case K_TSMQR + K_HQ: update<NB, K_TSMQR, CO, true>(a, tk, part, lds, prev, sch); break;
        default: update<NB, K_TTMQR, CO, true>(a, tk, part, lds, prev, sch); break;
        }
    } else {
        switch (tk.kind) {
        case K_GEQRT: panel<NB, K_GEQRT, CO>(a, tk, lds, prev); break;
        case K_TSQRT: panel<NB, K_TSQRT, CO>(a, tk, lds, prev); break;
        case K_TTQRT: panel<NB, K_TTQRT, CO>(a, tk, lds, prev); break;
        case K_UNMQR:
            if (PREC == 0) update<NB, K_UNMQR, CO, false>(a, tk, part, lds, prev, sch);
            else update32<NB, K_UNMQR, CO, PREC == 3>(a, tk, part, lds, prev, sch);
            break;
        case K_TSMQR:
            if (PREC == 0) update<NB, K_TSMQR, CO, false>(a, tk, part, lds, prev, sch);
            else update32<NB, K_TSMQR, CO, PREC == 3>(a, tk, part, lds, prev, sch);
            break;
        default:
            if (PREC == 0) update<NB, K_TTMQR, CO, false>(a, tk, part, lds, prev, sch);
            else update32<NB, K_TTMQR, CO, PREC == 3>(a, tk, part, lds, prev, sch);
            break;
        }
    }
    retire(a, prev);               // a kind that ran nothing
}

// A unit of a launch that mixes tile sizes: the task's own size, from its
// descriptor.
template <bool CO, int PREC>
__device__ __forceinline__ void run_unit_mixed(const KArgs& a, int task, int part, double* lds, Prev& prev,
                                               int* sch) {
    const int code = __builtin_amdgcn_readfirstlane(a.tasks[task].trans) >> 1;
    switch (code) {
    case 0: run_unit<32, CO, PREC>(a, task, part, lds, prev, sch); break;
    case 1: run_unit<64, CO, PREC>(a, task, part, lds, prev, sch); break;
    default: run_unit<128, CO, PREC>(a, task, part, lds, prev, sch); break;
    }
}

template <int NB, bool CO, int PREC>
__device__ __forceinline__ void run_any(const KArgs& a, int task, int part, double* lds, Prev& prev, int* sch) {
    if constexpr (NB == NB_MIXED) run_unit_mixed<CO, PREC>(a, task, part, lds, prev, sch);
    else run_unit<NB, CO, PREC>(a, task, part, lds, prev, sch);
}

// LDS of a kernel (doubles): the mixed kernels hold the largest size they run.
template <int NB>
constexpr int kernel_lds() { return NB == NB_MIXED ? Shape<128>::LDS : Shape<NB>::LDS; }

}  // namespace

// One launch per topological level: block b runs unit unit_base + b.
template <int NB, int PREC>
__global__ __launch_bounds__(NT) void level_kernel(KArgs a, int32_t unit_base) {
    __shared__ double lds[kernel_lds<NB>()];
    const int2 u = a.units[unit_base + blockIdx.x];
    Prev none{-1, 0, 0, 0, 0};
    run_any<NB, false, PREC>(a, u.x, u.y, lds, none, nullptr);
}

// Persistent scheduler.  The work units are listed in one priority order:
// the start order of a list-scheduling simulation of the task graph on the
// GPU's workgroups (most urgent ready unit first), which is topological (a
// unit's predecessors all come earlier).  Each workgroup takes the next
// position of that order (one atomic add on the ticket counter) and waits
// until the unit's task has no unfinished predecessor unit.  Tickets go only
// to running workgroups and every predecessor holds an earlier ticket, so the
// earliest unfinished ticket can always proceed: no deadlock for any grid
// size.  A finished unit is counted done only after the workgroup's next unit
// has issued its first loads (its output stores drain meanwhile), and never
// later than the workgroup's next wait on a dependency, so that argument still
// holds.  A wall-clock watchdog bounds every wait (error 3 after
// watchdog_ticks), and an error reported by any workgroup stops all of them.

template <int NB, int PREC>
__global__ __launch_bounds__(NT) void persistent_kernel(KArgs a) {
    __shared__ double lds[kernel_lds<NB>() + SCH_WORDS / 2];
    int* sch = (int*)(lds + kernel_lds<NB>());
    const int tid = threadIdx.x;
    Prev prev{-1, 0, 0, 0, 0};
    if (tid == 0) sch[SCH_TICKET] = -2;     // -2: no ticket taken yet
    for (;;) {
        lds_barrier();
        if (__builtin_amdgcn_readfirstlane(sch[SCH_TICKET]) == -2) take_next(a, sch);
        lds_barrier();
        // Uniform in the workgroup; readfirstlane lets the compiler see that,
        // which keeps the loop's exits uniform.
        int u = __builtin_amdgcn_readfirstlane(sch[SCH_TICKET]);
        const bool ready = __builtin_amdgcn_readfirstlane(sch[SCH_READY]) != 0;
        const uint64_t t_wait = *(const uint64_t*)(sch + SCH_TIME);
        lds_barrier();
        if (tid == 0) sch[SCH_TICKET] = -2;
        // Never wait while holding an unfinished unit: its successors may be
        // the units waited for.
        if (!ready) retire(a, prev);
        if (u < 0) break;
        if (!ready) {
            if (tid < 64) {
                const int r = wait_unit(a, u, tid);
                if (tid == 0) sch[SCH_READY] = r;
            }
            lds_barrier();
            u = __builtin_amdgcn_readfirstlane(sch[SCH_READY]);
            if (u < 0) break;
        }
        const int2 un0 = a.units[u];
        const int2 un = make_int2(__builtin_amdgcn_readfirstlane(un0.x),
                                  __builtin_amdgcn_readfirstlane(un0.y));
        // Acquire: drop stale lines of the inputs from this CU's caches and
        // this XCD's L2 (the predecessors' completion was observed above).
        // Release: a unit writes its outputs with agent-scope stores, and
        // waiting for them to complete publishes them to every XCD.  The
        // invalidation is issued without the full memory wait a fence would
        // add, which would also wait for the previous unit's stores.
        asm volatile("buffer_inv sc1" ::: "memory");
        const uint64_t t_run = a.trace != nullptr && tid == 0 ? wall_clock64() : 0;
        run_any<NB, true, PREC>(a, un.x, un.y, lds, prev, sch);
        prev.task = un.x;
        prev.ticket = u;
        prev.wait = t_wait;
        prev.run = t_run;
        prev.end = a.trace != nullptr && tid == 0 ? wall_clock64() : 0;
    }
}

#ifdef BB_KERNELS_COMMON
__global__ void init_kernel(int32_t* deps, const int32_t* ndeps, int32_t ntasks, int32_t* ctrl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < CTRL_WORDS) ctrl[i] = 0;
    for (int t = i; t < ntasks; t += gridDim.x * blockDim.x) deps[t] = ndeps[t];
}

hipError_t launch_init(const KArgs& a, const int32_t* ndeps_init, int32_t ntasks, hipStream_t s) {
    int blocks = (ntasks + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(256), 0, s, a.deps, ndeps_init, ntasks, a.ctrl);
    return hipGetLastError();
}

__global__ void batch_desc_kernel(MatDesc* mats, int32_t nmats, const int64_t* gidx, const int64_t* dims,
                                  const int64_t* recoff, double* const* A, const int64_t* lda, double* vt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nmats; i += gridDim.x * blockDim.x) {
        const int64_t g = gidx[i];
        mats[i] = MatDesc{A[g], lda[g], dims[2 * i], dims[2 * i + 1], vt + recoff[i]};
    }
}

hipError_t launch_batch_desc(MatDesc* mats, int32_t nmats, const int64_t* gidx, const int64_t* dims,
                             const int64_t* recoff, double* const* A, const int64_t* lda, double* vt,
                             hipStream_t s) {
    if (nmats <= 0) return hipSuccess;
    int blocks = (nmats + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(batch_desc_kernel, dim3(blocks), dim3(256), 0, s, mats, nmats, gidx, dims, recoff, A,
                       lda, vt);
    return hipGetLastError();
}

bool nb_supported(int nb) { return nb == 32 || nb == 64 || nb == 128 || nb == 256; }

// Workspace of bb_execute_noalloc: a file-scope device array, one copy per
// device for the life of the process.  Host code never passes the array's
// name to a kernel or a copy (on the host it is only a stand-in for the
// symbol): the device address of each device's copy is looked up once, with
// that device current, and used everywhere instead.
static __device__ __align__(256) unsigned char scratch[BB_NOALLOC_WS_MAX];

hipError_t noalloc_scratch(void** ptr, size_t* bytes) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = BB_NOALLOC_WS_MAX;
    return hipSuccess;
}

#endif  // BB_KERNELS_COMMON

template <int NB, int PREC>
hipError_t launch_level_np(const KArgs& a, int32_t unit_base, int32_t count, hipStream_t s) {
    hipLaunchKernelGGL((level_kernel<NB, PREC>), dim3(count), dim3(NT), 0, s, a, unit_base);
    return hipGetLastError();
}

template <int NB, int PREC>
hipError_t launch_persistent_np(const KArgs& a, int32_t workgroups, hipStream_t s) {
    hipLaunchKernelGGL((persistent_kernel<NB, PREC>), dim3(workgroups), dim3(NT), 0, s, a);
    return hipGetLastError();
}

// This file is compiled once per (tile size, arithmetic) pair (BB_KERNELS_NB,
// BB_KERNELS_PREC: that pair's kernels, the translation units built in
// parallel) and once for the size-independent part (BB_KERNELS_COMMON).
#if defined(BB_KERNELS_NB) && defined(BB_KERNELS_PREC)
template hipError_t launch_level_np<BB_KERNELS_NB, BB_KERNELS_PREC>(const KArgs&, int32_t, int32_t, hipStream_t);
template hipError_t launch_persistent_np<BB_KERNELS_NB, BB_KERNELS_PREC>(const KArgs&, int32_t, hipStream_t);
#endif

#ifdef BB_KERNELS_COMMON
#define BB_NP_CASES(F, ...)                                                        \
    switch (nb * 4 + prec) {                                                       \
    case NB_MIXED * 4 + 0: return F<NB_MIXED, 0>(__VA_ARGS__);                     \
    case NB_MIXED * 4 + 2: return F<NB_MIXED, 2>(__VA_ARGS__);                     \
    case NB_MIXED * 4 + 3: return F<NB_MIXED, 3>(__VA_ARGS__);                     \
    case 32 * 4 + 0: return F<32, 0>(__VA_ARGS__);                                 \
    case 32 * 4 + 2: return F<32, 2>(__VA_ARGS__);                                 \
    case 32 * 4 + 3: return F<32, 3>(__VA_ARGS__);                                 \
    case 64 * 4 + 0: return F<64, 0>(__VA_ARGS__);                                 \
    case 64 * 4 + 2: return F<64, 2>(__VA_ARGS__);                                 \
    case 64 * 4 + 3: return F<64, 3>(__VA_ARGS__);                                 \
    case 128 * 4 + 0: return F<128, 0>(__VA_ARGS__);                               \
    case 128 * 4 + 2: return F<128, 2>(__VA_ARGS__);                               \
    case 128 * 4 + 3: return F<128, 3>(__VA_ARGS__);                               \
    case 256 * 4 + 0: return F<256, 0>(__VA_ARGS__);                               \
    case 256 * 4 + 2: return F<256, 2>(__VA_ARGS__);                               \
    case 256 * 4 + 3: return F<256, 3>(__VA_ARGS__);                               \
    case 32 * 4 + PREC_APPLY: return F<32, PREC_APPLY>(__VA_ARGS__);               \
    case 64 * 4 + PREC_APPLY: return F<64, PREC_APPLY>(__VA_ARGS__);               \
    case 128 * 4 + PREC_APPLY: return F<128, PREC_APPLY>(__VA_ARGS__);             \
    case 256 * 4 + PREC_APPLY: return F<256, PREC_APPLY>(__VA_ARGS__);             \
    default: return hipErrorInvalidValue;                                          \
    }

hipError_t launch_level(int nb, int prec, const KArgs& a, int32_t unit_base, int32_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    BB_NP_CASES(launch_level_np, a, unit_base, count, s)
}

hipError_t launch_persistent(int nb, int prec, const KArgs& a, int32_t workgroups, hipStream_t s) {
    BB_NP_CASES(launch_persistent_np, a, workgroups, s)
}
#endif  // BB_KERNELS_COMMON

}  // namespace bbk
