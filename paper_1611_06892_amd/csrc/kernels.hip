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
// One workgroup of 256 threads (4 wave64) executes one work unit.  Panels keep
// the tile in LDS and run one Householder step per column; updates are three
// FP64 MFMA contractions (v_mfma_f64_16x16x4) over a column strip of the
// trailing tile(s), with the strip staged in LDS.
#include "kernels.hpp"

namespace bbk {

namespace {

constexpr int NT = 256;          // threads per workgroup
typedef double d4 __attribute__((ext_vector_type(4)));

enum : int { K_GEQRT = 0, K_TSQRT = 1, K_TTQRT = 2, K_UNMQR = 3, K_TSMQR = 4, K_TTMQR = 5 };

template <int NB>
struct Shape {
    static constexpr int LDX = NB + 1;                 // odd LDS stride: column walks hit distinct banks
    static constexpr int NS = NB >= 64 ? 64 : NB;      // update strip width
    static constexpr int PANEL = NB * LDX + 3 * NB + 8;
    static constexpr int UPD = 2 * NS * LDX;
    static constexpr int LDS = PANEL > UPD ? PANEL : UPD;   // doubles
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
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
};

__device__ __forceinline__ TileView view(const KArgs& a, int pr, int pc, int trans, int nb) {
    TileView t;
    t.base = a.A + (int64_t)pr * nb + (int64_t)pc * nb * a.lda;
    t.ld = a.lda;
    t.trans = trans;
    int prow = (int)min((int64_t)nb, a.m - (int64_t)pr * nb);
    int pcol = (int)min((int64_t)nb, a.n - (int64_t)pc * nb);
    t.vr = trans ? pcol : prow;
    t.vc = trans ? prow : pcol;
    return t;
}

// Copy logical columns [c0, c0+W) of a tile into LDS (column-major, stride ld),
// zero-filling the padding.  The thread-to-element map follows the physical
// layout so global accesses are contiguous for both frames.
template <int NB, int W>
__device__ __forceinline__ void load_block(const TileView& t, int c0, double* s, int ld) {
    const int tid = threadIdx.x;
    if (!t.trans) {
        for (int e = tid; e < NB * W; e += NT) {
            int r = e % NB, c = e / NB;
            s[r + c * ld] = (r < t.vr && c0 + c < t.vc) ? *t.ptr(r, c0 + c) : 0.0;
        }
    } else {
        for (int e = tid; e < NB * W; e += NT) {
            int c = e % W, r = e / W;
            s[r + c * ld] = (r < t.vr && c0 + c < t.vc) ? *t.ptr(r, c0 + c) : 0.0;
        }
    }
}

// Store (mode 0), or subtract from memory (mode 1), an LDS block into logical
// columns [c0, c0+W) of a tile; padding is skipped.
template <int NB, int W, int MODE>
__device__ __forceinline__ void store_block(const TileView& t, int c0, const double* s, int ld) {
    const int tid = threadIdx.x;
    if (!t.trans) {
        for (int e = tid; e < NB * W; e += NT) {
            int r = e % NB, c = e / NB;
            if (r < t.vr && c0 + c < t.vc) {
                double* g = t.ptr(r, c0 + c);
                *g = MODE ? *g - s[r + c * ld] : s[r + c * ld];
            }
        }
    } else {
        for (int e = tid; e < NB * W; e += NT) {
            int c = e % W, r = e / W;
            if (r < t.vr && c0 + c < t.vc) {
                double* g = t.ptr(r, c0 + c);
                *g = MODE ? *g - s[r + c * ld] : s[r + c * ld];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Panel kernels: GEQRT (kind 0), TSQRT (1), TTQRT (2).
//
// GEQRT factors tile X = T1: R overwrites its upper triangle, zeros below;
// V (unit lower triangular) goes to the task's record.  TSQRT/TTQRT factor
// [R1; X2] with R1 = T1 upper triangular and X2 = T2 square (TS) or upper
// triangular (TT): R1 is updated in place, X2 is zeroed, and V holds the lower
// parts of the reflectors (their upper parts are unit vectors e_c), which is
// full for TS and upper triangular for TT.
//
// Record layout (FP64, column-major, nb x nb each): V, V^T, T^T.
// T is formed from G = V^T V (strictly upper part, accumulated while the
// panel is factored, from the dot products of the reflector of column c with
// the finished columns j < c) by the forward recurrence
//   T(c,c) = tau_c,   T(0:c-1, c) = -tau_c T(0:c-1, 0:c-1) G(0:c-1, c),
// evaluated row by row: row i of T depends only on row i and on G.
// ---------------------------------------------------------------------------
template <int NB>
__device__ void panel(const KArgs& a, const DevTask& tk, double* lds) {
    using S = Shape<NB>;
    constexpr int LDX = S::LDX;
    constexpr int TPC = NT / NB;           // threads per column
    static_assert(NT % NB == 0 && TPC <= 64, "tile size");
    double* X = lds;
    double* tau = X + NB * LDX;
    double* rrow = tau + NB;               // two buffers of NB: R1 rows c and c+1
    double* sh = rrow + 2 * NB;
    const int tid = threadIdx.x;
    const bool pair = tk.kind != K_GEQRT;
    const bool tt = tk.kind == K_TTQRT;

    const TileView T1 = view(a, tk.r1, tk.c1, tk.trans, NB);
    TileView T2 = T1;
    if (pair) T2 = view(a, tk.r2, tk.c2, tk.trans, NB);
    double* rec = a.vt + (int64_t)tk.slot * a.slot_stride;
    double* gV = rec;
    double* gVt = rec + NB * NB;
    double* gTt = rec + 2 * NB * NB;       // holds G during the factorization

    load_block<NB, NB>(pair ? T2 : T1, 0, X, LDX);
    if (pair)
        for (int jj = tid; jj < NB; jj += NT) rrow[jj] = (0 < T1.vr && jj < T1.vc) ? *T1.ptr(0, jj) : 0.0;
    __syncthreads();

    const int j = tid / TPC, h = tid % TPC;
    for (int c = 0; c < NB; ++c) {
        double* rr = rrow + (c & 1) * NB;
        const int vlo = pair ? 0 : c + 1;      // rows of X holding the reflector's tail
        const int vhi = tt ? c + 1 : NB;
        if (tid < 64) {
            double ss = 0.0;
            for (int r = vlo + tid; r < vhi; r += 64) {
                double x = X[r + c * LDX];
                ss += x * x;
            }
            ss = wave_sum(ss);
            if (tid == 0) {
                double alpha = pair ? rr[c] : X[c + c * LDX];
                double t = 0.0, beta = alpha, scale = 0.0;
                if (ss != 0.0) {
                    double nrm = hypot(alpha, sqrt(ss));
                    beta = alpha >= 0.0 ? -nrm : nrm;
                    t = (beta - alpha) / beta;
                    scale = 1.0 / (alpha - beta);
                }
                tau[c] = t;
                sh[0] = scale;
                if (pair) rr[c] = beta; else X[c + c * LDX] = beta;
            }
        }
        if (pair && c + 1 < NB) {              // prefetch R1 row c+1 (untouched by step c)
            double* rn = rrow + ((c + 1) & 1) * NB;
            for (int jj = tid; jj < NB; jj += NT)
                if (jj >= c + 1) rn[jj] = (c + 1 < T1.vr && jj < T1.vc) ? *T1.ptr(c + 1, jj) : 0.0;
        }
        __syncthreads();
        const double tc = tau[c];
        if (tc != 0.0) {
            const double scale = sh[0];
            for (int r = vlo + tid; r < vhi; r += NT) X[r + c * LDX] *= scale;
        }
        __syncthreads();
        if (tc != 0.0 && j != c) {
            double d = 0.0;
            if (h == 0) d = (j > c) ? (pair ? rr[j] : X[c + j * LDX]) : (pair ? 0.0 : X[c + j * LDX]);
            for (int r = vlo + h; r < vhi; r += TPC) d += X[r + c * LDX] * X[r + j * LDX];
            d = group_sum<TPC>(d);
            if (j > c) {
                const double w = tc * d;
                for (int r = vlo + h; r < vhi; r += TPC) X[r + j * LDX] -= w * X[r + c * LDX];
                if (h == 0) {
                    if (pair) rr[j] -= w; else X[c + j * LDX] -= w;
                }
            } else if (h == 0) {
                gTt[j + c * NB] = d;           // G(j, c) = u_j . u_c
            }
        }
        __syncthreads();
        if (pair)
            for (int jj = tid; jj < NB; jj += NT)
                if (jj >= c && c < T1.vr && jj < T1.vc) *T1.ptr(c, jj) = rr[jj];
    }
    __syncthreads();

    // Outputs: R / zeros into the matrix, V and V^T into the record.
    if (!pair) {
        for (int e = tid; e < NB * NB; e += NT) {
            int r = e % NB, c = e / NB;
            double x = X[r + c * LDX];
            gV[r + c * NB] = r > c ? x : (r == c ? 1.0 : 0.0);
        }
        for (int e = tid; e < NB * NB; e += NT) {
            int c = e % NB, r = e / NB;        // V^T(c, r) = V(r, c)
            double x = X[r + c * LDX];
            gVt[c + r * NB] = r > c ? x : (r == c ? 1.0 : 0.0);
        }
        // R into T1 (logical upper triangle, zeros below), masked by the padding.
        if (!T1.trans) {
            for (int e = tid; e < NB * NB; e += NT) {
                int r = e % NB, c = e / NB;
                if (r < T1.vr && c < T1.vc) *T1.ptr(r, c) = r <= c ? X[r + c * LDX] : 0.0;
            }
        } else {
            for (int e = tid; e < NB * NB; e += NT) {
                int c = e % NB, r = e / NB;
                if (r < T1.vr && c < T1.vc) *T1.ptr(r, c) = r <= c ? X[r + c * LDX] : 0.0;
            }
        }
    } else {
        for (int e = tid; e < NB * NB; e += NT) {
            int r = e % NB, c = e / NB;
            gV[r + c * NB] = (tt && r > c) ? 0.0 : X[r + c * LDX];
        }
        for (int e = tid; e < NB * NB; e += NT) {
            int c = e % NB, r = e / NB;
            gVt[c + r * NB] = (tt && r > c) ? 0.0 : X[r + c * LDX];
        }
        if (!T2.trans) {
            for (int e = tid; e < NB * NB; e += NT) {
                int r = e % NB, c = e / NB;
                if (r < T2.vr && c < T2.vc) *T2.ptr(r, c) = 0.0;
            }
        } else {
            for (int e = tid; e < NB * NB; e += NT) {
                int c = e % NB, r = e / NB;
                if (r < T2.vr && c < T2.vc) *T2.ptr(r, c) = 0.0;
            }
        }
    }
    __syncthreads();

    // T from G: packed strictly-upper G and packed upper T share the X area.
    double* Gp = X;                          // G(l, c), l < c  at c(c-1)/2 + l
    double* Tp = X + NB * (NB - 1) / 2;      // T(i, c), i <= c at c(c+1)/2 + i
    for (int e = tid; e < NB * NB; e += NT) {
        int l = e % NB, c = e / NB;
        if (l < c) Gp[c * (c - 1) / 2 + l] = tau[c] != 0.0 ? gTt[l + c * NB] : 0.0;
    }
    __syncthreads();
    {
        constexpr int TPR = NT / NB;         // threads per row of T
        const int i = tid / TPR, hh = tid % TPR;
        if (hh == 0) Tp[i * (i + 1) / 2 + i] = tau[i];
        for (int c = i + 1; c < NB; ++c) {
            double s = 0.0;
            for (int l = i + hh; l < c; l += TPR) s += Tp[l * (l + 1) / 2 + i] * Gp[c * (c - 1) / 2 + l];
            s = group_sum<TPR>(s);
            if (hh == 0) Tp[c * (c + 1) / 2 + i] = -tau[c] * s;
            // the other lanes of the group read T(i, c) in later iterations;
            // LDS operations of one wave complete in order.
        }
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += NT) {
        int c = e % NB, i = e / NB;           // T^T(c, i) = T(i, c)
        gTt[c + i * NB] = i <= c ? Tp[c * (c + 1) / 2 + i] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Update kernels: UNMQR (kind 3), TSMQR (4), TTMQR (5), on the logical column
// strip [c0, c0+NS) of the trailing tile(s):
//   W  = C1 + V^T C2          (C1 absent for UNMQR: W = V^T C)
//   W  = T^T W
//   C1 = C1 - W ,  C2 = C2 - V W
// The three products run on v_mfma_f64_16x16x4.  Operand layouts of that
// instruction (wave64): A (16x4) lane l holds A(l%16, l/16); B (4x16) lane l
// holds B(l/16, l%16); result element r (0..3) of lane l is D(4r + l/16, l%16).  The first operand comes straight from the record (V, V^T, T^T
// are stored so that 16 consecutive lanes read 16 consecutive doubles); the
// second from the LDS copy of the strip.
// ---------------------------------------------------------------------------
template <int NB>
__device__ void update(const KArgs& a, const DevTask& tk, int part, double* lds) {
    using S = Shape<NB>;
    constexpr int NS = S::NS, LD = S::LDX;
    constexpr int MT = NB / 16, NTL = NS / 16;
    constexpr int WR = MT >= 4 ? 4 : MT, WC = 4 / WR;
    constexpr int RPW = MT / WR, CPW = NTL / WC;
    static_assert(WR * WC == 4 && RPW * WR == MT && CPW * WC == NTL, "wave tiling");
    double* Cs = lds;               // C2 strip, NB x NS
    double* Ws = lds + NS * LD;     // C1 strip, then W
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int c0 = part * NS;
    const bool hasC1 = tk.kind != K_UNMQR;

    const TileView T2 = view(a, tk.r2, tk.c2, tk.trans, NB);
    if (c0 >= T2.vc) return;                  // strip lies in the padding: nothing to do
    TileView T1 = T2;
    if (hasC1) T1 = view(a, tk.r1, tk.c1, tk.trans, NB);

    load_block<NB, NS>(T2, c0, Cs, LD);
    if (hasC1) {
        load_block<NB, NS>(T1, c0, Ws, LD);
    } else {
        for (int e = tid; e < NB * NS; e += NT) Ws[(e % NB) + (e / NB) * LD] = 0.0;
    }
    __syncthreads();

    const double* rec = a.vt + (int64_t)tk.slot * a.slot_stride;
    const double* gV = rec;
    const double* gVt = rec + NB * NB;
    const double* gTt = rec + 2 * NB * NB;
    const int row0 = (w % WR) * RPW * 16, col0 = (w / WR) * CPW * 16;
    const int li = lane & 15, lk = lane >> 4;
    d4 acc[RPW][CPW];

    auto load_acc = [&](const double* src) {
#pragma unroll
        for (int ri = 0; ri < RPW; ++ri)
#pragma unroll
            for (int ci = 0; ci < CPW; ++ci)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[ri][ci][r] = src[(row0 + ri * 16 + 4 * r + lk) + (col0 + ci * 16 + li) * LD];
    };
    auto store_acc = [&](double* dst) {
#pragma unroll
        for (int ri = 0; ri < RPW; ++ri)
#pragma unroll
            for (int ci = 0; ci < CPW; ++ci)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    dst[(row0 + ri * 16 + 4 * r + lk) + (col0 + ci * 16 + li) * LD] = acc[ri][ci][r];
    };
    // acc += sign * A(rows, k) * Bs(k, cols), A(i, k) = gA[i + k NB], Bs from LDS.
    auto gemm = [&](const double* gA, const double* Bs, double sign) {
        for (int k = 0; k < NB; k += 4) {
            double av[RPW], bv[CPW];
#pragma unroll
            for (int ri = 0; ri < RPW; ++ri) av[ri] = sign * gA[(row0 + ri * 16 + li) + (k + lk) * NB];
#pragma unroll
            for (int ci = 0; ci < CPW; ++ci) bv[ci] = Bs[(k + lk) + (col0 + ci * 16 + li) * LD];
#pragma unroll
            for (int ri = 0; ri < RPW; ++ri)
#pragma unroll
                for (int ci = 0; ci < CPW; ++ci)
                    acc[ri][ci] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ri], bv[ci], acc[ri][ci], 0, 0, 0);
        }
    };

    // W = C1 + V^T C2   (A operand V^T(i, k) = gVt[i + k NB])
    load_acc(Ws);
    gemm(gVt, Cs, 1.0);
    store_acc(Ws);                            // each wave owns its block of Ws
    __syncthreads();
    // W = T^T W
#pragma unroll
    for (int ri = 0; ri < RPW; ++ri)
#pragma unroll
        for (int ci = 0; ci < CPW; ++ci) acc[ri][ci] = d4{0.0, 0.0, 0.0, 0.0};
    gemm(gTt, Ws, 1.0);
    __syncthreads();
    store_acc(Ws);
    __syncthreads();
    // C1 -= W
    if (hasC1) store_block<NB, NS, 1>(T1, c0, Ws, LD);
    // C2 = C2 - V W
    load_acc(Cs);
    gemm(gV, Ws, -1.0);
    store_acc(Cs);
    __syncthreads();
    store_block<NB, NS, 0>(T2, c0, Cs, LD);
}

template <int NB>
__device__ __forceinline__ void run_unit(const KArgs& a, int task, int part, double* lds) {
    const DevTask tk = a.tasks[task];      // task is wave-uniform: scalar loads
    if (tk.kind <= K_TTQRT) panel<NB>(a, tk, lds);
    else update<NB>(a, tk, part, lds);
}

}  // namespace

// One launch per topological level: block b runs unit unit_base + b.
template <int NB>
__global__ __launch_bounds__(NT) void level_kernel(KArgs a, int32_t unit_base) {
    __shared__ double lds[Shape<NB>::LDS];
    const int2 u = a.units[unit_base + blockIdx.x];
    run_unit<NB>(a, u.x, u.y, lds);
}

// Persistent scheduler.  Each workgroup repeatedly takes the next ticket (a
// unit in a precomputed topological priority order), waits until the unit's
// task has no unfinished predecessor parts, runs it and decrements the
// counters of the task's successors.  Tickets are only taken by running
// workgroups and every predecessor of a ticket has a smaller ticket, so the
// lowest unfinished ticket can always proceed: no deadlock for any grid size.
// A wall-clock watchdog bounds every wait; on expiry (or when another
// workgroup reports an error) the workgroup records the error and exits.
template <int NB>
__global__ __launch_bounds__(NT) void persistent_kernel(KArgs a) {
    __shared__ double lds[Shape<NB>::LDS];
    __shared__ int s_unit, s_stop;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            s_unit = __hip_atomic_fetch_add(&a.ctrl[CTRL_TICKET], 1, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
            s_stop = 0;
        }
        __syncthreads();
        // The ticket is the same for every thread; readfirstlane makes that
        // visible to the compiler so the loop exits stay uniform.  (With
        // exits it must treat as divergent, the loop is restructured so that
        // lanes other than 0 re-enter the top barrier before lane 0 fetched
        // the next ticket.)
        const int u = __builtin_amdgcn_readfirstlane(s_unit);
        if (u >= a.nunits) break;
        const int2 un0 = a.units[u];
        const int2 un = make_int2(__builtin_amdgcn_readfirstlane(un0.x),
                                  __builtin_amdgcn_readfirstlane(un0.y));
        if (tid == 0) {
            const uint64_t t0 = wall_clock64();
            for (;;) {
                int d = __hip_atomic_load(&a.deps[un.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (d <= 0) break;
                if (__hip_atomic_load(&a.ctrl[CTRL_ERROR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    s_stop = 1;
                    break;
                }
                if ((int64_t)(wall_clock64() - t0) > a.watchdog_ticks) {
                    __hip_atomic_store(&a.ctrl[CTRL_ERROR], 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_stop = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_stop)) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        run_unit<NB>(a, un.x, un.y, lds);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) {
            const int s0 = a.succ_off[un.x], s1 = a.succ_off[un.x + 1];
            for (int s = s0; s < s1; ++s)
                __hip_atomic_fetch_add(&a.deps[a.succ_idx[s]], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&a.ctrl[CTRL_DONE], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

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

bool nb_supported(int nb) { return nb == 32 || nb == 64 || nb == 128; }

hipError_t launch_level(int nb, const KArgs& a, int32_t unit_base, int32_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch (nb) {
    case 32: hipLaunchKernelGGL(level_kernel<32>, dim3(count), dim3(NT), 0, s, a, unit_base); break;
    case 64: hipLaunchKernelGGL(level_kernel<64>, dim3(count), dim3(NT), 0, s, a, unit_base); break;
    case 128: hipLaunchKernelGGL(level_kernel<128>, dim3(count), dim3(NT), 0, s, a, unit_base); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_persistent(int nb, const KArgs& a, int32_t workgroups, hipStream_t s) {
    switch (nb) {
    case 32: hipLaunchKernelGGL(persistent_kernel<32>, dim3(workgroups), dim3(NT), 0, s, a); break;
    case 64: hipLaunchKernelGGL(persistent_kernel<64>, dim3(workgroups), dim3(NT), 0, s, a); break;
    case 128: hipLaunchKernelGGL(persistent_kernel<128>, dim3(workgroups), dim3(NT), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bbk
