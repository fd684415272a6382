// The two steps after the band reduction (the GE2VAL pipeline of Sections 2
// and 6.2): BND2BD, band to bidiagonal by bulge chasing, and BD2VAL,
// singular values of the bidiagonal, on gfx950.
//
// BND2BD.  The n x n upper band of bandwidth nb is copied into a band work
// array with room for the fill of the chase (nb - 1 diagonals below the
// main one, 2 nb - 1 above), column-major by diagonal offset:
//     W[(i - j + 2 nb - 1) + j * 3 nb]  holds entry (i, j).
// Sweep k clears row k beyond its superdiagonal and chases the bulge this
// makes down the band, one block of nb columns per step.  Step t of sweep k
// works at column c = k + 1 + t nb:
//   * a reflector from the right clears row rr (rr = k for t = 0, else
//     c - nb, the row the previous step filled) beyond column c; it is
//     applied to rows rr+1 .. c+nb-1 of columns c .. c+nb-1;
//   * a reflector from the left clears column c below the diagonal; it is
//     applied to rows c .. c+nb-1 of columns c+1 .. c+2nb-1.
// Only the first row or column of a bulge is cleared; the rest is cleared
// by later sweeps.  Step t of sweep k+1 touches one entry that step t+2 of
// sweep k also touches (row k+1+(t+1)nb, column k+1+(t+2)nb, the first
// entry of the row that step clears) and nothing of a later step, so it may
// start once sweep k has finished step t+1 and has written that entry's
// final value in step t+2 (its progress counter counts half steps): about
// two and a half steps separate consecutive sweeps, and about n / (2.5 nb)
// sweeps run at once.
//
// One persistent launch: each workgroup takes the next sweep (a ticket from
// an atomic counter, so a sweep is only ever waited for by a later one that
// a running workgroup holds: no deadlock for any grid) and runs its steps in
// order, each after the previous sweep's progress counter allows it.  The
// band array is written and read with agent-scope stores and loads (past the
// XCD's L2, at the coherence point), so a counter is published once every
// wave has waited for its own memory operations and the workgroup has met,
// with no L2 write-back, and the loads that follow a counter's load see every
// store performed before it was written, with no L2 invalidation; a
// wall-clock watchdog bounds every wait.
//
// BD2VAL.  The singular values of the bidiagonal (d, e) are the positive
// eigenvalues of the 2n x 2n Golub-Kahan matrix, symmetric tridiagonal with
// a zero diagonal and off-diagonal d1, e1, d2, ..., dn.  A Sturm count (the
// signs of the pivots of T - x I, safeguarded against zero pivots) gives the
// number of singular values below x; a group of lanes narrows the interval
// of one singular value by multisection, so all n are found at once (the
// bisection method of the paper's list of BD2VAL methods, chosen over the
// serial bidiagonal QR for its parallelism).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>

#include "bidiag.h"

namespace bbg {

constexpr int NT = 256;                 // threads of the chase kernel (4 waves)
constexpr int NW = NT / 64;
constexpr int MAX_NB = 256;
enum : int { G_ERROR = 1, G_HEAD = 32, G_WORDS = 64 };

struct ChaseArgs {
    double* W;
    int64_t ldw;          // 3 nb
    int64_t n;
    int nb;
    int nsweeps;
    int32_t* ctrl;        // G_* words
    int32_t* prog;        // steps finished, per sweep
    int32_t* bar;         // group barrier arrivals, per sweep (nb > LDS_NB)
    int group;            // workgroups per sweep (nb > LDS_NB; 1 for the LDS steps)
    int64_t watchdog_ticks;
};

__host__ __device__ inline int64_t nsteps(int64_t n, int nb, int64_t k) {
    return (n - 1 - k + nb - 1) / nb;
}

__device__ __forceinline__ double* at(const ChaseArgs& a, int64_t i, int64_t j) {
    return a.W + (i - j + 2 * a.nb - 1) + j * a.ldw;
}

// Stores to the band array: agent-scope stores, performed past the XCD's L2
// at the device's coherence point, so no L2 line of the band array is ever
// dirty and a publication needs no L2 write-back, only each wave's wait for
// its own stores (the same protocol as the band reduction's scheduler).
__device__ __forceinline__ void st(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads from the band array: agent-scope loads, served at the coherence
// point, so they see every store that completed before the progress counter
// they follow was written, with no L2 invalidation.
__device__ __forceinline__ double ld(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int aload(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Sum over the workgroup; the result is returned to every thread.
__device__ __forceinline__ double block_sum(double x, double* red) {
    x = wave_sum(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w];
    return s;
}

// Householder reflector of the L values in v[0 .. L-1] (LDS), in place:
// v becomes (1, x2 / (alpha - beta)); returns tau (0: the identity) and
// beta, the value left in the first position.
__device__ __forceinline__ double reflector(double* v, int L, double* red, double* beta_out) {
    const int tid = threadIdx.x;
    const double x = tid < L ? v[tid] : 0.0;
    const double ss = block_sum(tid >= 1 && tid < L ? x * x : 0.0, red);
    const double alpha = v[0];
    __syncthreads();                      // every thread has read v[0] and red
    if (ss == 0.0) {
        *beta_out = alpha;
        return 0.0;
    }
    const double beta = -copysign(sqrt(alpha * alpha + ss), alpha);
    const double scal = 1.0 / (alpha - beta);
    if (tid < L) v[tid] = tid == 0 ? 1.0 : x * scal;
    __syncthreads();
    *beta_out = beta;
    return (beta - alpha) / beta;
}

// Wait until *p >= target (wave 0 polls), then acquire.  false: stop (an
// error was reported, or the watchdog fired here).
__device__ bool wait_geq(const ChaseArgs& a, const int32_t* p, int target, int* flag) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int ok = 1;
        const uint64_t t0 = wall_clock64();
        for (;;) {
            int v = 0, err = 0;
            if (lane == 0) {
                v = aload(p);
                if (v < target) err = aload(&a.ctrl[G_ERROR]);
            }
            v = __builtin_amdgcn_readfirstlane(v);
            if (v >= target) break;
            if (__builtin_amdgcn_readfirstlane(err) != 0) {
                ok = 0;
                break;
            }
            if ((int64_t)(wall_clock64() - t0) > a.watchdog_ticks) {
                if (lane == 0)
                    __hip_atomic_store(&a.ctrl[G_ERROR], BB_ETIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (lane == 0) *flag = ok;
        // no acquire: the band array is read with agent-scope loads, issued
        // only after this load of the counter has returned
    }
    __syncthreads();
    const int ok = __builtin_amdgcn_readfirstlane(*flag);
    return ok != 0;
}

// Step t of sweep k for nb > LDS_NB, on the band array in global memory, by
// member g of the group of a.group workgroups that runs the sweep (with
// a group of one, as bb_bnd2bd_group allows, no group barriers).  Only
// about n / (2.5 nb) sweeps can run at once (26 at n = 16384, nb = 256), so
// each sweep's steps are spread over a group to use the other CUs.
//   * Every member reads row rr and forms the right reflector (the same
//     arithmetic, the same result); the right update M -= tau (M v) v^T of
//     rows rr+1 .. c+L-1 of columns c .. c+L-1 is split by rows, TPR lanes a
//     row, in two passes (the row products, then the update).  Every sum
//     is taken in the same order whatever the group size, so the result
//     does not depend on it.
//   * Group barrier: column c is final.
//   * Every member reads column c and forms the left reflector; the left
//     update M -= tau v (v^T M) of rows c .. c+L-1 of columns c+1 .. ce-1 is
//     split by chunks of CHUNK columns, one row per thread, the column sums
//     formed through LDS, each entry read and written once.
//   * Group barrier: the step's updates are done.  Member 0 then writes the
//     cleared row rr and column c (beta, zeros), which no member reads later
//     in the step or in the next one (the corner of row rr went out with the
//     half step, after the first group barrier).
// In the band array entry (i, j+1) follows entry (i, j) at a distance of
// ldw - 1.  false: an error was reported or the watchdog fired.
constexpr int GROUP_NB = 64;
constexpr int GROUP_MAX = 16;
constexpr int CHUNK = 32;
constexpr int PLD = NT + 8;              // LDS stride of a product column: lanes 8u+s hit distinct banks
constexpr int RB = 32;                   // loads in flight per thread in the row passes
constexpr int TPR = 4;                   // lanes a row in the right update

// A barrier for LDS traffic only: it waits for this wave's LDS operations,
// not for its global loads, so loads issued before it stay in flight.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The half of step t of sweep k that the next sweep waits for: the corner
// (rr, c), the first entry of the row the right reflector clears, is final
// (beta; alpha when the row needs no reflector).  Thread 0 stores it (the
// LDS steps hold a newer value than memory even then), waits for the store
// and moves the progress counter to 2t+1; every earlier store of the sweep
// has completed too, each wave having waited for its own before the
// preceding barrier (2T marks the whole sweep).  The step's own stores leave
// the corner alone afterwards: the next sweep changes it from here on.
__device__ __forceinline__ void publish_corner(const ChaseArgs& a, int64_t k, int64_t t, double* corner,
                                               double beta) {
    if (threadIdx.x < 64) {
        if (threadIdx.x == 0) st(corner, beta);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if (threadIdx.x == 0)
            __hip_atomic_store(&a.prog[k], (int)(2 * t + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Publish value through *p after every wave's earlier accesses.  Each wave
// first waits for its own loads and stores to complete (the barrier alone
// does not wait for them; the band array's stores are agent-scope, so a
// completed one has been performed past the XCD's L2 and no write-back is
// needed), the workgroup meets, and thread 0 stores or adds.
__device__ __forceinline__ void publish_after_barrier(int32_t* p, int value, bool add) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x < 64) {
        if (threadIdx.x == 0) {
            if (add) __hip_atomic_fetch_add(p, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else __hip_atomic_store(p, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__device__ bool group_barrier(const ChaseArgs& a, int64_t k, int target, int* flag) {
    publish_after_barrier(&a.bar[k], 1, true);
    return wait_geq(a, &a.bar[k], target, flag);
}

__device__ bool chase_step(const ChaseArgs& a, int64_t k, int64_t t, int g, double* v, double* red, double* P,
                           double* wq, int* flag) {
    const int tid = threadIdx.x;
    const int nb = a.nb;
    const int G = a.group;
    const int64_t c = k + 1 + t * nb;
    const int64_t rr = t == 0 ? k : c - nb;
    const int L = (int)(a.n - c < nb ? a.n - c : nb);
    const int64_t s = a.ldw - 1;

    // right reflector: clear row rr beyond column c; the previous step's
    // stores complete in every wave before the reflector's barriers, so the
    // corner's release below covers them too
    if (tid < L) v[tid] = ld(at(a, rr, c + tid));
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    double beta_r, beta_l;
    const double tau_r = reflector(v, L, red, &beta_r);
    if (G == 1) publish_corner(a, k, t, at(a, rr, c), beta_r);
    if (tau_r != 0.0) {
        const int R = (int)(c + L - 1 - rr);          // rows rr+1 .. c+L-1
        const int rpm = (R + G - 1) / G;              // rows of this member: r0 .. r1-1
        const int r0 = g * rpm, r1 = r0 + rpm < R ? r0 + rpm : R;
        // TPR lanes a row whatever the group size, so that every row's
        // products are summed in the same order for any group
        constexpr int tpr = TPR;
        const int part = tid & (tpr - 1);
        // the tpr lanes of a row are adjacent and share its loop trips, so
        // the shuffles that sum their parts stay within active lanes
        for (int r = r0 + tid / tpr; r < r1; r += NT / tpr) {
            double* p = at(a, rr + 1 + r, c);
            double w0 = 0.0, w1 = 0.0;
            int j = part;
            for (; j + (RB - 1) * tpr < L; j += RB * tpr) {
                double x[RB];
#pragma unroll
                for (int u = 0; u < RB; ++u) x[u] = ld(p + (j + u * tpr) * s);
#pragma unroll
                for (int u = 0; u < RB; u += 2) {
                    w0 += x[u] * v[j + u * tpr];
                    w1 += x[u + 1] * v[j + (u + 1) * tpr];
                }
            }
            for (; j < L; j += tpr) w0 += ld(p + j * s) * v[j];
            double w = w0 + w1;
            for (int o = 1; o < tpr; o *= 2) w += __shfl_xor(w, o, 64);
            w *= tau_r;
            j = part;
            for (; j + (RB - 1) * tpr < L; j += RB * tpr) {
                double x[RB];
#pragma unroll
                for (int u = 0; u < RB; ++u) x[u] = ld(p + (j + u * tpr) * s);
#pragma unroll
                for (int u = 0; u < RB; ++u) st(p + (j + u * tpr) * s, x[u] - w * v[j + u * tpr]);
            }
            for (; j < L; j += tpr) st(p + j * s, ld(p + j * s) - w * v[j]);
        }
    }
    if (G > 1) {
        // every member has read row rr: its corner may now change
        if (!group_barrier(a, k, (int)(2 * t + 1) * G, flag)) return false;
        if (g == 0) publish_corner(a, k, t, at(a, rr, c), beta_r);
    }
    __syncthreads();

    // left reflector: clear column c below the diagonal
    if (tid < L) v[tid] = ld(at(a, c + tid, c));
    __syncthreads();
    const double tau_l = reflector(v, L, red, &beta_l);
    if (tau_l != 0.0) {
        const int64_t ce = c + 2 * nb < a.n ? c + 2 * nb : a.n;
        const int C = (int)(ce - c - 1);              // columns c+1 .. ce-1
        const double vi = tid < L ? v[tid] : 0.0;
        double* p = tid < L ? at(a, c + tid, c + 1) : nullptr;
        const int cu = tid >> 3, cs = tid & 7;        // column sums: column cu, rows cs + 8 r
        // the next chunk's loads are issued before this chunk's sums
        double x[CHUNK];
        int q0 = g * CHUNK;
#pragma unroll
        for (int u = 0; u < CHUNK; ++u) x[u] = (tid < L && q0 + u < C) ? ld(p + (q0 + u) * s) : 0.0;
        for (; q0 < C; q0 += G * CHUNK) {
#pragma unroll
            for (int u = 0; u < CHUNK; ++u) P[u * PLD + tid] = vi * x[u];
            lds_barrier();
            const int qn = q0 + G * CHUNK;
            double y[CHUNK];
#pragma unroll
            for (int u = 0; u < CHUNK; ++u) y[u] = (tid < L && qn + u < C) ? ld(p + (qn + u) * s) : 0.0;
            double sum = 0.0;
            for (int r = cs; r < L; r += 8) sum += P[cu * PLD + r];
            sum += __shfl_xor(sum, 1, 64);
            sum += __shfl_xor(sum, 2, 64);
            sum += __shfl_xor(sum, 4, 64);
            if (cs == 0) wq[cu] = tau_l * sum;
            lds_barrier();
            if (tid < L) {
#pragma unroll
                for (int u = 0; u < CHUNK; ++u)
                    if (q0 + u < C) st(p + (q0 + u) * s, x[u] - vi * wq[u]);
            }
#pragma unroll
            for (int u = 0; u < CHUNK; ++u) x[u] = y[u];
        }
    }
    if (G > 1 && !group_barrier(a, k, (int)(2 * t + 2) * G, flag)) return false;
    if (g == 0) {
        if (tau_r != 0.0 && tid >= 1 && tid < L) st(at(a, rr, c + tid), 0.0);   // the corner went out early
        if (tau_l != 0.0 && tid < L) st(at(a, c + tid, c), tid == 0 ? beta_l : 0.0);
    }
    __syncthreads();
    return true;
}

// Reflector of the L <= 64 values x[i ld] (LDS), formed by wave 0 alone: v
// gets (1, x2 / (alpha - beta)), x gets (beta, 0, ..), sc[0] tau (0: the
// identity, x left as it is).  The caller synchronizes after it.
__device__ __forceinline__ void reflector_wave(double* x, int ld, int L, double* v, double* sc) {
    const int lane = threadIdx.x;
    const double xi = lane < L ? x[lane * ld] : 0.0;
    const double ss = wave_sum(lane >= 1 ? xi * xi : 0.0);
    const double alpha = __shfl(xi, 0, 64);
    double tau = 0.0;
    if (ss != 0.0) {
        const double beta = -copysign(sqrt(alpha * alpha + ss), alpha);
        const double scal = 1.0 / (alpha - beta);
        tau = (beta - alpha) / beta;
        if (lane < L) {
            v[lane] = lane == 0 ? 1.0 : xi * scal;
            x[lane * ld] = lane == 0 ? beta : 0.0;
        }
    }
    if (lane == 0) sc[0] = tau;
}

// The same step with its region staged in LDS, for nb <= LDS_NB.  The region
// is three nb x nb quadrants, each stored by column with stride LDS_LD: U
// (rows c-nb .. c-1 of columns c .. c+nb-1; only rows from rr on are in
// use), D (rows and columns c .. c+nb-1) and Q (rows c .. c+nb-1, columns
// c+nb .. c+2nb-1).  Q of step t is U of step t+1, and no other sweep
// touches it between the two (the sweep ahead finished its steps there
// before step t started, the sweep behind waits for step t+1), so it stays
// in LDS: the three buffers rotate, step t loads only D and Q (and, for
// t = 0, the row k), and stores U and D; Q reaches memory as the next
// step's U (the last step of a sweep has no Q).  Thread tid moves row
// tid % nb of columns tid / nb + j (NT / nb), all its loads issued before
// the first is used.  With the band array's column stride ldw and the
// entry (i, j+1) at ldw - 1 after (i, j), for d0 = W + 2nb - 1 + c ldw:
//     D(r, q) = d0 + r + q (ldw - 1),  U(r, q) = D(r, q) - nb,
//     Q(r, q) = D(r, q) - nb + nb ldw.
constexpr int LDS_NB = 64;
constexpr int LDS_LD = LDS_NB + 1;
// columns a thread moves, at most: cpp = NT / nb >= NT / LDS_NB, so LDS_J cpp >= nb
constexpr int LDS_J = (LDS_NB + NT / LDS_NB - 1) / (NT / LDS_NB);
static_assert(LDS_J <= 16, "per-thread staging registers");
// the updates give each row (column) of a quadrant pair two lanes, each with
// half of it in registers: 2 (2 nb - 1) <= NT lanes
constexpr int HALF = LDS_NB / 2;
static_assert(2 * (2 * LDS_NB - 1) <= NT, "one pass of lane pairs");

__device__ void chase_step_lds(const ChaseArgs& a, int64_t k, int64_t t, double* U, double* D, double* Q,
                               double* v, double* sc) {
    const int tid = threadIdx.x;
    const int nb = a.nb;
    const int64_t c = k + 1 + t * nb;
    const int L = (int)(a.n - c < nb ? a.n - c : nb);
    const int64_t nq = a.n - (c + nb);
    const int Lq = nq <= 0 ? 0 : (int)(nq < nb ? nq : nb);
    const int u0 = t == 0 ? nb - 1 : 0;          // first U row in use
    const int64_t s = a.ldw - 1;
    const int cpp = NT / nb;                     // columns moved at once
    const int tr = tid % nb, tq = tid / nb;
    const bool mover = tq < cpp && tr < L;       // D and Q rows < L exist
    const double* db = a.W + (2 * nb - 1) + c * a.ldw;
    const double* d0 = db + tr;
    const double* q0p = d0 - nb + (int64_t)nb * a.ldw;
    {
        double xd[LDS_J], xq[LDS_J];
        const double xu = t == 0 && tid < L ? ld(db + tid * s - 1) : 0.0;     // U(nb-1, tid): the row k
#pragma unroll
        for (int j = 0; j < LDS_J; ++j) {
            const int q = tq + j * cpp;
            xd[j] = mover && q < L ? ld(d0 + q * s) : 0.0;
            xq[j] = mover && q < Lq ? ld(q0p + q * s) : 0.0;
        }
        if (t == 0 && tid < L) U[(nb - 1) + tid * LDS_LD] = xu;
#pragma unroll
        for (int j = 0; j < LDS_J; ++j) {
            const int q = tq + j * cpp;
            if (mover && q < L) D[tr + q * LDS_LD] = xd[j];
            if (mover && q < Lq) Q[tr + q * LDS_LD] = xq[j];
        }
    }
    __syncthreads();

    // right reflector (wave 0): clear row rr (U row u0) beyond column c;
    // then rows U u0+1 .. nb-1 and D 0 .. L-1 take M -= tau (M v) v^T
    if (tid < 64) reflector_wave(U + u0, LDS_LD, L, v, sc);
    // the previous step's stores complete in every wave before the barrier,
    // so wave 0's release in publish_corner covers them too
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    publish_corner(a, k, t, const_cast<double*>(db) - nb + u0, U[u0]);
    const int pr = tid >> 1, ph = tid & 1;       // a pair of lanes per row (column): halves of it
    double tau = sc[0];
    if (tau != 0.0) {
        const int ru = nb - 1 - u0;
        const bool act = pr < ru + L;
        double* p = pr < ru ? U + (u0 + 1 + pr) : D + (pr - ru);
        double x[HALF];
        double w = 0.0;
#pragma unroll
        for (int u = 0; u < HALF; ++u) {
            const int j = ph * HALF + u;
            x[u] = act && j < L ? p[j * LDS_LD] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < HALF; ++u) {
            const int j = ph * HALF + u;
            if (j < L) w += x[u] * v[j];
        }
        w = tau * (w + __shfl_xor(w, 1, 64));
#pragma unroll
        for (int u = 0; u < HALF; ++u) {
            const int j = ph * HALF + u;
            if (act && j < L) p[j * LDS_LD] = x[u] - w * v[j];
        }
    }
    __syncthreads();

    // left reflector (wave 0): clear column c (D column 0) below the
    // diagonal; then D columns 1 .. L-1 and Q columns 0 .. Lq-1 take
    // M -= tau v (v^T M)
    if (tid < 64) reflector_wave(D, 1, L, v, sc);
    __syncthreads();
    tau = sc[0];
    if (tau != 0.0) {
        const bool act = pr < L - 1 + Lq;
        double* p = pr < L - 1 ? D + (pr + 1) * LDS_LD : Q + (pr - (L - 1)) * LDS_LD;
        double x[HALF];
        double w = 0.0;
#pragma unroll
        for (int u = 0; u < HALF; ++u) {
            const int i = ph * HALF + u;
            x[u] = act && i < L ? p[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < HALF; ++u) {
            const int i = ph * HALF + u;
            if (i < L) w += v[i] * x[u];
        }
        w = tau * (w + __shfl_xor(w, 1, 64));
#pragma unroll
        for (int u = 0; u < HALF; ++u) {
            const int i = ph * HALF + u;
            if (act && i < L) p[i] = x[u] - w * v[i];
        }
    }
    __syncthreads();

    // store U (rows u0 .. nb-1) and D back; Q stays for the next step
    double* ud = const_cast<double*>(d0);
    if (tq < cpp && tr >= u0) {
#pragma unroll
        for (int j = 0; j < LDS_J; ++j) {
            const int q = tq + j * cpp;
            if (q < L && (q > 0 || tr > u0)) st(ud + q * s - nb, U[tr + q * LDS_LD]);   // not the corner
        }
    }
    if (mover) {
#pragma unroll
        for (int j = 0; j < LDS_J; ++j) {
            const int q = tq + j * cpp;
            if (q < L) st(ud + q * s, D[tr + q * LDS_LD]);
        }
    }
}

template <bool TILE>
__global__ __launch_bounds__(NT) void chase_kernel(ChaseArgs a) {
    __shared__ double v[MAX_NB];
    __shared__ double red[NW];
    // TILE: the three rotating quadrant buffers; else the left update's
    // column products and sums
    __shared__ double lds[TILE ? 3 * LDS_NB * LDS_LD : CHUNK * PLD + CHUNK];
    __shared__ int sk, flag;
    const int tid = threadIdx.x;
    const int G = TILE ? 1 : a.group;
    for (;;) {
        // ticket = sweep * G + member: a group's members are consecutive
        // tickets, all taken by running workgroups before any of them can
        // be needed by a later sweep (grid >= G)
        if (tid == 0) sk = __hip_atomic_fetch_add(&a.ctrl[G_HEAD], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int ticket = __builtin_amdgcn_readfirstlane(sk);
        __syncthreads();
        const int64_t k = ticket / G;
        const int g = ticket - (int)k * G;
        if (k >= a.nsweeps) return;
        const int64_t T = nsteps(a.n, a.nb, k);
        const int64_t Tp = k > 0 ? nsteps(a.n, a.nb, k - 1) : 0;
        for (int64_t t = 0; t < T; ++t) {
            // the previous sweep's step t+1 done and step t+2 half done
            // (2t+5), or the whole sweep when it is shorter
            if (k > 0 && !wait_geq(a, &a.prog[k - 1], (int)(t + 2 < Tp ? 2 * t + 5 : 2 * Tp), &flag)) return;
            if constexpr (TILE) {
                const int u = (int)((2 * t) % 3);    // Q of step t is U of step t+1
                double* U = lds + u * LDS_NB * LDS_LD;
                double* D = lds + ((u + 1) % 3) * LDS_NB * LDS_LD;
                double* Q = lds + ((u + 2) % 3) * LDS_NB * LDS_LD;
                chase_step_lds(a, k, t, U, D, Q, v, red);   // red[0]: tau
            } else {
                if (!chase_step(a, k, t, g, v, red, lds, lds + CHUNK * PLD, &flag)) return;
            }
            // The next sweep waits for half steps (2t+5: step t+1 done, the
            // corner of step t+2 final), whose release also covers every
            // earlier store of the sweep; only the last step is published
            // whole (2T).  The barrier keeps a step's LDS buffers until
            // every wave has stored them.
            if (g == 0 && t + 1 == T) publish_after_barrier(&a.prog[k], (int)(2 * T), false);
            else __syncthreads();
        }
    }
}

// Copy the upper band of B into W (zero elsewhere), clear the control words
// (the error word too unless keep_error: then a status already there, such as
// the band reduction's in the one-shot pipeline, stops the chase at its
// first wait and stays visible) and the progress counters.  Entry (i, j) of
// the band is B[i rs + j cs]: rs = 1, cs = ldb for an upper band stored as
// is, rs = ldb, cs = 1 for the transpose of a lower band.
__global__ void pack_kernel(const double* B, int64_t rs, int64_t cs, int64_t n, int nb, double* W, int64_t ldw,
                            int32_t* ctrl, int32_t* prog, int32_t* bar, int nsweeps, int keep_error) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (g < G_WORDS && !(keep_error && g == G_ERROR)) ctrl[g] = 0;
    for (int64_t s = g; s < nsweeps; s += stride) {
        prog[s] = 0;
        bar[s] = 0;
    }
    const int64_t total = ldw * n;
    for (int64_t x = g; x < total; x += stride) {
        const int64_t j = x / ldw;
        const int64_t i = j + (x - j * ldw) - (2 * nb - 1);
        W[x] = (i >= 0 && i <= j && j - i <= nb) ? B[i * rs + j * cs] : 0.0;
    }
}

__global__ void extract_kernel(const double* W, int64_t ldw, int64_t n, int nb, double* d, double* e) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    d[i] = W[(2 * nb - 1) + i * ldw];
    if (i + 1 < n) e[i] = W[(2 * nb - 2) + (i + 1) * ldw];
}

// Number of singular values of (d, e) below x > 0: the negative pivots of
// T_GK - x I, less the n eigenvalues -sigma_i that are always below x.
__device__ __forceinline__ int64_t sturm_below(const double* d, const double* e, int64_t n, double x,
                                               double pivmin) {
    double q = -x;                   // the first pivot
    if (fabs(q) < pivmin) q = -pivmin;
    int64_t cnt = 1;
    for (int64_t i = 0; i < n; ++i) {
        const double di = d[i];
        q = -x - (di * di) / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
        if (i + 1 < n) {
            const double ei = e[i];
            q = -x - (ei * ei) / q;
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += q < 0.0;
        }
    }
    return cnt - n;
}

// MS lanes per singular value (multisection): each round, lane l counts
// below x_l = lo + (l+1)(hi-lo)/(MS+1), and the interval shrinks to the
// one between the largest x with at most s values below it and the
// smallest x with more, a factor MS+1 a round (13 rounds to full precision
// at MS = 16, against 53 for bisection), with MS times the lanes.  The host
// picks MS so that about MS_LANES lanes run (measured: n = 16384 76 ms at
// MS = 8, 92 ms at 4 and 16; n = 4096 13 ms at 16 or 32, 23 ms at 4).
constexpr int MS_LANES = 1 << 17;

template <int MS>
__global__ void bisect_kernel(const double* d, const double* e, int64_t n, double* sigma) {
    static_assert(64 % MS == 0, "a value's lanes lie in one wave");
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = gt / MS;
    const int lane = (int)(gt % MS);
    if (j >= n) return;                 // whole groups leave together (n MS threads are a multiple of MS)
    // Gershgorin bound of T_GK and the pivot floor
    double amax = 0.0, bound = 0.0, prev = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double di = fabs(d[i]);
        const double ei = i + 1 < n ? fabs(e[i]) : 0.0;
        bound = fmax(bound, fmax(prev + di, di + ei));
        amax = fmax(amax, fmax(di, ei));
        prev = ei;
    }
    const double pivmin = DBL_MIN * fmax(1.0, amax * amax);
    const int64_t s = n - 1 - j;     // sigma[j] is the s-th smallest (decreasing order)
    double lo = 0.0, hi = bound * (1.0 + 4.0 * DBL_EPSILON) + pivmin;
    const double abstol = DBL_EPSILON * bound;
    for (int it = 0; it < 128; ++it) {
        if (hi - lo <= fmax(abstol, 2.0 * DBL_EPSILON * hi)) break;
        const double x = lo + (hi - lo) * (double)(lane + 1) / (double)(MS + 1);
        const bool inside = x > lo && x < hi;
        const bool below = inside && sturm_below(d, e, n, x, pivmin) <= s;   // x <= sigma_j
        double nlo = below ? x : lo;
        double nhi = inside && !below ? x : hi;
#pragma unroll
        for (int o = 1; o < MS; o *= 2) {
            nlo = fmax(nlo, __shfl_xor(nlo, o, 64));
            nhi = fmin(nhi, __shfl_xor(nhi, o, 64));
        }
        if (nlo >= nhi || (nlo == lo && nhi == hi)) break;   // counts out of order, or no progress
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) sigma[j] = 0.5 * (lo + hi);
}

// workspace: control words (256 B), the band array (3 nb n doubles), the
// progress counters and the group barrier counters (one int32 per sweep each)
inline int64_t ws_prog_off(int64_t n, int nb) { return 256 + (int64_t)3 * nb * n * 8; }

inline int nsweeps_of(int64_t n, int nb) { return nb <= 1 || n <= 2 ? 0 : (int)(n - 2); }

inline size_t ws_bytes(int64_t n, int nb) {
    return (size_t)(ws_prog_off(n, nb) + 2 * (((int64_t)nsweeps_of(n, nb) * 4 + 255) / 256 * 256));
}

int device_attr(hipDeviceAttribute_t attr, int fallback) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, attr, dev) != hipSuccess) return fallback;
    return v;
}

}  // namespace bbg

extern "C" {

int bb_bnd2bd_workspace(int64_t n, int nb, size_t* ws_bytes) {
    if (n < 0) return -1;
    if (nb < 1 || nb > bbg::MAX_NB) return -2;
    if (!ws_bytes) return -3;
    *ws_bytes = bbg::ws_bytes(n, nb);
    return BB_OK;
}

}  // extern "C"

namespace bbg {

// The chase after argument checks: band entry (i, j) at B[i rs + j cs].
int bnd2bd_launch(const double* B, int64_t rs, int64_t cs, int64_t n, int nb, double* d, double* e, void* ws,
                  double watchdog_s, int group, bool keep_error, void* stream);

}  // namespace bbg

extern "C" {

int bb_bnd2bd_group(const double* B, int64_t ldb, int64_t n, int nb, double* d, double* e, void* ws,
                    size_t ws_bytes, double watchdog_s, int group, void* stream) {
    if (group < 0 || group > bbg::GROUP_MAX) return -10;
    if (n < 0) return -3;
    if (!B && n > 0) return -1;
    if (ldb < (n > 1 ? n : 1)) return -2;
    if (nb < 1 || nb > bbg::MAX_NB) return -4;
    if (!d && n > 0) return -5;
    if (!e && n > 1) return -6;
    if (!ws && n > 0) return -7;
    if (ws_bytes < bbg::ws_bytes(n, nb)) return BB_EWORKSPACE;
    if (n == 0) return BB_OK;
    return bbg::bnd2bd_launch(B, 1, ldb, n, nb, d, e, ws, watchdog_s, group, false, stream);
}

}  // extern "C"

int bbg::bnd2bd_launch(const double* B, int64_t rs, int64_t cs, int64_t n, int nb, double* d, double* e,
                       void* ws, double watchdog_s, int group, bool keep_error, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const int nsw = bbg::nsweeps_of(n, nb);
    bbg::ChaseArgs a;
    a.W = (double*)((char*)ws + 256);
    a.ldw = 3 * (int64_t)nb;
    a.n = n;
    a.nb = nb;
    a.nsweeps = nsw;
    a.ctrl = (int32_t*)ws;
    a.prog = (int32_t*)((char*)ws + bbg::ws_prog_off(n, nb));
    a.bar = a.prog + ((int64_t)nsw * 4 + 255) / 256 * 64;
    const double khz = (double)bbg::device_attr(hipDeviceAttributeWallClockRate, 100000);
    a.watchdog_ticks = (int64_t)((watchdog_s > 0 ? watchdog_s : 30.0) * khz * 1000.0);
    const int cus = bbg::device_attr(hipDeviceAttributeMultiprocessorCount, 256);
    const int64_t total = a.ldw * n;
    int blocks = (int)std::min<int64_t>((total + 255) / 256, 8 * (int64_t)cus);
    hipLaunchKernelGGL(bbg::pack_kernel, dim3(blocks < 1 ? 1 : blocks), dim3(256), 0, s, B, rs, cs, n, nb, a.W,
                       a.ldw, a.ctrl, a.prog, a.bar, nsw, keep_error ? 1 : 0);
    if (hipGetLastError() != hipSuccess) return BB_EHIP;
    // nb > GROUP_NB: a group of ceil(nb / 16) workgroups a sweep, so that a
    // member takes about 32 rows of the right update and one 32-column chunk
    // of the left one (measured at n = 16384: nb = 256 1.35 s with 16
    // workgroups a sweep, 1.60 s with 8, 2.64 s with 4; nb = 128 1.01 s with
    // 8, 1.06 s with 4, 1.58 s with 12); the grid holds whole groups, at
    // least one
    a.group = 1;
    if (nb > bbg::GROUP_NB) {
        a.group = std::min(std::min((nb + 15) / 16, bbg::GROUP_MAX), cus);
        if (group > 0) a.group = std::min(group, cus);
    }
    if (nsw > 0) {
        const int grid = nb <= bbg::LDS_NB ? std::min(nsw, cus)
                                           : (int)std::min<int64_t>((int64_t)nsw * a.group, cus / a.group * a.group);
        if (nb <= bbg::LDS_NB)
            hipLaunchKernelGGL(bbg::chase_kernel<true>, dim3(grid), dim3(bbg::NT), 0, s, a);
        else
            hipLaunchKernelGGL(bbg::chase_kernel<false>, dim3(grid), dim3(bbg::NT), 0, s, a);
        if (hipGetLastError() != hipSuccess) return BB_EHIP;
    }
    hipLaunchKernelGGL(bbg::extract_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a.W, a.ldw, n,
                       nb, d, e);
    return hipGetLastError() == hipSuccess ? BB_OK : BB_EHIP;
}

extern "C" {

int bb_bnd2bd(const double* B, int64_t ldb, int64_t n, int nb, double* d, double* e, void* ws,
              size_t ws_bytes, double watchdog_s, void* stream) {
    return bb_bnd2bd_group(B, ldb, n, nb, d, e, ws, ws_bytes, watchdog_s, 0, stream);
}

int bb_bd2val(const double* d, const double* e, int64_t n, double* sigma, void* stream) {
    if (n < 0) return -3;
    if (!d && n > 0) return -1;
    if (!e && n > 1) return -2;
    if (!sigma && n > 0) return -4;
    if (n == 0) return BB_OK;
    int ms = 4;
    while (ms < 32 && n * ms < bbg::MS_LANES) ms *= 2;
    const dim3 grid((unsigned)((n * ms + 255) / 256));
    hipStream_t s = (hipStream_t)stream;
    switch (ms) {
        case 4: hipLaunchKernelGGL(bbg::bisect_kernel<4>, grid, dim3(256), 0, s, d, e, n, sigma); break;
        case 8: hipLaunchKernelGGL(bbg::bisect_kernel<8>, grid, dim3(256), 0, s, d, e, n, sigma); break;
        case 16: hipLaunchKernelGGL(bbg::bisect_kernel<16>, grid, dim3(256), 0, s, d, e, n, sigma); break;
        default: hipLaunchKernelGGL(bbg::bisect_kernel<32>, grid, dim3(256), 0, s, d, e, n, sigma); break;
    }
    return hipGetLastError() == hipSuccess ? BB_OK : BB_EHIP;
}

// bb_ge2val's workspace: the band reduction's, and after it (stream order)
// the chase's with the bidiagonal (d, e) behind it.
static int ge2val_sizes(int64_t m, int64_t n, int nb, int tree, int variant, int prec, const bb_opts* opts,
                        size_t* vt_bytes, size_t* ws_bytes, size_t* de_off) {
    size_t vt = 0, wsb = 0;
    const int rc = bb_query(m, n, nb, tree, variant, prec, opts, &vt, &wsb);
    if (rc != BB_OK) return rc;
    const int64_t k = m < n ? m : n;
    const size_t chase = bbg::ws_bytes(k, nb);
    const size_t off = (chase + 255) / 256 * 256;
    const size_t need = off + (size_t)(2 * (k > 0 ? k : 1)) * sizeof(double);
    if (vt_bytes) *vt_bytes = vt;
    if (ws_bytes) *ws_bytes = wsb > need ? wsb : need;
    if (de_off) *de_off = off;
    return BB_OK;
}

int bb_ge2val_workspace(int64_t m, int64_t n, int nb, int tree, int variant, int prec, const bb_opts* opts,
                        size_t* vt_bytes, size_t* ws_bytes) {
    if (!vt_bytes || !ws_bytes) return -8;
    return ge2val_sizes(m, n, nb, tree, variant, prec, opts, vt_bytes, ws_bytes, nullptr);
}

int bb_ge2val(void* A, int64_t m, int64_t n, int64_t lda, int nb, int tree, int variant, int prec, double* sigma,
              void* vt, size_t vt_bytes, void* ws, size_t ws_bytes, const bb_opts* opts, void* stream) {
    size_t need_vt = 0, need_ws = 0, de_off = 0;
    int rc = ge2val_sizes(m, n, nb, tree, variant, prec, opts, &need_vt, &need_ws, &de_off);
    if (rc != BB_OK) return rc;
    const int64_t k = m < n ? m : n;
    if (!sigma && k > 0) return -9;
    if (vt_bytes < need_vt || ws_bytes < need_ws) return BB_EWORKSPACE;
    rc = bidiag_band(A, m, n, lda, nb, tree, variant, prec, vt, vt_bytes, ws, ws_bytes, opts, stream);
    if (rc != BB_OK || k == 0) return rc;
    double* d = (double*)((char*)ws + de_off);
    double* e = d + k;
    // m >= n: upper band in the leading n x n part; m < n: lower band in the
    // leading m x m part, chased as its transpose
    const double* B = (const double*)A;
    rc = m >= n ? bbg::bnd2bd_launch(B, 1, lda, k, nb, d, e, ws, opts ? opts->watchdog_s : 0.0, 0, true, stream)
                : bbg::bnd2bd_launch(B, lda, 1, k, nb, d, e, ws, opts ? opts->watchdog_s : 0.0, 0, true, stream);
    if (rc != BB_OK) return rc;
    return bb_bd2val(d, e, k, sigma, stream);
}

}  // extern "C"
