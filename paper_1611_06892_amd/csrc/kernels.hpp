// Interface between the host driver (api.cpp) and the gfx950 kernels
// (kernels.hip).  Plain structs passed by value to the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace bbk {

// One task of the graph as the device reads it (physical tile coordinates of
// matrix `mat` of the launch; slot: the record index within that matrix's
// records).  Bit 0 of trans is the transpose flag; in a launch that mixes
// tile sizes, trans >> 1 is the task's tile-size code (32 << code).
struct DevTask {
    int32_t kind, trans, r1, c1, r2, c2, slot, mat;
};

// One matrix of a launch: column-major, m x n, leading dimension lda; rec is
// the start of its V/T records (record k at rec + k * record_doubles(nb)).
struct MatDesc {
    double* A;
    int64_t lda, m, n;
    double* rec;
};

// Scheduler control words at the start of the workspace: error flag,
// completed-unit count and the ticket counter, each in its own 64-byte line.
enum : int { CTRL_ERROR = 1, CTRL_DONE = 16, CTRL_HEAD = 32, CTRL_WORDS = 64 };

struct KArgs {
    MatDesc single;          // the matrix of a single-matrix launch (mats == NULL)
    const MatDesc* mats;     // batched launch: the matrices' descriptors (in the workspace)
    const DevTask* tasks;
    const int2* units;       // levels: (task, part) by level; persistent: (task, part) by priority
    int32_t nunits;
    const int32_t* succ_off; // CSR successors
    const int32_t* succ_idx;
    int32_t* deps;           // live dependency counters (persistent mode)
    int32_t* ctrl;           // CTRL_* words
    int64_t watchdog_ticks;  // wall-clock ticks without progress before giving up
    int64_t* trace;          // NULL, or 4 int64 per unit (persistent mode):
                             // {ready-wait start, run start, run end, workgroup}
    double* pscratch;        // nb = 256: panel scratch, panel_scratch_doubles(nb) per slot;
                             // slot = workgroup (persistent) or block of the level launch
};

// Update strip width (columns of the logical C tile per work unit): one
// 16-column slice per wave of the 512-thread workgroup, so the whole tile up
// to nb = 128 and a 128-column half at nb = 256.
inline int strip_width(int nb) { return nb < 128 ? nb : 128; }

// Scratch of one nb = 256 panel: the trailing column tiles (nb x 16 each)
// between blocks, in the order the workgroup's lanes hold them.
__host__ __device__ inline int64_t panel_scratch_doubles(int nb) { return nb == 256 ? 16LL * nb * 16 : 0; }

// One V/T record: V (nb x nb) and nb/16 blocks T_b^T (16 x 16).
inline int64_t record_doubles(int nb) { return 1LL * nb * nb + 16LL * nb; }

// Launchers (return hipSuccess or the launch error).
// Resets the scheduler words and the dependency counters.
hipError_t launch_init(const KArgs& a, const int32_t* ndeps_init, int32_t ntasks, hipStream_t s);
// Fills mats[i] = {A[gidx[i]], lda[gidx[i]], dims[2i], dims[2i+1], ...} for
// the nmats matrices of one group of a batched launch (A, lda: the caller's
// device arrays; gidx, dims, recoff: the plan's device copy),
// and rec = vt + recoff[i] (doubles) for the group's records at vt.
hipError_t launch_batch_desc(MatDesc* mats, int32_t nmats, const int64_t* gidx, const int64_t* dims,
                             const int64_t* recoff, double* const* A, const int64_t* lda, double* vt,
                             hipStream_t s);
// prec: 0 = FP64, 2 = FP32-MFMA updates, 3 = split-FP32 updates (bidiag.h's
// BB_F64*) for reductions; PREC_APPLY for the application graphs of Q and P.
// nb = NB_MIXED: one launch whose tasks carry their own tile size (32, 64 or
// 128, in DevTask::trans).
constexpr int PREC_APPLY = 1;
constexpr int NB_MIXED = 0;
hipError_t launch_level(int nb, int prec, const KArgs& a, int32_t unit_base, int32_t count, hipStream_t s);
hipError_t launch_persistent(int nb, int prec, const KArgs& a, int32_t workgroups, hipStream_t s);
// The same for one (tile size, arithmetic) pair (each pair's kernels are
// built in their own translation unit).
template <int NB, int PREC>
hipError_t launch_level_np(const KArgs& a, int32_t unit_base, int32_t count, hipStream_t s);
template <int NB, int PREC>
hipError_t launch_persistent_np(const KArgs& a, int32_t workgroups, hipStream_t s);
bool nb_supported(int nb);

// Workspace for callers that cannot allocate: the current device's copy of a
// file-scope device array of *bytes bytes (looked up once per device).
hipError_t noalloc_scratch(void** ptr, size_t* bytes);

}  // namespace bbk
