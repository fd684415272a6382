// Adjoint of the band reduction: shared definitions of the host-side
// operation list (adjoint_ops.cpp) and the gfx950 block kernels
// (adjoint.hip).
//
// With B = Q^T A P the band form, a perturbation dA moves B by
//   dB = C - Omega B + B Psi,   C = Q^T dA P,
// where Omega = Q^T dQ and Psi = P^T dP are skew (Psi zero on the first nb
// rows and columns, which P leaves untouched, Sections 3.4 and 3.5) and are
// fixed by dB keeping the band structure.  Only the top n x n part C_1 of C
// reaches the band, so for a loss L = sum(W .* B) the gradient is
//   dL/dA = Q_thin G P^T,   G = dL/dC_1 (n x n).
// G follows from W by the transpose of the block sweep that solves the band
// constraints for Omega and Psi (block column k, then block row k, k = 0..q-1);
// that transpose runs k = q-1..0 and is a sequence of nb x nb block products,
// triangular solves with the diagonal and super-diagonal blocks of B, and
// masked elementwise updates, listed here as operations on views of a few
// buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace bbk {

// Buffers the operations refer to (by index).
enum : int32_t { AB_B = 0, AB_W = 1, AB_G = 2, AB_OM = 3, AB_PS = 4, AB_TMP = 5, AB_GT = 6, AB_ABAR = 7,
                 AB_INV = 8, AB_NBUF = 9 };

// View of a buffer: element (r, c) is buf[(r0 + r) + (c0 + c) ld] when
// trans = 0 and buf[(r0 + c) + (c0 + r) ld] when trans = 1.
struct AView {
    int32_t buf, trans;
    int64_t r0, c0;
};

enum : int32_t { AOP_GEMM = 0, AOP_TRSM = 1, AOP_EW = 2 };
// Elementwise masks (r, c of the destination).
// AM_IDENT writes the identity (X is not read).
enum : int32_t { AM_ALL = 0, AM_SUPPER = 1, AM_SLOWER = 2, AM_UPPER = 3, AM_LOWER = 4, AM_IDENT = 5 };

// GEMM: D = beta D + alpha X Y (M x N, inner K); beta = 0 does not read D.
// TRSM: D = alpha X^-1 D with X M x M triangular (flag 1: upper, 0: lower),
//       D M x N, in place.
// EW:   D = beta D + [mask] (alpha X + b2 X^T), M x N (b2 != 0 needs M == N);
//       beta = 0 does not read D.
struct AOp {
    int32_t kind, flag;
    int32_t M, N, K, pad;
    AView X, Y, D;
    double alpha, beta, b2;
};

struct ABuf {
    double* p;
    int64_t ld;
};
struct AArgs {
    ABuf buf[AB_NBUF];
};

// Operation list of the adjoint sweep for an n x n band part with tile nb,
// grouped into stages: the operations of one stage are of one kind and touch
// disjoint blocks, so they run in one launch; stages run in order.
// Stages [0, finish_stage) compute G and write G^T to AB_GT; the caller then
// applies P to AB_GT; stages [finish_stage, end) write (P G^T)^T into the top
// n rows of AB_ABAR and zero its other m - n rows; the caller then applies Q.
struct AdjointOps {
    int64_t m = 0, n = 0, npad = 0;
    int nb = 0;
    std::vector<AOp> ops;
    std::vector<int32_t> stage_off;   // ops of stage s: [stage_off[s], stage_off[s+1])
    std::vector<int32_t> stage_m, stage_n;   // largest M, N of each stage
    int32_t finish_stage = 0;
};
void build_adjoint_ops(int64_t m, int64_t n, int nb, AdjointOps& out);

// Launch stage [o0, o1) of `ops` (device copy), all of kind `kind`.
hipError_t launch_adjoint_stage(const AArgs& a, const AOp* ops_dev, int32_t o0, int32_t o1, int32_t kind,
                                int32_t max_m, int32_t max_n, hipStream_t s);

}  // namespace bbk
