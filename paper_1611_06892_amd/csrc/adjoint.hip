// gfx950 kernels of the band-form adjoint: batched block GEMM, triangular
// solve and masked elementwise updates on strided views (see adjoint.hpp).
// Each launch runs one stage: blockIdx.y selects the operation, blockIdx.x a
// tile of it.  These are O(n^2 nb) flops against the O(m n^2) of applying Q
// and P, so they favour simplicity (FP64 FMA through LDS) over peak speed.
#include "adjoint.hpp"

namespace bbk {

namespace {

__device__ __forceinline__ double* at(const AArgs& a, const AView& v, int r, int c) {
    const ABuf b = a.buf[v.buf];
    return v.trans ? b.p + (v.r0 + c) + (v.c0 + r) * b.ld : b.p + (v.r0 + r) + (v.c0 + c) * b.ld;
}

constexpr int TS = 32;

// D = beta D + alpha X Y, one 32 x 32 tile of D per workgroup.
__global__ __launch_bounds__(256) void adj_gemm(AArgs a, const AOp* ops, int32_t o0) {
    const AOp op = ops[o0 + blockIdx.y];
    const int tm = (op.M + TS - 1) / TS, tn = (op.N + TS - 1) / TS;
    if ((int)blockIdx.x >= tm * tn) return;
    const int bi = blockIdx.x % tm, bj = blockIdx.x / tm;
    __shared__ double Xs[TS][TS + 1], Ys[TS][TS + 1];
    const int tid = threadIdx.x, tr = tid % TS, tc = tid / TS;   // rows tr, columns tc + 8u
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < op.K; k0 += TS) {
        for (int e = tid; e < TS * TS; e += 256) {
            const int r = e % TS, c = e / TS;
            const int gr = bi * TS + r, gk = k0 + c;
            Xs[r][c] = (gr < op.M && gk < op.K) ? *at(a, op.X, gr, gk) : 0.0;
            const int gk2 = k0 + r, gc = bj * TS + c;
            Ys[r][c] = (gk2 < op.K && gc < op.N) ? *at(a, op.Y, gk2, gc) : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < TS; ++kk) {
            const double x = Xs[tr][kk];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = fma(x, Ys[kk][tc + 8 * u], acc[u]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = bi * TS + tr, c = bj * TS + tc + 8 * u;
        if (r < op.M && c < op.N) {
            double* d = at(a, op.D, r, c);
            *d = (op.beta != 0.0 ? op.beta * *d : 0.0) + op.alpha * acc[u];
        }
    }
}

// D = alpha X^-1 D, X triangular (flag: upper), 64 columns of D per
// workgroup held in LDS; column r of X is broadcast through LDS per step.
constexpr int TRSM_COLS = 64, TRSM_MAXM = 128;
__global__ __launch_bounds__(64) void adj_trsm(AArgs a, const AOp* ops, int32_t o0) {
    const AOp op = ops[o0 + blockIdx.y];
    const int c = blockIdx.x * TRSM_COLS + threadIdx.x;
    if ((int)blockIdx.x * TRSM_COLS >= op.N) return;
    __shared__ double xs[TRSM_MAXM][TRSM_COLS + 1];
    __shared__ double tc[TRSM_MAXM];
    const int M = op.M, t = threadIdx.x;
    const bool live = c < op.N;
    for (int r = 0; r < M; ++r) xs[r][t] = live ? op.alpha * *at(a, op.D, r, c) : 0.0;
    for (int s = 0; s < M; ++s) {
        const int r = op.flag ? M - 1 - s : s;        // upper: backward, lower: forward
        __syncthreads();
        for (int i = t; i < M; i += TRSM_COLS) tc[i] = *at(a, op.X, i, r);
        __syncthreads();
        const double xr = xs[r][t] / tc[r];
        xs[r][t] = xr;
        if (op.flag) {
            for (int i = 0; i < r; ++i) xs[i][t] = fma(-tc[i], xr, xs[i][t]);
        } else {
            for (int i = r + 1; i < M; ++i) xs[i][t] = fma(-tc[i], xr, xs[i][t]);
        }
    }
    if (live)
        for (int r = 0; r < M; ++r) *at(a, op.D, r, c) = xs[r][t];
}

// D = beta D + [mask] (alpha X + b2 X^T), one thread per element.
__global__ __launch_bounds__(256) void adj_ew(AArgs a, const AOp* ops, int32_t o0) {
    const AOp op = ops[o0 + blockIdx.y];
    const int64_t total = (int64_t)op.M * op.N;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int r = (int)(e % op.M), c = (int)(e / op.M);
        bool keep = true;
        switch (op.flag) {
        case AM_SUPPER: keep = r < c; break;
        case AM_SLOWER: keep = r > c; break;
        case AM_UPPER: keep = r <= c; break;
        case AM_LOWER: keep = r >= c; break;
        default: break;
        }
        double v = 0.0;
        if (op.flag == AM_IDENT) {
            v = r == c ? 1.0 : 0.0;
        } else if (keep) {
            if (op.alpha != 0.0) v += op.alpha * *at(a, op.X, r, c);
            if (op.b2 != 0.0) v += op.b2 * *at(a, op.X, c, r);
        }
        double* d = at(a, op.D, r, c);
        *d = (op.beta != 0.0 ? op.beta * *d : 0.0) + v;
    }
}

}  // namespace

hipError_t launch_adjoint_stage(const AArgs& a, const AOp* ops_dev, int32_t o0, int32_t o1, int32_t kind,
                                int32_t max_m, int32_t max_n, hipStream_t s) {
    const int nops = o1 - o0;
    if (nops <= 0) return hipSuccess;
    if (kind == AOP_GEMM) {
        const int tiles = ((max_m + TS - 1) / TS) * ((max_n + TS - 1) / TS);
        hipLaunchKernelGGL(adj_gemm, dim3(tiles, nops), dim3(256), 0, s, a, ops_dev, o0);
    } else if (kind == AOP_TRSM) {
        if (max_m > TRSM_MAXM) return hipErrorInvalidValue;
        hipLaunchKernelGGL(adj_trsm, dim3((max_n + TRSM_COLS - 1) / TRSM_COLS, nops), dim3(TRSM_COLS), 0, s,
                           a, ops_dev, o0);
    } else {
        int64_t tiles = ((int64_t)max_m * max_n + 255) / 256;
        if (tiles > 4096) tiles = 4096;
        hipLaunchKernelGGL(adj_ew, dim3((unsigned)tiles, nops), dim3(256), 0, s, a, ops_dev, o0);
    }
    return hipGetLastError();
}

}  // namespace bbk
