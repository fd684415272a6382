// Operation list of the band-form adjoint (see adjoint.hpp).
//
// Forward sweep being transposed (blocks of nb, B_ij the blocks of the band
// form, om/ps the blocks of Omega/Psi, Z temporaries):
//   column step k:  Omega_ik = (C_ik - Omega_i,k-1 B_k-1,k + B_ii Psi_ik
//                              + B_i,i+1 Psi_i+1,k) B_kk^-1          (i > k)
//                   Omega_kk = L - L^T, L = strict lower part of Z_k B_kk^-1,
//                   dB_kk = upper part of (Z_k - Omega_kk B_kk);
//   row step k:     Psi_k+1,j = -B_k,k+1^-1 (C_kj - Omega_k,j-1 B_j-1,j
//                              - Omega_kj B_jj + B_kk Psi_kj)        (j > k+1)
//                   Psi_k+1,k+1 = -(U - U^T), U = strict upper part of
//                   B_k,k+1^-1 Z'_k, dB_k,k+1 = lower part of (Z'_k + B_k,k+1 Psi).
// Each unknown block is "stored" once (Omega_ik with i >= k, Psi_ij with
// 1 <= i <= j); a read of the mirrored block is minus its transpose.  The
// adjoint visits these steps in reverse and accumulates the bars of C (= G),
// Omega and Psi.
#include <algorithm>
#include <map>
#include <set>
#include <tuple>

#include "adjoint.hpp"

namespace bbk {

namespace {

struct Builder {
    int64_t n;
    int nb, q;
    std::vector<AOp> ops;
    int sz(int i) const { return (int)std::min<int64_t>(nb, n - (int64_t)i * nb); }
    AView v(int32_t buf, int64_t r0, int64_t c0, int32_t trans = 0) const { return AView{buf, trans, r0, c0}; }
    AView blk(int32_t buf, int i, int j, int32_t trans = 0) const {
        return AView{buf, trans, (int64_t)i * nb, (int64_t)j * nb};
    }
    static AView T(AView x) { x.trans ^= 1; return x; }

    void gemm(AView D, double alpha, AView X, AView Y, int M, int N, int K, double beta = 1.0) {
        AOp o{};
        o.kind = AOP_GEMM; o.M = M; o.N = N; o.K = K;
        o.X = X; o.Y = Y; o.D = D; o.alpha = alpha; o.beta = beta;
        ops.push_back(o);
    }
    void trsm(AView D, AView X, int upper, int M, int N) {
        AOp o{};
        o.kind = AOP_TRSM; o.flag = upper; o.M = M; o.N = N; o.K = M;
        o.X = X; o.Y = X; o.D = D; o.alpha = 1.0;
        ops.push_back(o);
    }
    void ew(AView D, int mask, double a, AView X, double b2, int M, int N, double beta) {
        AOp o{};
        o.kind = AOP_EW; o.flag = mask; o.M = M; o.N = N; o.K = 0;
        o.X = X; o.Y = X; o.D = D; o.alpha = a; o.beta = beta; o.b2 = b2;
        ops.push_back(o);
    }
    // bar(Omega_ij) += alpha X Y  (X: M x K, Y: K x N)
    void ombar(int i, int j, double alpha, AView X, AView Y, int M, int N, int K) {
        if (i >= j) gemm(blk(AB_OM, i, j), alpha, X, Y, M, N, K);
        else gemm(blk(AB_OM, j, i), -alpha, T(Y), T(X), N, M, K);
    }
    void psbar(int i, int j, double alpha, AView X, AView Y, int M, int N, int K) {
        if (i == 0 || j == 0) return;          // Psi is zero there (constant)
        if (i <= j) gemm(blk(AB_PS, i, j), alpha, X, Y, M, N, K);
        else gemm(blk(AB_PS, j, i), -alpha, T(Y), T(X), N, M, K);
    }
};

// Blocks (buffer, r0, c0) an operation reads and writes, for staging.
typedef std::tuple<int32_t, int64_t, int64_t> Key;
Key key(const AView& x) { return Key(x.buf, x.r0, x.c0); }

}  // namespace

void build_adjoint_ops(int64_t m, int64_t n, int nb, AdjointOps& out) {
    Builder b;
    b.n = n;
    b.nb = nb;
    b.q = (int)((n + nb - 1) / nb);
    const int q = b.q;
    const int64_t NB = nb;
    // TMP layout (npad x 3nb): column block 0 holds Z per block row, blocks 1
    // and 2 two nb x nb scratch matrices.
    const AView T1 = b.v(AB_TMP, 0, NB), T2 = b.v(AB_TMP, 0, 2 * NB);
    auto Z = [&](int i) { return b.v(AB_TMP, (int64_t)i * nb, 0); };
    auto Bv = [&](int i, int j) { return b.blk(AB_B, i, j); };
    const int64_t npad = (int64_t)q * nb;

    // Inverses of the triangular blocks, once: INV block row k holds
    // B_kk^-1 (upper) in columns [0, nb) and, for k < q-1, the inverse of the
    // leading r x r (lower) part of B_k,k+1 in columns [nb, 2nb).  Every
    // triangular solve of the sweep is then a block product.
    auto Ikk = [&](int k) { return b.v(AB_INV, (int64_t)k * nb, 0); };
    auto I1 = [&](int k) { return b.v(AB_INV, (int64_t)k * nb, NB); };
    for (int k = 0; k < q; ++k) {
        b.ew(Ikk(k), AM_IDENT, 0.0, Ikk(k), 0.0, b.sz(k), b.sz(k), 0.0);
        if (k + 1 < q) b.ew(I1(k), AM_IDENT, 0.0, I1(k), 0.0, b.sz(k + 1), b.sz(k + 1), 0.0);
    }
    for (int k = 0; k < q; ++k) {
        b.trsm(Ikk(k), Bv(k, k), 1, b.sz(k), b.sz(k));
        if (k + 1 < q) b.trsm(I1(k), Bv(k, k + 1), 0, b.sz(k + 1), b.sz(k + 1));
    }

    // bars start at zero
    b.ew(b.v(AB_G, 0, 0), AM_ALL, 0.0, b.v(AB_G, 0, 0), 0.0, (int)n, (int)n, 0.0);
    b.ew(b.v(AB_OM, 0, 0), AM_ALL, 0.0, b.v(AB_OM, 0, 0), 0.0, (int)npad, (int)npad, 0.0);
    b.ew(b.v(AB_PS, 0, 0), AM_ALL, 0.0, b.v(AB_PS, 0, 0), 0.0, (int)npad, (int)npad, 0.0);

    for (int k = q - 1; k >= 0; --k) {
        const int nk = b.sz(k);
        if (k + 1 < q) {
            // ---- row step k, diagonal block (k, k+1) ----
            const int nk1 = b.sz(k + 1), r = nk1;
            b.ew(Z(k), AM_LOWER, 1.0, b.blk(AB_W, k, k + 1), 0.0, nk, nk1, 0.0);     // Xbar
            b.ew(T1, AM_ALL, 1.0, b.blk(AB_PS, k + 1, k + 1), 0.0, nk1, nk1, 0.0);
            b.gemm(T1, 1.0, Builder::T(Bv(k, k + 1)), Z(k), nk1, nk1, nk);           // Pdbar
            b.ew(T2, AM_SUPPER, -1.0, T1, 1.0, nk1, nk1, 0.0);                         // Ybar
            b.gemm(Z(k), 1.0, Builder::T(I1(k)), T2, r, r, r);                        // += B1[:r,:r]^-T Ybar
            b.ew(b.blk(AB_G, k, k + 1), AM_ALL, 1.0, Z(k), 0.0, nk, nk1, 1.0);
            b.ombar(k, k, -1.0, Z(k), Builder::T(Bv(k, k + 1)), nk, nk, nk1);
            b.ombar(k, k + 1, -1.0, Z(k), Builder::T(Bv(k + 1, k + 1)), nk, nk1, nk1);
            b.psbar(k, k + 1, 1.0, Builder::T(Bv(k, k)), Z(k), nk, nk1, nk);
            // ---- row step k, blocks (k, j), j > k+1 (block k+1 is full) ----
            for (int j = k + 2; j < q; ++j) {
                const int nj = b.sz(j);
                b.gemm(Z(j), -1.0, Builder::T(I1(k)), b.blk(AB_PS, k + 1, j), nb, nj, nb, 0.0);
                b.ew(b.blk(AB_G, k, j), AM_ALL, 1.0, Z(j), 0.0, nk, nj, 1.0);
                b.ombar(k, j - 1, -1.0, Z(j), Builder::T(Bv(j - 1, j)), nk, b.sz(j - 1), nj);
                b.ombar(k, j, -1.0, Z(j), Builder::T(Bv(j, j)), nk, nj, nj);
                b.psbar(k, j, 1.0, Builder::T(Bv(k, k)), Z(j), nk, nj, nk);
            }
        }
        // ---- column step k, diagonal block ----
        b.ew(Z(k), AM_UPPER, 1.0, b.blk(AB_W, k, k), 0.0, nk, nk, 0.0);               // Xbar
        b.ew(T1, AM_ALL, 1.0, b.blk(AB_OM, k, k), 0.0, nk, nk, 0.0);
        b.gemm(T1, -1.0, Z(k), Builder::T(Bv(k, k)), nk, nk, nk);                      // Okbar
        b.ew(T2, AM_SLOWER, 1.0, T1, -1.0, nk, nk, 0.0);                               // Ybar
        b.gemm(Z(k), 1.0, T2, Builder::T(Ikk(k)), nk, nk, nk);                        // += Ybar B_kk^-T
        b.ew(b.blk(AB_G, k, k), AM_ALL, 1.0, Z(k), 0.0, nk, nk, 1.0);
        if (k > 0) b.ombar(k, k - 1, -1.0, Z(k), Builder::T(Bv(k - 1, k)), nk, b.sz(k - 1), nk);
        b.psbar(k, k, 1.0, Builder::T(Bv(k, k)), Z(k), nk, nk, nk);
        if (k + 1 < q) b.psbar(k + 1, k, 1.0, Builder::T(Bv(k, k + 1)), Z(k), b.sz(k + 1), nk, nk);
        // ---- column step k, blocks (i, k), i > k ----
        for (int i = k + 1; i < q; ++i) {
            const int ni = b.sz(i);
            b.gemm(Z(i), 1.0, b.blk(AB_OM, i, k), Builder::T(Ikk(k)), ni, nk, nk, 0.0);  // Ombar B_kk^-T
            b.ew(b.blk(AB_G, i, k), AM_ALL, 1.0, Z(i), 0.0, ni, nk, 1.0);
            if (k > 0) b.ombar(i, k - 1, -1.0, Z(i), Builder::T(Bv(k - 1, k)), ni, b.sz(k - 1), nk);
            b.psbar(i, k, 1.0, Builder::T(Bv(i, i)), Z(i), ni, nk, ni);
            if (i + 1 < q) b.psbar(i + 1, k, 1.0, Builder::T(Bv(i, i + 1)), Z(i), b.sz(i + 1), nk, ni);
        }
    }

    // G^T for the application of P, then (P G^T)^T on top of Abar.
    b.ew(b.v(AB_GT, 0, 0), AM_ALL, 1.0, b.v(AB_G, 0, 0, 1), 0.0, (int)n, (int)n, 0.0);
    const size_t n_sweep = b.ops.size();
    b.ew(b.v(AB_ABAR, 0, 0), AM_ALL, 1.0, b.v(AB_GT, 0, 0, 1), 0.0, (int)n, (int)n, 0.0);
    if (m > n) b.ew(b.v(AB_ABAR, n, 0), AM_ALL, 0.0, b.v(AB_ABAR, n, 0), 0.0, (int)(m - n), (int)n, 0.0);

    // Stages: consecutive operations of one kind whose blocks do not
    // conflict (no block written by one and read or written by another).
    out.m = m;
    out.n = n;
    out.nb = nb;
    out.npad = npad;
    out.ops.clear();
    out.stage_off.assign(1, 0);
    std::set<Key> rd, wr;
    int32_t kind = -1;
    bool prev_big = false;
    for (size_t oi = 0; oi < b.ops.size(); ++oi) {
        const AOp& o = b.ops[oi];
        if (oi == n_sweep) {
            // the application of P runs between these two parts
            out.stage_off.push_back((int32_t)out.ops.size());
            out.finish_stage = (int32_t)out.stage_off.size() - 1;
            rd.clear();
            wr.clear();
            kind = o.kind;
            out.ops.push_back(o);
            prev_big = true;
            continue;
        }
        std::set<Key> r;
        if (o.kind == AOP_GEMM) { r.insert(key(o.X)); r.insert(key(o.Y)); if (o.beta != 0.0) r.insert(key(o.D)); }
        if (o.kind == AOP_TRSM) { r.insert(key(o.X)); r.insert(key(o.D)); }
        if (o.kind == AOP_EW) { r.insert(key(o.X)); if (o.beta != 0.0) r.insert(key(o.D)); }
        const Key w = key(o.D);
        bool conflict = o.kind != kind || wr.count(w) || rd.count(w);
        for (const Key& x : r) conflict = conflict || wr.count(x);
        // whole-buffer clears run alone in their stage
        const bool big = o.M > nb || o.N > nb;
        conflict = conflict || big || prev_big;
        prev_big = big;
        if (conflict && !out.ops.empty()) {
            out.stage_off.push_back((int32_t)out.ops.size());
            rd.clear();
            wr.clear();
        }
        kind = o.kind;
        out.ops.push_back(o);
        rd.insert(r.begin(), r.end());
        wr.insert(w);
    }
    out.stage_off.push_back((int32_t)out.ops.size());
    const size_t ns = out.stage_off.size() - 1;
    out.stage_m.assign(ns, 0);
    out.stage_n.assign(ns, 0);
    for (size_t st = 0; st < ns; ++st)
        for (int32_t o = out.stage_off[st]; o < out.stage_off[st + 1]; ++o) {
            out.stage_m[st] = std::max(out.stage_m[st], out.ops[o].M);
            out.stage_n[st] = std::max(out.stage_n[st], out.ops[o].N);
        }
}

}  // namespace bbk
