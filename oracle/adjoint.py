"""Reference gradient of the band form -- TEST INFRASTRUCTURE ONLY (used by
``tests/`` alone; the GPU library never imports it and shares no code with it).

The band form B = Q^T A P (Sections 3.4 and 3.5) is unique up to B -> D1 B D2
(D1, D2 = diag(+-1), D2 = I on the first nb columns), because A P = Q B and
A^T Q = P B^T fix, block by block, each new block of Q and P by a thin QR
(block Golub-Kahan).  That recurrence, written with plain torch CPU operations
in FP64 and differentiated by torch's autograd, gives the derivative of the
sign-normalized band matrix B~(A) -- a route entirely independent of the tile
algorithm and of its adjoint.

For a loss L = sum(W * B) on a band form B = S1 B~ S2 (S1, S2 the sign
matrices that normalize B), L = sum((S1 W S2) * B~), so the reference
gradient is d/dA sum((S1 W S2) * B~(A)).

Parity status: pinned in ``tests/test_oracle.py`` against central finite
differences of the C oracle's unblocked reduction (a different algorithm).
"""
from __future__ import annotations

import numpy as np


def block_golub_kahan_torch(A, nb):
    """Sign-normalized n x n band matrix B~ of A (m x n torch FP64 tensor, m >= n)
    by the block Golub-Kahan recurrence with P's first block = I[:, :nb]:
        Q_k B_kk        = A P_k - Q_{k-1} B_{k-1,k}          (thin QR)
        P_{k+1} B_{k,k+1}^T = A^T Q_k - P_k B_kk^T            (thin QR)
    each new block reorthogonalized twice against all previous blocks, and the
    signs chosen so that diag(B_kk) >= 0 and diag(B_{k,k+1}) >= 0 (the band edge
    j = i + nb), which is the sign-normalized representative."""
    import torch
    m, n = A.shape
    blocks = [(k, min(n, k + nb)) for k in range(0, n, nb)]
    B = torch.zeros(n, n, dtype=A.dtype)
    Qs, Ps = [], []
    P0 = torch.zeros(n, blocks[0][1] - blocks[0][0], dtype=A.dtype)
    P0[: blocks[0][1], :] = torch.eye(blocks[0][1], dtype=A.dtype)
    Pk = P0
    Ps.append(Pk)
    Bprev = None

    def reorth(X, basis):
        if not basis:
            return X
        Y = torch.cat(basis, dim=1)
        for _ in range(2):
            X = X - Y @ (Y.t() @ X)
        return X

    def qr_pos(X):
        Qx, Rx = torch.linalg.qr(X)
        d = torch.sign(torch.diagonal(Rx))
        d = torch.where(d == 0, torch.ones_like(d), d)
        return Qx * d[None, :], Rx * d[:, None]

    for k, (c0, c1) in enumerate(blocks):
        X = A @ Pk
        if Bprev is not None:
            X = X - Qs[-1] @ Bprev
        X = reorth(X, Qs)
        Qk, Rk = qr_pos(X)
        Qs.append(Qk)
        Bkk = Rk
        B = B.index_put((torch.arange(c0, c1)[:, None], torch.arange(c0, c1)[None, :]), Bkk)
        if k + 1 == len(blocks):
            break
        d0, d1 = blocks[k + 1]
        Y = A.t() @ Qk - Pk @ Bkk.t()
        Y = reorth(Y, Ps)
        r = d1 - d0
        if r == Y.shape[1]:
            Pn, Rn = qr_pos(Y)          # Y = Pn Rn, B_{k,k+1} = Rn^T (lower triangular)
        else:
            # a last block narrower than nb: Y has rank r; its first r columns
            # fix P_{k+1}, and B_{k,k+1} = (P_{k+1}^T Y)^T is lower trapezoidal
            Pn, _ = qr_pos(Y[:, :r])
            Rn = Pn.t() @ Y
        Bk1 = Rn.t()
        B = B.index_put((torch.arange(c0, c1)[:, None], torch.arange(d0, d1)[None, :]), Bk1)
        Ps.append(Pn)
        Pk = Pn
        Bprev = Bk1
    return B


def sign_vectors(B, nb):
    """(s, t) with diag(s) B diag(t) sign-normalized (s_i B_ii t_i >= 0,
    s_i B_{i,i+nb} t_{i+nb} >= 0, t = 1 on the first nb columns)."""
    B = np.asarray(B)
    n = B.shape[1]
    s, t = np.ones(n), np.ones(n)
    for i in range(n):
        s[i] = 1.0 if B[i, i] * t[i] >= 0 else -1.0
        if i + nb < n:
            t[i + nb] = 1.0 if B[i, i + nb] * s[i] >= 0 else -1.0
    return s, t


def band_loss_gradient(A, W, nb, B_signs):
    """Gradient of L(A) = sum(W * B(A)[:n]) where B(A) has the sign pattern of
    B_signs (an m x n band form of A, e.g. the GPU's): A (m x n numpy), W
    (n x n, only its band entries matter).  Returns (L, dL/dA) in FP64."""
    import torch
    n = A.shape[1]
    s, t = sign_vectors(B_signs, nb)
    Wn = (s[:, None] * np.asarray(W)[:n, :n]) * t[None, :]
    At = torch.tensor(np.asarray(A, dtype=np.float64), requires_grad=True)
    Bt = block_golub_kahan_torch(At, nb)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    band = torch.tensor(((j >= i) & (j <= i + nb)).astype(np.float64))
    L = torch.sum(torch.tensor(Wn) * band * Bt)
    L.backward()
    return float(L.detach()), At.grad.numpy().copy()
