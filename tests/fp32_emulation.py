"""NumPy emulation of the GPU path's arithmetic (test infrastructure).

It repeats the order of operations of the HIP implementation with the same
storage precisions, on the host:
* the A-products in FP32 (NumPy float32 matrix products, FP32 accumulation);
* the power iterate deflated in the m-space, T <- (I - Q Q^T) T applied twice
  with FP32 products (the explicit orthonormal basis Q of span(Y));
* orth() as CholeskyQR in two passes: FP64 Gram of the FP32 block, FP64
  Cholesky factor (a column whose pivot falls to 1e-10 of its diagonal is
  dropped: zero), X R^-1 formed in FP64 and stored in FP32; the second pass
  is left out when the Gram is the identity to 1e-8;
* the new basis block: two projections, one CholeskyQR pass, one more
  projection, the second pass;
* the indicator E = ||A||^2 - sum_j ||C_j||_F^2 with C_j^T = A^T Q_j (FP32) and
  the sums in FP64;
* the final step as the FP64 eigendecomposition of K = C C^T, U = Q U~ and
  V = C^T U~ S^-1 in FP32.
It shares no code with the library (it is NumPy), and the test matrices come
from the oracle's generator.  Its only use is to measure how far an FP32
execution of the method lands from the FP64 oracle, which sets the tolerance of
the whole-path parity tests on the approximation itself.  No shift (P <= 2).
"""
from __future__ import annotations

import numpy as np

from oracle.farpca import default_block, default_maxit
from oracle.omega import bernoulli_mask, default_p, omega_dense

F32 = np.float32


def _project(q, t, passes=2):
    for _ in range(passes):
        if q.shape[1]:
            r = q.T @ t
            t = t - q @ r
    return t


def _project_twice(q, t):
    return _project(q, t, 2)


def _chol_drop(g, drop_rel=1e-10):
    """Upper factor R (g = R^T R on the kept columns); a column whose pivot is
    at most drop_rel times its diagonal is dropped (its row of R stays zero)."""
    b = g.shape[0]
    w = g.copy()
    r = np.zeros_like(g)
    keep = np.zeros(b, bool)
    for k in range(b):
        piv = w[k, k]
        if g[k, k] == 0.0 or piv <= drop_rel * g[k, k]:
            continue
        keep[k] = True
        rk = w[k, k:] / np.sqrt(piv)
        r[k, k:] = rk
        w[k + 1:, k + 1:] -= np.outer(rk[1:], rk[1:])
    return r, keep


def _cholqr_pass(x, repeat):
    x64 = x.astype(np.float64)
    g = x64.T @ x64
    if repeat:
        kept = np.diag(g) != 0.0
        dev = np.abs(g - np.eye(len(g)))[np.ix_(kept, kept)]
        if dev.size == 0 or dev.max() <= 1e-8:
            return x
    r, keep = _chol_drop(g)
    rinv = np.zeros_like(r)
    idx = np.where(keep)[0]
    if len(idx):
        rinv[np.ix_(idx, idx)] = np.linalg.inv(r[np.ix_(idx, idx)])
    return (x64 @ rinv).astype(F32)


def _cholqr2(x):
    return _cholqr_pass(_cholqr_pass(x, False), True)


def _orth_block(q, y):
    y = _project(q, y, 2)
    y = _cholqr_pass(y, False)
    y = _project(q, y, 1)
    return _cholqr_pass(y, True)


def farpca_fp32(a32, tol=0.0, rank=0, block=0, power=1, sketch="sparse_sign", p=0.0, zeta=0,
                seed=0, max_blocks=0):
    a32 = np.ascontiguousarray(a32, dtype=F32)
    m, n = a32.shape
    assert power <= 2
    b = block or default_block(m, n)
    p = p or (default_p(sketch, m, n) if sketch != "gaussian" else 0.0)
    maxit = max_blocks or default_maxit(m, n, b)
    maxit = min(maxit, min(m, n) // b)
    if rank > 0:
        maxit = min(-(-rank // b), min(m, n) // b)
    norm_a2 = float(np.sum(a32.astype(np.float64) ** 2))
    thr = tol * tol * norm_a2
    if sketch == "std_bernoulli":
        z = (a32.astype(np.float64) @ (p * np.ones(n))).astype(F32)
    q = np.zeros((m, 0), F32)
    ct = np.zeros((n, 0), F32)
    e = norm_a2
    blocks = 0
    status = 1
    for j in range(maxit):
        if sketch == "std_bernoulli":
            s = a32 @ bernoulli_mask(n, b, j, seed, p).astype(F32) - z[:, None]
        else:
            s = a32 @ omega_dense(n, b, j, sketch, seed, p, zeta).astype(F32)
        if power == 0:
            y = s
        else:
            t = s
            for k in range(1, power + 1):
                t = _project_twice(q, t)
                g = _cholqr2(a32.T @ t)
                if k < power:
                    t = a32 @ g
            y = a32 @ g
        qj = _orth_block(q, y)
        cj = a32.T @ qj
        q = np.hstack([q, qj])
        ct = np.hstack([ct, cj])
        e -= float(np.sum(cj.astype(np.float64) ** 2))
        blocks = j + 1
        if rank > 0:
            if blocks * b >= rank:
                status = 0
                break
        elif e < thr:
            status = 0
            break
    c64 = ct.astype(np.float64)
    lam, ut = np.linalg.eigh(c64.T @ c64)
    order = np.argsort(lam)[::-1]
    lam, ut = np.clip(lam[order], 0.0, None), ut[:, order]
    sv = np.sqrt(lam)
    u = q @ ut.astype(F32)
    inv = np.where(sv > 0, 1.0 / np.where(sv > 0, sv, 1.0), 0.0)
    v = ct @ (ut * inv[None, :]).astype(F32)
    k = rank if rank > 0 else q.shape[1]
    return dict(U=u[:, :k], S=sv[:k], V=v[:, :k], rank=q.shape[1], blocks=blocks, status=status,
                err_indicator=e, norm_a2=norm_a2)
