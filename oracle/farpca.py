"""farPCA with the paper's test matrices, in float64 - the oracle.
Test infrastructure only (see oracle/__init__.py).

Follows Algorithm 1 (farPCA with shifted power iteration, Section 2.1) for the
Gaussian, sparse sign, sparse Gaussian and plain Bernoulli test matrices, and
Algorithm 2 (farPCASB, Section 3.1) for the standardized Bernoulli matrix,
which works with the 0/1 matrix B_j, w = p 1_n and z = A w instead of Omega_j.

Readings taken where the paper is silent or ambiguous:
* E after block j is ||A||_F^2 - tr(T Z^{-1}) with the accumulated T and Z
  (the update written as E = E - tr(T Z^{-1}) would subtract earlier blocks
  twice); this equals ||A - Q Q^T A||_F^2 for Q an orthonormal basis of Y.
* The stop test is relative: E < tol^2 ||A||_F^2, strict (Section 5.2).
* eigSVD (used, not defined, in the paper) is the Gram-eigen economy SVD:
  X^T X = V D V^T, S = D^{1/2} ascending, U = X V S^{-1}.
* The shift uses the smallest singular value of the block (the entry the
  algorithms index as Sigma_hat(b, b) when values are descending).
* Singular values are returned in descending order.
* Z^{-1} is applied with an LU solve; if Z is numerically singular the
  symmetric pseudo-inverse (eigenvalues below lambda_max * l * eps dropped)
  is used instead.
* Fixed-rank use (Section 5.1): blocks are added until l = j b >= k, then the
  top k singular triplets are kept.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .omega import bernoulli_mask, default_p, omega_dense

STATUS_OK = 0
STATUS_NOT_CONVERGED = 1


@dataclass
class FarpcaParams:
    tol: float = 0.0          # relative Frobenius tolerance (fixed precision)
    rank: int = 0             # fixed rank k (0: fixed precision)
    block: int = 0            # b (0: Section 5 rule)
    power: int = 1            # P
    sketch: str = "gaussian"
    p: float = 0.0            # Bernoulli / density parameter (0: Section 5 rule)
    zeta: int = 0             # sparse sign: nonzeros per row (0: i.i.d. Def. 2.2)
    seed: int = 0
    max_blocks: int = 0       # 0: ceil(min(m, n) / (2 b))


@dataclass
class FarpcaResult:
    U: np.ndarray
    S: np.ndarray
    V: np.ndarray
    rank: int
    blocks: int
    status: int
    norm_a2: float
    err_indicator: float
    e_history: list = field(default_factory=list)
    Y: np.ndarray | None = None
    W: np.ndarray | None = None


def default_block(m: int, n: int) -> int:
    """Section 5.2 / 5.4: b = min(max(20, floor(min(m, n) / 100)), 50)."""
    return min(max(20, min(m, n) // 100), 50)


def default_maxit(m: int, n: int, b: int) -> int:
    """Section 5.2: at most ceil(n / (2 b)) blocks, and l = j b <= min(m, n)."""
    return max(1, min(math.ceil(min(m, n) / (2 * b)), min(m, n) // b))


def eig_svd(x: np.ndarray):
    """Economy SVD of a tall matrix through the eigendecomposition of its Gram
    matrix (the eigSVD step of Algorithms 1 and 2).  Ascending order.
    Eigenvalues of the Gram at or below lambda_max * b * eps belong to
    numerically dependent columns (e.g. two equal test-matrix columns): as in
    the pseudo-inverse reading of Z^{-1}, their singular values are set to 0
    and their columns of U to zero instead of amplifying rounding noise."""
    c = x.T @ x
    d, v = np.linalg.eigh(c)
    d = np.clip(d, 0.0, None)
    keep = d > (d[-1] if d.size else 0.0) * c.shape[0] * np.finfo(np.float64).eps
    s = np.where(keep, np.sqrt(d), 0.0)
    inv = np.where(keep, 1.0 / np.where(keep, s, 1.0), 0.0)
    u = (x @ v) * inv[None, :]
    return u, s, v


def _z_solve(z: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Z^{-1} rhs (LU solve; symmetric pseudo-inverse if Z is singular)."""
    try:
        lam = np.linalg.eigvalsh(z)
        if lam[0] > lam[-1] * z.shape[0] * np.finfo(np.float64).eps:
            return np.linalg.solve(z, rhs)
    except np.linalg.LinAlgError:
        pass
    lam, vec = np.linalg.eigh(z)
    keep = lam > lam[-1] * z.shape[0] * np.finfo(np.float64).eps
    return (vec[:, keep] / lam[keep][None, :]) @ (vec[:, keep].T @ rhs)


def farpca(a: np.ndarray, params: FarpcaParams, keep_bases: bool = False,
           trace: list | None = None) -> FarpcaResult:
    """Run the method.  ``trace`` (optional list) receives one dict per power
    step with the block index, the step k, the deflated W_j and the previous Y."""
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    b = params.block or default_block(m, n)
    big_p = params.power
    sketch = params.sketch
    p = params.p or (default_p(sketch, m, n) if sketch != "gaussian" else 0.0)
    maxit = params.max_blocks or default_maxit(m, n, b)
    maxit = min(maxit, min(m, n) // b)
    if params.rank > 0:
        maxit = min(math.ceil(params.rank / b), min(m, n) // b)

    # Setup: Y = W = Z = [], E = ||A||_F^2 (Alg. 1 / Alg. 2, first step).
    norm_a2 = float(np.sum(a * a))
    thr = params.tol ** 2 * norm_a2
    y = np.zeros((m, 0))
    w_big = np.zeros((n, 0))
    z = np.zeros((0, 0))
    t = np.zeros((0, 0))
    if sketch == "std_bernoulli":
        # Alg. 2: w = p 1_n, z = A w (rank-1 correction of the sketch).
        w_vec = p * np.ones(n)
        z_vec = a @ w_vec
    e = norm_a2
    e_hist = []
    blocks = 0
    status = STATUS_NOT_CONVERGED

    for j in range(maxit):
        alpha = 0.0
        if sketch == "std_bernoulli":
            b_hat = bernoulli_mask(n, b, j, params.seed, p).astype(np.float64)
            sk = a @ b_hat - z_vec[:, None]                    # A B_j - z
            wt_om = w_big.T @ b_hat - (w_big.T @ w_vec)[:, None]  # W^T B_j - W^T w
        else:
            om = omega_dense(n, b, j, sketch, params.seed, p, params.zeta)
            sk = a @ om                                        # A Omega_j
            wt_om = w_big.T @ om                               # W^T Omega_j
        if big_p == 0:
            y_j = sk
            w_j = a.T @ y_j
        else:
            # k = 1: W_j = A^T (A Omega_j) - W (Z^{-1} (W^T Omega_j)), alpha = 0.
            w_j = a.T @ sk
            if w_big.shape[1] > 0:
                w_j = w_j - w_big @ _z_solve(z, wt_om)
            if trace is not None:
                trace.append(dict(j=j, k=1, w_j=w_j.copy(), y_prev=y.copy(), sketch=sk.copy()))
            g, _, _ = eig_svd(w_j)
            for _k in range(2, big_p + 1):
                # W_j = A^T (A G_j) - W (Z^{-1} (W^T G_j)) - alpha G_j
                g_in = g
                w_j = a.T @ (a @ g)
                if w_big.shape[1] > 0:
                    w_j = w_j - w_big @ _z_solve(z, w_big.T @ g)
                w_j = w_j - alpha * g
                if trace is not None:
                    trace.append(dict(j=j, k=_k, w_j=w_j.copy(), y_prev=y.copy(), alpha=alpha,
                                      g_in=g_in.copy()))
                g, s_hat, _ = eig_svd(w_j)
                s_small = float(s_hat[0])      # ascending: smallest first
                if alpha < s_small:
                    alpha = (s_small + alpha) / 2.0
            y_j = a @ g
            w_j = a.T @ y_j
        y = np.hstack([y, y_j])
        w_big = np.hstack([w_big, w_j])
        z = y.T @ y
        t = w_big.T @ w_big
        e = norm_a2 - float(np.trace(_z_solve(z, t)))
        e_hist.append(e)
        blocks = j + 1
        if params.rank > 0:
            if blocks * b >= params.rank:
                status = STATUS_OK
                break
        elif e < thr:
            status = STATUS_OK
            break

    # Final step: eig(Z) -> D = V_hat S_hat^{-1/2}; eig(D^T T D) -> V_tilde,
    # Sigma = S_tilde^{1/2}; U = Y D V_tilde, V = W D V_tilde Sigma^{-1}.
    lam, v_hat = np.linalg.eigh(z)
    keep = lam > lam[-1] * z.shape[0] * np.finfo(np.float64).eps
    d = v_hat[:, keep] / np.sqrt(lam[keep])[None, :]
    s_t, v_t = np.linalg.eigh(d.T @ t @ d)
    order = np.argsort(s_t)[::-1]
    s_t = np.clip(s_t[order], 0.0, None)
    v_t = v_t[:, order]
    sigma = np.sqrt(s_t)
    u = y @ (d @ v_t)
    inv = np.where(sigma > 0, 1.0 / np.where(sigma > 0, sigma, 1.0), 0.0)
    v = (w_big @ (d @ v_t)) * inv[None, :]
    if params.rank > 0:
        u, sigma, v = u[:, :params.rank], sigma[:params.rank], v[:, :params.rank]
    res = FarpcaResult(U=u, S=sigma, V=v, rank=y.shape[1], blocks=blocks, status=status,
                       norm_a2=norm_a2, err_indicator=e, e_history=e_hist)
    if keep_bases:
        res.Y, res.W = y, w_big
    return res


def projection_svd(a: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Singular values (descending) of C = Q^T A with Q an orthonormal basis of
    range(Y): the direct SVD of Section 2.1 written out plainly (LAPACK SVDs),
    without the Gram matrices Z and T.  Used as the definition the final step
    reaches for a given basis.  Q is the left singular vectors of Y whose
    squared singular values pass the dependence threshold of the pseudo-inverse
    reading of Z^{-1} (lambda > lambda_max * l * eps for the eigenvalues
    lambda = sigma^2 of Z = Y^T Y): numerically dependent columns of Y (e.g.
    two equal test-matrix columns) span no extra direction."""
    y = np.asarray(y, dtype=np.float64)
    u, sv, _ = np.linalg.svd(y, full_matrices=False)
    keep = sv * sv > sv[0] * sv[0] * y.shape[1] * np.finfo(np.float64).eps
    q = u[:, keep]
    return np.linalg.svd(q.T @ np.asarray(a, dtype=np.float64), compute_uv=False)


def truncation_rank(s: np.ndarray, err_indicator: float, norm_a2: float, tol: float) -> int:
    """Post-processing for the fixed-precision problem (Section 5.4, after
    Hallman's block method): the smallest rank r to which the computed SVD
    U S V^T can be truncated while still meeting the tolerance.  With Q the
    orthonormal basis behind U (U = Q U~), A - Q Q^T A is orthogonal to every
    matrix with columns in range(Q), so the error of the rank-r truncation is
    ||A - U_r S_r V_r^T||_F^2 = E + sum_{i >= r} s_i^2 (E the indicator,
    singular values descending).  r is the smallest r with that error below
    tol^2 ||A||_F^2, with the strict test of the stop rule (reading of the
    stop test); len(s) when even r = len(s) fails it."""
    s = np.asarray(s, dtype=np.float64)
    thr = tol * tol * norm_a2
    k = s.size
    r = k
    tail = 0.0
    for i in range(k - 1, -1, -1):   # r = i is valid iff E + sum_{j >= i} s_j^2 < thr
        tail += s[i] * s[i]
        if err_indicator + tail < thr:
            r = i
        else:
            break
    if not (err_indicator < thr):
        return k
    return r

