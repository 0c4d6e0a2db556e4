"""Random test matrices Omega_j (n x b) of the paper, materialised densely in
float64 from the counter-based draws.  Test infrastructure only.

Sketch kinds (names used across the project):
  "gaussian"        standard Gaussian G_j (farPCA, Algorithm 1).
  "std_bernoulli"   Definition 2.3: (B - p) / sqrt(p (1 - p)), B Bernoulli(p)
                    (farPCASB, Algorithm 2 works with B_j and the rank-1
                    correction instead of Omega_j itself).
  "sparse_sign"     Definition 2.2 when zeta == 0: i.i.d. entries +-1/sqrt(p)
                    with probability p/2 each, else 0.
                    zeta > 0: the fixed-count variant the paper mentions after
                    Definition 2.2 - every row of Omega_j (one column of A's
                    range) has exactly zeta nonzeros +-1/sqrt(zeta) at distinct
                    columns (farPCASS).
  "sparse_gaussian" Definition 2.4: B o G / sqrt(p) (farPCASG).
  "bernoulli"       Definition 2.1: plain 0/1 Bernoulli(p) (farPCAB, Section 5).

Draw layout (shared written contract, see philox.py for counters):
  purpose 0, 32-bit draws: mask / index draws.
     i.i.d. kinds: entry (r, c) is nonzero iff draw32(r, 0, c) < T(p),
                   T(p) = floor(p * 2^32).
     fixed-count sparse sign: Floyd's sampling of zeta distinct columns out of
                   b.  For s = 0..zeta-1 with jj = b - zeta + s:
                   t = floor(draw32(r, 0, s) * (jj + 1) / 2^32);
                   if column t is already chosen choose jj, else choose t.
  purpose 1, 64-bit draw 0: sign word w.  i.i.d. sparse sign: entry (r, c) is
                   negative iff bit c of w is set.  Fixed count: the k-th
                   chosen column in ascending order is negative iff bit k of w
                   is set.
  purpose 2, 64-bit draws 2c and 2c+1: Box-Muller for entry (r, c):
                   u1 = ((w1 >> 11) + 1) 2^-53 in (0, 1], u2 = (w2 >> 11) 2^-53,
                   g = sqrt(-2 ln u1) cos(2 pi u2).
Blocks are numbered j = 0, 1, 2, ... in the order the algorithm draws them.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import draws32, draws64

SKETCHES = ("gaussian", "std_bernoulli", "sparse_sign", "sparse_gaussian", "bernoulli")
MAX_BLOCK = 64


def threshold32(p: float) -> int:
    """Integer acceptance threshold T(p) = floor(p * 2^32) for p in (0, 1)."""
    if not (0.0 < p < 1.0):
        raise ValueError("p must lie in (0, 1)")
    return int(math.floor(p * 4294967296.0))


def default_p(sketch: str, m: int, n: int) -> float:
    """Section 5.2 / 5.4 rules: p1 = max(1e-3, ln n / n) for the standardized
    Bernoulli sketch, p2 = max(1e-3, 10 / n) for the others.  The paper's
    matrices are square; for an m x n A the n here is the number of rows of the
    n x b test matrix Omega_j, so that a column of Omega_j holds about ln n
    (p1) or 10 (p2) nonzeros whatever m is."""
    del m
    if sketch == "std_bernoulli":
        return max(1e-3, math.log(n) / n)
    return max(1e-3, 10.0 / n)


def sketch_scale(sketch: str, p: float, zeta: int) -> float:
    """Value scale of the nonzeros (Definitions 2.2-2.4)."""
    if sketch == "sparse_sign":
        return 1.0 / math.sqrt(zeta) if zeta > 0 else 1.0 / math.sqrt(p)
    if sketch == "sparse_gaussian":
        return 1.0 / math.sqrt(p)
    if sketch == "std_bernoulli":
        return 1.0 / math.sqrt(p * (1.0 - p))
    return 1.0


def bernoulli_mask(n: int, b: int, block: int, seed: int, p: float) -> np.ndarray:
    """Definition 2.1 mask B_j (n x b, bool): entry nonzero iff draw < T(p)."""
    u = draws32(seed, block, 0, np.arange(n), b)
    return u < np.uint64(threshold32(p))


def _sign_word(n: int, block: int, seed: int) -> np.ndarray:
    return draws64(seed, block, 1, np.arange(n), 1)[:, 0]


def sparse_sign_fixed_mask_signs(n: int, b: int, block: int, seed: int, zeta: int):
    """Fixed-count sparse sign pattern: (mask n x b bool, negative n x b bool)."""
    if not (1 <= zeta <= b <= MAX_BLOCK):
        raise ValueError("need 1 <= zeta <= b <= 64")
    u = draws32(seed, block, 0, np.arange(n), zeta)
    chosen = np.zeros((n, b), dtype=bool)
    rows = np.arange(n)
    for s in range(zeta):
        jj = b - zeta + s
        t = ((u[:, s] * np.uint64(jj + 1)) >> np.uint64(32)).astype(np.int64)
        already = chosen[rows, t]
        pick = np.where(already, jj, t)
        chosen[rows, pick] = True
    w = _sign_word(n, block, seed)
    negative = np.zeros((n, b), dtype=bool)
    rank = np.cumsum(chosen, axis=1) - 1          # index of this column among chosen ones
    for c in range(b):
        bit = (w >> rank[:, c].clip(0).astype(np.uint64)) & np.uint64(1)
        negative[:, c] = chosen[:, c] & (bit == 1)
    return chosen, negative


def gaussian_values(n: int, b: int, block: int, seed: int) -> np.ndarray:
    """Box-Muller standard normals for every entry (n x b, float64)."""
    w = draws64(seed, block, 2, np.arange(n), 2 * b)
    w1 = w[:, 0::2]
    w2 = w[:, 1::2]
    u1 = ((w1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (w2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def omega_dense(n: int, b: int, block: int, sketch: str, seed: int,
                p: float = 0.0, zeta: int = 0) -> np.ndarray:
    """Omega_j (n x b) in float64, exactly as the definitions state it."""
    if not (1 <= b <= MAX_BLOCK):
        raise ValueError("block size must be in [1, 64]")
    if sketch == "gaussian":
        return gaussian_values(n, b, block, seed)
    if sketch == "sparse_sign" and zeta > 0:
        chosen, negative = sparse_sign_fixed_mask_signs(n, b, block, seed, zeta)
        val = np.where(negative, -1.0, 1.0) * chosen
        return val * sketch_scale(sketch, p, zeta)
    mask = bernoulli_mask(n, b, block, seed, p)
    if sketch == "bernoulli":
        return mask.astype(np.float64)
    if sketch == "std_bernoulli":
        return (mask.astype(np.float64) - p) / math.sqrt(p * (1.0 - p))
    if sketch == "sparse_sign":
        w = _sign_word(n, block, seed)
        cols = np.arange(b, dtype=np.uint64)
        negative = ((w[:, None] >> cols[None, :]) & np.uint64(1)) == 1
        return np.where(negative, -1.0, 1.0) * mask / math.sqrt(p)
    if sketch == "sparse_gaussian":
        return mask * gaussian_values(n, b, block, seed) / math.sqrt(p)
    raise ValueError(f"unknown sketch {sketch!r}")
