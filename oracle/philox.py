"""Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11), written from the published definition with numpy uint64
arithmetic.  Test infrastructure only (see oracle/__init__.py).

Definition used:
  state  : counter c = (c0, c1, c2, c3), key k = (k0, k1), 64-bit words.
  round  : (hi0, lo0) = c0 * M0,  (hi1, lo1) = c2 * M1   (full 128-bit products)
           c <- (hi1 ^ c1 ^ k0,  lo1,  hi0 ^ c3 ^ k1,  lo0)
  key    : between rounds k0 += W0, k1 += W1 (mod 2^64)
  output : the counter after 10 rounds.
  M0 = 0xD2E7470EE14C6C93, M1 = 0xCA5A826395121157,
  W0 = 0x9E3779B97F4A7C15, W1 = 0xBB67AE8584CAA73B.

Draw layout used by the test matrices (both implementations follow it):
  counter = (row r, block j, purpose, t), key = (seed, 0).
  A call yields four 64-bit words.  64-bit draw q of (r, j, purpose) is word
  q % 4 of call t = q // 4.  32-bit draw q is the low (q even) or high (q odd)
  half of 64-bit draw q // 2.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: np.uint64):
    """(hi, lo) of the 128-bit product of uint64 arrays, via 32-bit halves."""
    a = a.astype(np.uint64)
    b = np.full_like(a, b)
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = (mid << _S32) | (p00 & _LO32)
    return hi, lo


def philox4x64_10(ctr: np.ndarray, key) -> np.ndarray:
    """ctr: (N, 4) uint64, key: (k0, k1).  Returns (N, 4) uint64."""
    with np.errstate(over="ignore"):
        c = np.array(ctr, dtype=np.uint64, copy=True).reshape(-1, 4)
        k0 = np.uint64(key[0])
        k1 = np.uint64(key[1])
        for rnd in range(10):
            if rnd > 0:
                k0 = np.uint64((int(k0) + int(W0)) & 0xFFFFFFFFFFFFFFFF)
                k1 = np.uint64((int(k1) + int(W1)) & 0xFFFFFFFFFFFFFFFF)
            hi0, lo0 = _mulhilo(c[:, 0], M0)
            hi1, lo1 = _mulhilo(c[:, 2], M1)
            c = np.stack([hi1 ^ c[:, 1] ^ k0, lo1, hi0 ^ c[:, 3] ^ k1, lo0], axis=1)
        return c


def draws64(seed: int, block: int, purpose: int, rows: np.ndarray, count: int) -> np.ndarray:
    """(len(rows), count) uint64: 64-bit draws 0..count-1 of each row."""
    rows = np.asarray(rows, dtype=np.uint64).reshape(-1)
    calls = (count + 3) // 4
    out = np.empty((rows.shape[0], calls * 4), dtype=np.uint64)
    for t in range(calls):
        ctr = np.zeros((rows.shape[0], 4), dtype=np.uint64)
        ctr[:, 0] = rows
        ctr[:, 1] = np.uint64(block)
        ctr[:, 2] = np.uint64(purpose)
        ctr[:, 3] = np.uint64(t)
        out[:, 4 * t:4 * t + 4] = philox4x64_10(ctr, (np.uint64(seed), np.uint64(0)))
    return out[:, :count]


def draws32(seed: int, block: int, purpose: int, rows: np.ndarray, count: int) -> np.ndarray:
    """(len(rows), count) uint64 holding 32-bit draws 0..count-1 of each row."""
    w = draws64(seed, block, purpose, rows, (count + 1) // 2)
    out = np.empty((w.shape[0], 2 * w.shape[1]), dtype=np.uint64)
    out[:, 0::2] = w & _LO32
    out[:, 1::2] = w >> _S32
    return out[:, :count]
