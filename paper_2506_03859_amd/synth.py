"""Seeded synthetic input matrices shaped like the paper's experiments.

This module only builds test inputs A; it holds none of the low-rank method's
arithmetic, and both the HIP path's tests and the CPU oracle's tests take their
inputs from here.

Constructions (all seeded, numpy PCG64 unless stated):

* ``spectral(m, n, sigma, seed)``: A = U diag(sigma) V^T with U (m x k) and
  V (n x k) Haar-distributed orthonormal factors, obtained by QR of standard
  Gaussian matrices with the sign of diag(R) forced positive (Section 5: the
  factors are orthonormalised Gaussian matrices).
* ``matrix1`` / ``matrix2``: the paper's square test matrices of Section 5,
  sigma_j = j^-2 (slow decay) and sigma_j = exp(-j/20) (fast decay).
* ``exp_floor_spectrum``: sigma_i = exp(-i/50) + 1e-6 (additive floor).
* ``tall_lowrank``: L diag(1/i) R + N with Gaussian L (m x r), R (r x n) and
  i.i.d. N(0, var) noise, the tall fixed-rank workload.
* ``spectral_blockdiag_v``: A = U diag(sigma) V^T with U Haar and V block
  diagonal, d Haar blocks of size n/d (Section 5.5: the right singular
  vectors are sparse when d is large; V is diagonal, +-1, for d = n).
* ``integer_matrix``: small-integer-valued matrices, for which any ordering
  of a short FP32 sum is exact.
* ``bf16_bits`` / ``bf16_value``: BF16 storage of an FP32 matrix (round to
  nearest even) for the precision form, and the exact values it holds.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(int(seed)))


def haar_columns(rows: int, cols: int, rng: np.random.Generator) -> np.ndarray:
    """rows x cols matrix with orthonormal columns, Haar distributed (rows >= cols)."""
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def spectral(m: int, n: int, sigma: np.ndarray, seed: int) -> np.ndarray:
    """A = U diag(sigma) V^T in float64, U, V Haar, len(sigma) <= min(m, n)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    k = sigma.shape[0]
    assert k <= min(m, n)
    rng = _rng(seed)
    u = haar_columns(m, k, rng)
    v = haar_columns(n, k, rng)
    return (u * sigma[None, :]) @ v.T


def spectral_torch(m: int, n: int, sigma: np.ndarray, seed: int, device: str = "cpu"):
    """Same construction as ``spectral`` with the QR and product done by torch in
    float64 on ``device`` (for sizes where a CPU QR takes minutes). The Gaussian
    draws still come from numpy PCG64 so the input is defined by the seed; the
    result can differ from ``spectral`` in the last bits (different QR)."""
    import torch

    sigma = np.asarray(sigma, dtype=np.float64)
    k = sigma.shape[0]
    rng = _rng(seed)

    def haar_t(rows, cols):
        g = torch.from_numpy(rng.standard_normal((rows, cols))).to(device)
        q, r = torch.linalg.qr(g, mode="reduced")
        d = torch.sign(torch.diagonal(r))
        d[d == 0] = 1.0
        return q * d[None, :]

    u = haar_t(m, k)
    v = haar_t(n, k)
    s = torch.from_numpy(sigma).to(device)
    return (u * s[None, :]) @ v.T


def spectral_blockdiag_v(n: int, sigma: np.ndarray, d: int, seed: int) -> np.ndarray:
    """n x n A = U diag(sigma) V^T in float64: U Haar (n x n), V block diagonal
    with d Haar blocks of size n / d (d divides n), drawn after U from the same
    stream, block by block."""
    sigma = np.asarray(sigma, dtype=np.float64)
    assert sigma.shape[0] == n and n % d == 0
    rng = _rng(seed)
    u = haar_columns(n, n, rng)
    w = n // d
    us = u * sigma[None, :]
    a = np.empty((n, n))
    for j in range(d):
        vj = haar_columns(w, w, rng)
        a[:, j * w:(j + 1) * w] = us[:, j * w:(j + 1) * w] @ vj.T
    return a


def spectral_blockdiag_v_torch(n: int, sigma: np.ndarray, d: int, seed: int, device: str = "cpu"):
    """Same construction as ``spectral_blockdiag_v`` (same draws from the same
    stream) with the QRs and products done by torch in float64 on ``device``."""
    import torch

    sigma = np.asarray(sigma, dtype=np.float64)
    assert sigma.shape[0] == n and n % d == 0
    rng = _rng(seed)
    w = n // d

    def haar_t(g):
        q, r = torch.linalg.qr(g, mode="reduced")
        sg = torch.sign(torch.diagonal(r, dim1=-2, dim2=-1))
        sg[sg == 0] = 1.0
        return q * sg[..., None, :]

    u = haar_t(torch.from_numpy(rng.standard_normal((n, n))).to(device))
    g = np.stack([rng.standard_normal((w, w)) for _ in range(d)])
    v = haar_t(torch.from_numpy(g).to(device))                     # d x w x w
    us = u * torch.from_numpy(sigma).to(device)[None, :]
    a = torch.bmm(us.reshape(n, d, w).transpose(0, 1).contiguous(), v.transpose(1, 2).contiguous())
    return a.transpose(0, 1).reshape(n, n)


def matrix1_sigma(n: int) -> np.ndarray:
    return 1.0 / np.arange(1, n + 1, dtype=np.float64) ** 2


def matrix2_sigma(n: int) -> np.ndarray:
    return np.exp(-np.arange(1, n + 1, dtype=np.float64) / 20.0)


def exp_floor_sigma(k: int, decay: float = 50.0, floor: float = 1e-6) -> np.ndarray:
    return np.exp(-np.arange(1, k + 1, dtype=np.float64) / decay) + floor


def matrix1(n: int, seed: int) -> np.ndarray:
    """Section 5 Matrix 1: n x n, sigma_j = 1/j^2."""
    return spectral(n, n, matrix1_sigma(n), seed)


def matrix2(n: int, seed: int) -> np.ndarray:
    """Section 5 Matrix 2: n x n, sigma_j = exp(-j/20)."""
    return spectral(n, n, matrix2_sigma(n), seed)


def tall_lowrank(m: int, n: int, r: int, noise_var: float, seed: int,
                 dtype=np.float64) -> np.ndarray:
    """L diag(1/i)_{i<=r} R + N; L m x r and R r x n standard Gaussian, N i.i.d.
    N(0, noise_var). Built in float64 then cast."""
    rng = _rng(seed)
    left = rng.standard_normal((m, r))
    right = rng.standard_normal((r, n))
    scale = 1.0 / np.arange(1, r + 1, dtype=np.float64)
    a = (left * scale[None, :]) @ right
    a += np.sqrt(noise_var) * rng.standard_normal((m, n))
    return a.astype(dtype, copy=False)


def integer_matrix(m: int, n: int, seed: int, amax: int = 1024) -> np.ndarray:
    """Integer-valued entries in [-amax, amax] (float64 storage)."""
    rng = _rng(seed)
    return rng.integers(-amax, amax + 1, size=(m, n)).astype(np.float64)


def gaussian_matrix(m: int, n: int, seed: int) -> np.ndarray:
    return _rng(seed).standard_normal((m, n))


def bf16_bits(a) -> np.ndarray:
    """Storage of a finite FP32 matrix in BF16: the upper 16 bits of each value
    after round-to-nearest-even at bit 16 (uint16 bit patterns).  This is the
    input of the precision form; the matrix it represents is bf16_value(bits)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    """The FP32 values (exact) of BF16 bit patterns."""
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)
