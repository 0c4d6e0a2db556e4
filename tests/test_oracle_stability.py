"""Section 5.5 inputs and the oracle on them (CPU): the block-diagonal
right-singular-vector matrices have the requested spectrum and structure,
and the oracle shows the section's effect - the sparser V_A (larger d), the
more blocks the sparse test matrices need at a small p."""
import math

import numpy as np
import pytest

from oracle import FarpcaParams, farpca
from paper_2506_03859_amd import synth


@pytest.mark.parametrize("d", [1, 6, 60])
def test_blockdiag_v_structure(d):
    n = 60
    sig = synth.matrix1_sigma(n)
    a = synth.spectral_blockdiag_v(n, sig, d, seed=4)
    np.testing.assert_allclose(np.linalg.svd(a, compute_uv=False), sig, rtol=0, atol=1e-14)
    # A^T A = V diag(sigma^2) V^T is block diagonal with blocks of size n / d
    w = n // d
    off = (a.T @ a) * (1.0 - np.kron(np.eye(d), np.ones((w, w))))
    assert np.abs(off).max() <= 1e-15
    if d == n:
        # V = diagonal +-1: A's columns are orthogonal with norms sigma
        np.testing.assert_allclose(np.linalg.norm(a, axis=0), sig, rtol=1e-12)


def test_blockdiag_v_torch_matches_numpy():
    torch = pytest.importorskip("torch")
    n = 40
    for d in (1, 8, 40):
        a = synth.spectral_blockdiag_v(n, synth.matrix1_sigma(n), d, seed=3)
        t = synth.spectral_blockdiag_v_torch(n, synth.matrix1_sigma(n), d, seed=3)
        assert isinstance(t, torch.Tensor)
        np.testing.assert_allclose(t.numpy(), a, rtol=0, atol=1e-15)


def test_sparse_v_needs_more_blocks():
    n = 400
    tol = 1e-3
    p = math.log(n) / n
    mean_blocks = {}
    for d in (1, n):
        a = synth.spectral_blockdiag_v(n, synth.matrix1_sigma(n), d, seed=7)
        nb = [farpca(a, FarpcaParams(tol=tol, block=20, power=1, sketch="sparse_gaussian", p=p,
                                     seed=s)).blocks for s in range(4)]
        mean_blocks[d] = np.mean(nb)
    assert mean_blocks[n] > mean_blocks[1] + 1.5
