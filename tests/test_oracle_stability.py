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


def test_stored_stability_grid_reproduces():
    # tests/golden/stability_oracle_5000x5000.json (written by
    # tests/golden/stability_oracle.py, oracle only): the whole grid is there,
    # and one stored run comes out the same when the oracle is run again
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "stability_oracle_5000x5000.json")
    with open(path) as f:
        g = json.load(f)
    n, trials = g["n"], g["trials"]
    assert n == 5000 and g["tol"] == 1e-4 and trials == 10
    cells = g["cells"]
    assert len(cells) == 36 and all(len(v) == trials for v in cells.values())
    assert all(s in (0, 1) and 1 <= b <= 50 and e >= 0 for v in cells.values() for s, b, e in v)
    a = synth.spectral_blockdiag_v(n, synth.matrix1_sigma(n), n, seed=g["seed_matrix"])
    r = farpca(a, FarpcaParams(tol=1e-4, power=1, sketch="sparse_gaussian", p=1e-2, seed=1))
    err = float(np.linalg.norm(a - (r.U * r.S) @ r.V.T) / np.linalg.norm(a))
    s0, b0, e0 = cells[f"SG p=1e-2 d={n}"][0]
    assert (r.status, r.blocks) == (s0, b0)
    # the relative error moves by ~1e-9 with the BLAS thread count (the
    # oracle's ill-conditioned Z on this input amplifies rounding)
    assert abs(err - e0) <= 1e-8
