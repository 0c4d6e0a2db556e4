"""Pins of the oracle's random test matrices against things other than itself:
numpy's own Philox4x64-10, the definitions' moments and support, Hoeffding's
bound on nonzero counts (Section 3.1), and Theorem 3.2's Gaussian limit."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import omega as om
from oracle.philox import draws32, draws64, philox4x64_10
from paper_2506_03859_amd import synth


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((5, 7, 9, 11), (123, 456)),
    ((2**64 - 2, 2**64 - 1, 3, 2**63), (2**64 - 1, 2**62 + 5)),
    ((17, 3, 2, 1), (20260101, 0)),
])
def test_philox_matches_numpy_library(ctr, key):
    # numpy's Philox increments its 256-bit counter before each block, so its
    # first block is philox(ctr + 1).
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    ref = bg.random_raw(8)
    c = list(ctr)
    blocks = []
    for _ in range(2):
        carry = 1
        for i in range(4):
            v = c[i] + carry
            c[i] = v & (2**64 - 1)
            carry = v >> 64
        blocks.append(list(c))
    mine = philox4x64_10(np.array(blocks, dtype=np.uint64), key).reshape(-1)
    assert np.array_equal(mine, ref)


def test_philox_known_answer_zero():
    # Published known-answer vector of Philox4x64-10 for counter = key = 0.
    out = philox4x64_10(np.zeros((1, 4), dtype=np.uint64), (0, 0))[0]
    assert [int(x) for x in out] == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC,
                                     0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


def test_draw_layout():
    rows = np.array([0, 3, 1000])
    w = draws64(42, 5, 2, rows, 6)
    ctr = np.array([[r, 5, 2, t] for r in rows for t in range(2)], dtype=np.uint64)
    raw = philox4x64_10(ctr, (42, 0)).reshape(len(rows), 8)
    assert np.array_equal(w, raw[:, :6])
    d32 = draws32(42, 5, 2, rows, 5)
    assert np.array_equal(d32[:, 0], raw[:, 0] & np.uint64(0xFFFFFFFF))
    assert np.array_equal(d32[:, 1], raw[:, 0] >> np.uint64(32))
    assert np.array_equal(d32[:, 4], raw[:, 2] & np.uint64(0xFFFFFFFF))


def test_threshold32():
    assert om.threshold32(0.5) == 2**31
    assert om.threshold32(0.25) == 2**30
    assert om.threshold32(1e-3) == 4294967
    with pytest.raises(ValueError):
        om.threshold32(1.0)


def test_fixed_count_sparse_sign_rows():
    n, b, zeta = 4000, 64, 8
    o = om.omega_dense(n, b, 3, "sparse_sign", seed=9, zeta=zeta)
    nz = o != 0
    assert np.all(nz.sum(axis=1) == zeta)
    assert np.allclose(np.abs(o[nz]), 1.0 / math.sqrt(zeta), rtol=0, atol=0)
    # signs balanced, columns used uniformly (each column gets zeta/b of rows)
    assert abs(np.mean(o[nz] > 0) - 0.5) < 4 * math.sqrt(0.25 / nz.sum())
    col = nz.sum(axis=0)
    expect = n * zeta / b
    assert np.all(np.abs(col - expect) < 6 * math.sqrt(expect))


def test_floyd_sampling_uniform_over_subsets():
    # Floyd's algorithm draws each of the C(b, zeta) subsets with equal
    # probability; chi-square over 20000 rows, b = 5, zeta = 2 (10 subsets).
    n, b, zeta = 20000, 5, 2
    chosen, _ = om.sparse_sign_fixed_mask_signs(n, b, 0, 77, zeta)
    codes = (chosen * (1 << np.arange(b))).sum(axis=1)
    _, counts = np.unique(codes, return_counts=True)
    assert counts.size == math.comb(b, zeta)
    chi2 = stats.chisquare(counts)
    assert chi2.pvalue > 1e-4


@pytest.mark.parametrize("sketch,p", [
    ("std_bernoulli", 0.01), ("std_bernoulli", 0.3), ("sparse_sign", 0.05),
    ("sparse_gaussian", 0.05), ("gaussian", 0.0),
])
def test_mean_zero_unit_variance(sketch, p):
    # Theorem 3.2 proof / Remark 3.7: entries i.i.d. mean 0, variance 1.
    n, b = 30000, 64
    o = om.omega_dense(n, b, 1, sketch, seed=5, p=p)
    cnt = o.size
    mean, var = o.mean(), o.var()
    # fourth moment bounds the standard error of the variance
    m4 = np.mean(o ** 4)
    assert abs(mean) < 5 / math.sqrt(cnt)
    assert abs(var - 1.0) < 5 * math.sqrt(m4 / cnt)


def test_std_bernoulli_half_is_rademacher():
    o = om.omega_dense(2000, 32, 0, "std_bernoulli", seed=1, p=0.5)
    assert set(np.unique(o)) == {-1.0, 1.0}


@pytest.mark.parametrize("sketch", ["bernoulli", "sparse_sign", "sparse_gaussian", "std_bernoulli"])
def test_nnz_hoeffding(sketch):
    # Section 3: P(|nnz(B) - n l p| >= t) <= exp(-2 t^2 / (n l)); take the
    # t whose bound is 1e-9.
    n, b, p = 20000, 64, 0.003
    o = om.omega_dense(n, b, 2, sketch, seed=13, p=p)
    if sketch == "std_bernoulli":
        nnz = np.sum(o > 0)          # the positive entries are B's ones
    else:
        nnz = np.count_nonzero(o)
    t = math.sqrt(n * b * math.log(1e9) / 2)
    assert abs(nnz - n * b * p) < t


def test_sparse_gaussian_pattern_is_bernoulli_mask():
    n, b, p = 3000, 40, 0.1
    sg = om.omega_dense(n, b, 4, "sparse_gaussian", seed=3, p=p)
    mask = om.bernoulli_mask(n, b, 4, 3, p)
    assert np.array_equal(sg != 0, mask)
    g = om.gaussian_values(n, b, 4, 3)
    assert np.allclose(sg[mask], g[mask] / math.sqrt(p), rtol=1e-15)


def test_gaussian_values_ks():
    g = om.gaussian_values(5000, 20, 0, 99).reshape(-1)
    assert stats.kstest(g, "norm").pvalue > 1e-4


@pytest.mark.parametrize("sketch,p", [("std_bernoulli", 0.01), ("sparse_sign", 0.02),
                                      ("sparse_gaussian", 0.02)])
def test_theorem_3_2_rotated_entries_gaussian(sketch, p):
    # Theorem 3.2 / Props 3.5-3.6: for an orthogonal V with small entries,
    # the entries of V^T Omega are close to N(0, 1).
    n, b = 2000, 8
    rng = np.random.default_rng(4)
    v = synth.haar_columns(n, n, rng)
    o = om.omega_dense(n, b, 0, sketch, seed=21, p=p)
    x = (v.T @ o).reshape(-1)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # and the sparse matrix itself is far from Gaussian
    assert stats.kstest(o.reshape(-1), "norm").pvalue < 1e-10


def test_blocks_and_seeds_independent_streams():
    a = om.omega_dense(500, 16, 0, "sparse_sign", seed=1, zeta=4)
    b = om.omega_dense(500, 16, 1, "sparse_sign", seed=1, zeta=4)
    c = om.omega_dense(500, 16, 0, "sparse_sign", seed=2, zeta=4)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.array_equal(a, om.omega_dense(500, 16, 0, "sparse_sign", seed=1, zeta=4))


def test_default_p_rules():
    # Section 5's rules for the paper's n x n matrices: p1 = max(1e-3, ln n / n)
    # (standardized Bernoulli), p2 = max(1e-3, 10 / n) (the other sparse matrices)
    from oracle import default_p
    assert default_p("std_bernoulli", 5000, 5000) == pytest.approx(math.log(5000) / 5000, rel=1e-15)
    assert default_p("sparse_sign", 5000, 5000) == pytest.approx(2e-3, rel=1e-15)
    assert default_p("std_bernoulli", 30000, 30000) == 1e-3      # ln n / n = 3.4e-4 < 1e-3
    assert default_p("sparse_gaussian", 30000, 30000) == 1e-3
    # for m x n A the rule follows the n rows of Omega_j: the expected number of
    # nonzeros in a column of Omega_j, p n, is at least ln n (p1) or 10 (p2) for any m
    for m in (300, 4000, 200000):
        assert default_p("std_bernoulli", m, 4000) * 4000 >= math.log(4000) * (1 - 1e-12)
        assert default_p("bernoulli", m, 4000) * 4000 >= 10 * (1 - 1e-12)
