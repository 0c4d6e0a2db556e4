"""The post-processing truncation of the fixed-precision output (Section 5.4,
after Hallman's block method), pinned independently of its formula: the error
of every rank-r truncation is computed directly from the factors and A, and
the truncation rank is checked for validity and minimality against those
residuals; a matrix of known exact rank gives the rank in closed form."""
import numpy as np
import pytest

from oracle import FarpcaParams, farpca, truncation_rank
from paper_2506_03859_amd import synth


def direct_residuals(a, res):
    """||A - U_r S_r V_r^T||_F^2 for r = 0 .. l, by forming each truncation."""
    out = []
    for r in range(res.S.size + 1):
        approx = (res.U[:, :r] * res.S[:r][None, :]) @ res.V[:, :r].T
        out.append(float(np.sum((a - approx) ** 2)))
    return np.array(out)


@pytest.mark.parametrize("sketch,p,zeta", [("gaussian", 0.0, 0), ("sparse_sign", 0.0, 4),
                                           ("std_bernoulli", 0.0, 0)])
def test_truncation_error_identity_and_minimality(sketch, p, zeta):
    m, n = 160, 120
    a = synth.spectral(m, n, np.arange(1, n + 1, dtype=np.float64) ** -1.5, seed=3)
    tol = 0.05
    res = farpca(a, FarpcaParams(tol=tol, block=10, power=1, sketch=sketch, p=p, zeta=zeta, seed=9))
    assert res.status == 0
    resid = direct_residuals(a, res)
    # identity: the truncation error is E + the discarded singular values squared
    tail = np.concatenate([np.cumsum((res.S ** 2)[::-1])[::-1], [0.0]])
    np.testing.assert_allclose(resid, res.err_indicator + tail, rtol=0, atol=1e-10 * res.norm_a2)
    r = truncation_rank(res.S, res.err_indicator, res.norm_a2, tol)
    thr = tol * tol * res.norm_a2
    assert r < res.S.size                      # the block output has slack to cut
    assert resid[r] < thr                      # valid
    assert r == 0 or resid[r - 1] >= thr * (1 - 1e-12)   # minimal


def test_truncation_exact_rank_closed_form():
    # rank-10 matrix with singular values 10, 9, ..., 1: once the basis holds
    # the range (E = 0 up to rounding) the truncation rank follows from the
    # spectrum alone
    m, n, k = 90, 70, 10
    sig = np.arange(k, 0, -1, dtype=np.float64)
    a = synth.spectral(m, n, np.concatenate([sig, np.zeros(n - k)]), seed=5)
    norm2 = float(np.sum(sig ** 2))
    res = farpca(a, FarpcaParams(tol=1e-6, block=5, power=1, sketch="gaussian", seed=2, max_blocks=4))
    assert res.err_indicator < 1e-20 * norm2
    # keep all ten for a tight tolerance
    assert truncation_rank(res.S, res.err_indicator, res.norm_a2, 1e-6) == k
    # dropping sigma_10 = 1 costs 1 / 385 of ||A||^2: allowed just above, not just below
    edge = np.sqrt(1.0 / norm2)
    assert truncation_rank(res.S, res.err_indicator, res.norm_a2, edge * 1.01) == k - 1
    assert truncation_rank(res.S, res.err_indicator, res.norm_a2, edge * 0.99) == k
    # dropping 1 and 2 costs 5 / 385
    assert truncation_rank(res.S, res.err_indicator, res.norm_a2, np.sqrt(5.0 / norm2) * 1.01) == k - 2


def test_truncation_not_converged_keeps_all():
    s = np.array([3.0, 2.0, 1.0])
    # E already above the threshold: nothing can be cut
    assert truncation_rank(s, 10.0, 14.0, 0.5) == 3
    # E = 0: the tail 1 is below 3.5, the tail 1 + 4 is not
    assert truncation_rank(s, 0.0, 14.0, 0.5) == 2
    assert truncation_rank(np.zeros(0), 0.0, 1.0, 0.5) == 0
