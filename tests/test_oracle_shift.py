"""Pin of the shifted power iteration (Algorithm 1 and Algorithm 2, the
alpha update after each eigSVD of a power step) against the mathematics of
subspace iteration, not against the oracle itself.

The reading taken: alpha is compared with the smallest singular value of the
block's power iterate and, when below it, moved half way towards it.  Its
consequences that hold whatever the implementation:

* X = A^T A G - alpha G is the shifted operator A^T A - alpha I applied to G.
  Once span(G) is close to the top-b right singular subspace, the smallest
  singular value of X is sigma_b^2 - alpha, so the update has the fixed point
  alpha = sigma_b^2 / 2: alpha stays below sigma_b^2 and settles there.
* With that shift the iteration contracts the unwanted directions by
  max_i>b |sigma_i^2 - alpha| / (sigma_b^2 - alpha), which is smaller than the
  unshifted sigma_{b+1}^2 / sigma_b^2 for the spectrum used here, so after the
  same number of steps the subspace is no farther from the exact one than
  plain subspace iteration (numpy QR) leaves it.

The spectrum is chosen so that the two plausible misreadings fail: driving
alpha by the largest singular value of the block (the garbled index read
literally with ascending values) sends alpha to sigma_1^2 / 2 = sigma_b^2,
and dropping the halving sets alpha to sigma_b^2 at the first update; both
put the shift on the b-th eigenvalue, which annihilates that direction.
"""
import numpy as np
import pytest

from oracle import FarpcaParams, farpca

B = 8          # block size = rank: one block, no deflation
P = 10         # power steps (the shift acts for P > 2)
N = 160


def _spectrum():
    # sigma^2: top b evenly from 1.0 down to 0.5, the rest in [0.1, 0.35]
    top = np.linspace(1.0, 0.5, B)
    rng = np.random.default_rng(20240611)
    tail = np.sort(rng.uniform(0.1, 0.35, N - B))[::-1]
    return np.sqrt(np.concatenate([top, tail]))


def _haar(n, seed):
    g = np.random.default_rng(seed).standard_normal((n, n))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


@pytest.fixture(scope="module")
def shifted_case():
    sigma = _spectrum()
    u = _haar(N, 1)
    v = _haar(N, 2)
    a = (u * sigma[None, :]) @ v.T
    trace = []
    prm = FarpcaParams(rank=B, block=B, power=P, sketch="gaussian", seed=7)
    res = farpca(a, prm, trace=trace)
    return a, sigma, u, v, res, trace, prm


def _max_angle_sin(q1, q2):
    # sine of the largest principal angle between two orthonormal bases
    s = np.linalg.svd(q1.T @ q2, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2)))


def test_shift_fixed_point(shifted_case):
    _, sigma, _, _, _, trace, _ = shifted_case
    sb2 = sigma[B - 1] ** 2
    alphas = [t["alpha"] for t in trace if t["k"] >= 2]
    assert len(alphas) == P - 1
    assert alphas[0] == 0.0                      # alpha = 0 at the first shifted step
    assert all(a < sb2 for a in alphas)          # never reaches sigma_b^2
    assert all(x <= y + 1e-15 for x, y in zip(alphas, alphas[1:]))   # non-decreasing
    # settled at the fixed point sigma_b^2 / 2
    assert abs(alphas[-1] - sb2 / 2) <= 0.03 * sb2
    assert abs(alphas[-2] - sb2 / 2) <= 0.03 * sb2


def test_shifted_iteration_converges_at_least_as_fast(shifted_case):
    a, sigma, u, v, res, _, prm = shifted_case
    # exact top-b left singular subspace
    u_top = u[:, :B]
    q_oracle, _ = np.linalg.qr(res.U)
    err_shift = _max_angle_sin(q_oracle, u_top)
    # plain (unshifted) subspace iteration from the same Gaussian start with the
    # same number of products with A^T A, orthonormalised by numpy QR each step
    from oracle.omega import omega_dense
    om = omega_dense(N, B, 0, "gaussian", prm.seed, 0.0, 0)
    g, _ = np.linalg.qr(a.T @ (a @ om))
    for _ in range(2, P + 1):
        g, _ = np.linalg.qr(a.T @ (a @ g))
    q_plain, _ = np.linalg.qr(a @ g)
    err_plain = _max_angle_sin(q_plain, u_top)
    assert err_plain > 1e-6          # the unshifted run has not converged
    assert err_shift <= err_plain
    # the predicted contraction: with alpha = sigma_b^2 / 2 the shifted ratio
    # is 0.6 against 0.7 unshifted here, so the gain compounds over the steps
    sb2 = sigma[B - 1] ** 2
    rho_shift = max(abs(sigma[B:] ** 2 - sb2 / 2)) / (sb2 - sb2 / 2)
    rho_plain = sigma[B] ** 2 / sb2
    assert rho_shift < rho_plain
    assert err_shift <= 0.5 * err_plain
