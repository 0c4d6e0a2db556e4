"""Pins of the oracle's method against mathematics it does not use itself:
brute-force residuals, library SVD/QR, textbook randQB, the deterministic
bound of Lemma 4.1 and the Eckart-Young optimum."""
import math

import numpy as np
import pytest

from oracle import FarpcaParams, eig_svd, farpca, projection_svd
from oracle import omega as om
from paper_2506_03859_amd import synth

SKETCHES = [("gaussian", 0.0, 0), ("std_bernoulli", 0.05, 0), ("sparse_sign", 0.05, 0),
            ("sparse_sign", 0.0, 4), ("sparse_gaussian", 0.05, 0), ("bernoulli", 0.05, 0)]


@pytest.fixture(scope="module")
def a_small():
    return synth.spectral(500, 300, synth.matrix1_sigma(300), seed=2)


@pytest.fixture(scope="module")
def a_fast():
    return synth.spectral(400, 350, synth.matrix2_sigma(350), seed=3)


def orth(y):
    q, _ = np.linalg.qr(y)
    return q


def brute_residual2(a, y):
    q = orth(y)
    return float(np.linalg.norm(a - q @ (q.T @ a)) ** 2)


@pytest.mark.parametrize("sketch,p,zeta", SKETCHES)
@pytest.mark.parametrize("power", [0, 1, 2, 3])
def test_indicator_equals_brute_force_residual(a_small, sketch, p, zeta, power):
    # The indicator identity ||A - QC||^2 = ||A||^2 - ||C||^2 behind E, and
    # E_j = ||A||^2 - tr(T_j Z_j^{-1}) for every block j.
    prm = FarpcaParams(tol=3e-3, block=16, power=power, sketch=sketch, p=p, zeta=zeta, seed=11)
    r = farpca(a_small, prm, keep_bases=True)
    assert r.blocks >= 2
    nA2 = r.norm_a2
    eps = np.finfo(np.float64).eps
    for j, e in enumerate(r.e_history):
        y = r.Y[:, :(j + 1) * 16]
        # rounding of tr(T Z^{-1}) grows with cond(Z) = cond(Y)^2 (large for
        # P = 0, where Y = A Omega is not conditioned by power steps)
        tol = max(1e-12, 10 * eps * np.linalg.cond(y.T @ y))
        assert abs(e - brute_residual2(a_small, y)) <= tol * nA2


@pytest.mark.parametrize("sketch,p,zeta", SKETCHES)
def test_final_svd_is_svd_of_projection(a_small, sketch, p, zeta):
    # U Sigma V^T = Q Q^T A with orthonormal U, V, and Sigma equals the
    # singular values of Q^T A from LAPACK.
    prm = FarpcaParams(tol=1e-2, block=20, power=1, sketch=sketch, p=p, zeta=zeta, seed=5)
    r = farpca(a_small, prm, keep_bases=True)
    q = orth(r.Y)
    qa = q @ (q.T @ a_small)
    rec = (r.U * r.S) @ r.V.T
    assert np.linalg.norm(rec - qa) <= 1e-9 * np.linalg.norm(a_small)
    sv = np.linalg.svd(q.T @ a_small, compute_uv=False)
    assert np.allclose(r.S, sv, rtol=1e-8, atol=1e-12 * sv[0])
    assert np.all(np.diff(r.S) <= 0)
    k = r.U.shape[1]
    assert np.abs(r.U.T @ r.U - np.eye(k)).max() < 1e-8
    assert np.abs(r.V.T @ r.V - np.eye(k)).max() < 1e-6


def test_eig_svd_matches_lapack():
    x = synth.gaussian_matrix(300, 20, seed=1) * np.logspace(0, -3, 20)[None, :]
    u, s, v = eig_svd(x)
    assert np.all(np.diff(s) >= 0)                       # ascending
    ref = np.linalg.svd(x, compute_uv=False)[::-1]
    assert np.allclose(s, ref, rtol=1e-9)
    assert np.abs(u.T @ u - np.eye(20)).max() < 1e-9
    assert np.linalg.norm(u * s @ v.T - x) < 1e-10 * np.linalg.norm(x)


def test_eig_svd_dependent_columns():
    # two equal columns (an empty test-matrix column twice gives this): one
    # singular value is exactly 0 with a zero column of U (LAPACK finds it at
    # rounding level); the others are LAPACK's
    x = synth.gaussian_matrix(200, 10, seed=2)
    x[:, 7] = x[:, 3]
    u, s, v = eig_svd(x)
    assert s[0] == 0.0 and np.all(u[:, 0] == 0.0)
    ref = np.linalg.svd(x, compute_uv=False)[::-1]
    assert ref[0] < 1e-13 * ref[-1]
    assert np.allclose(s[1:], ref[1:], rtol=1e-9)
    assert np.abs(u[:, 1:].T @ u[:, 1:] - np.eye(9)).max() < 1e-9
    assert np.linalg.norm(u * s @ v.T - x) < 1e-10 * np.linalg.norm(x)


@pytest.mark.parametrize("sketch,p,zeta", SKETCHES)
def test_power0_is_textbook_randqb(a_fast, sketch, p, zeta):
    # With P = 0 the basis after j blocks spans A [Omega_0 ... Omega_{j-1}]
    # (randQB, Halko et al. Alg. 4.3 without power steps).
    b = 12
    prm = FarpcaParams(tol=1e-3, block=b, power=0, sketch=sketch, p=p, zeta=zeta, seed=8)
    r = farpca(a_fast, prm, keep_bases=True)
    n = a_fast.shape[1]
    om_all = np.hstack([om.omega_dense(n, b, j, sketch, 8, p, zeta) for j in range(r.blocks)])
    q_ref = orth(a_fast @ om_all)
    q = orth(r.Y)
    # compare the projectors onto the leading directions (well separated here)
    assert np.linalg.norm(q @ q.T @ q_ref - q_ref) < 1e-6 * math.sqrt(q_ref.shape[1])


@pytest.mark.parametrize("sketch,p,zeta", SKETCHES)
def test_first_block_power_is_textbook_power_scheme(a_fast, sketch, p, zeta):
    # First block, P = 2: span(Y_0) = range((A A^T)^2 A Omega_0).
    b = 10
    prm = FarpcaParams(rank=b, block=b, power=2, sketch=sketch, p=p, zeta=zeta, seed=4)
    r = farpca(a_fast, prm, keep_bases=True)
    n = a_fast.shape[1]
    o = om.omega_dense(n, b, 0, sketch, 4, p, zeta)
    if sketch == "std_bernoulli":
        o = o * math.sqrt(p * (1 - p))
    x = a_fast @ o
    for _ in range(2):
        x = orth(a_fast @ (a_fast.T @ x))
    q = orth(r.Y)
    assert np.linalg.norm(q - x @ (x.T @ q)) < 1e-8


@pytest.mark.parametrize("sketch,p,zeta", SKETCHES)
@pytest.mark.parametrize("power", [2, 4])
def test_deflated_power_step(a_small, sketch, p, zeta, power):
    # W_j = A^T(A Omega_j) - W Z^{-1} W^T Omega_j equals A^T (I - Q Q^T) A Omega_j
    # with Q an orthonormal basis of the previous Y (projector form).
    trace = []
    prm = FarpcaParams(tol=1e-3, block=16, power=power, sketch=sketch, p=p, zeta=zeta, seed=6)
    farpca(a_small, prm, trace=trace)
    checked = 0
    if power > 2:     # the shift is active from the third power step on
        assert any(t.get("alpha", 0.0) > 0 for t in trace)
    for t in trace:
        if t["y_prev"].shape[1] == 0:
            continue
        q = orth(t["y_prev"])
        if t["k"] == 1:
            s = t["sketch"]
            ref = a_small.T @ (s - q @ (q.T @ s))
        else:
            g = t["g_in"]
            ag = a_small @ g
            ref = a_small.T @ (ag - q @ (q.T @ ag)) - t["alpha"] * g
        assert np.linalg.norm(t["w_j"] - ref) <= 1e-8 * np.linalg.norm(ref)
        checked += 1
    assert checked >= 2


@pytest.mark.parametrize("p", [0.01, 0.3])
def test_alg2_rank_one_correction(a_small, p):
    # Section 3.1: sqrt(p(1-p)) A Omega_j = A B_j - p A 1_n.
    n = a_small.shape[1]
    omega = om.omega_dense(n, 16, 3, "std_bernoulli", 12, p)
    bmask = om.bernoulli_mask(n, 16, 3, 12, p).astype(float)
    lhs = math.sqrt(p * (1 - p)) * (a_small @ omega)
    rhs = a_small @ bmask - (a_small @ (p * np.ones(n)))[:, None]
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-14 * np.abs(a_small).max())


@pytest.mark.parametrize("sketch,p,zeta", SKETCHES)
def test_lemma_4_1_deterministic_bound(a_fast, sketch, p, zeta):
    # Lemma 4.1 (Halko et al. Thm 9.1): for Y = A Phi with Phi_1 = V_1^T Phi of
    # full row rank, ||(I - QQ^T)A||_F^2 <= ||S2||_F^2 + ||S2 Phi_2 Phi_1^+||_F^2.
    b, blocks = 10, 4
    n = a_fast.shape[1]
    phi = np.hstack([om.omega_dense(n, b, j, sketch, 31, p, zeta) for j in range(blocks)])
    prm = FarpcaParams(rank=b * blocks, block=b, power=0, sketch=sketch, p=p, zeta=zeta, seed=31)
    r = farpca(a_fast, prm, keep_bases=True)
    err2 = brute_residual2(a_fast, r.Y)
    assert abs(err2 - r.err_indicator) < 1e-9 * r.norm_a2
    _, s, vt = np.linalg.svd(a_fast, full_matrices=False)
    for k in (20, 30, 35):
        phi1 = vt[:k] @ phi
        phi2 = vt[k:] @ phi
        s2 = s[k:]
        bound = np.sum(s2 ** 2) + np.linalg.norm((s2[:, None] * phi2) @ np.linalg.pinv(phi1)) ** 2
        assert err2 <= bound * (1 + 1e-9)
        # Eckart-Young: no rank-l basis beats the tail of the spectrum
        assert err2 >= np.sum(s[blocks * b:] ** 2) * (1 - 1e-9)


def test_fixed_rank_mode(a_small):
    prm = FarpcaParams(rank=45, block=20, power=1, sketch="sparse_sign", zeta=4, seed=2)
    r = farpca(a_small, prm, keep_bases=True)
    assert r.blocks == 3 and r.rank == 60
    assert r.U.shape == (500, 45) and r.S.shape == (45,) and r.V.shape == (300, 45)
    _, s, _ = np.linalg.svd(a_small, full_matrices=False)
    err = np.linalg.norm(a_small - (r.U * r.S) @ r.V.T)
    assert err >= math.sqrt(np.sum(s[45:] ** 2)) * (1 - 1e-9)
    assert np.allclose(r.S[:10], s[:10], rtol=1e-6)


def test_stop_rule_and_cap(a_small):
    # strict relative stop test and the block cap
    prm = FarpcaParams(tol=1e-2, block=10, power=1, sketch="gaussian", seed=1)
    r = farpca(a_small, prm)
    assert r.status == 0 and r.err_indicator < 1e-4 * r.norm_a2
    assert all(e >= 1e-4 * r.norm_a2 for e in r.e_history[:-1])
    prm = FarpcaParams(tol=1e-12, block=10, power=1, sketch="gaussian", seed=1, max_blocks=3)
    r = farpca(a_small, prm)
    assert r.status == 1 and r.blocks == 3 and r.rank == 30


def test_shift_monotone_indicator(a_small):
    # P > 2 activates the shift; its rule is a reading of the paper (parity
    # unpinned).  Still: the indicator decreases block by block.
    prm = FarpcaParams(tol=1e-3, block=16, power=4, sketch="sparse_gaussian", p=0.05, seed=3)
    r = farpca(a_small, prm)
    assert r.status == 0
    assert np.all(np.diff(r.e_history) < 0)


def test_same_seed_same_result(a_small):
    prm = FarpcaParams(tol=1e-2, block=16, power=1, sketch="sparse_sign", zeta=4, seed=9)
    r1 = farpca(a_small, prm)
    r2 = farpca(a_small, prm)
    assert np.array_equal(r1.S, r2.S) and np.array_equal(r1.U, r2.U)


def test_wide_matrix(a_small):
    # m < n is allowed: the same loop on the 300 x 500 transpose.
    at = a_small.T.copy()
    prm = FarpcaParams(tol=1e-2, block=16, power=1, sketch="sparse_sign", zeta=4, seed=1)
    r = farpca(at, prm, keep_bases=True)
    assert abs(r.err_indicator - brute_residual2(at, r.Y)) < 1e-9 * r.norm_a2
    assert r.err_indicator < 1e-4 * r.norm_a2


def test_expected_error_bound_eq_4_9(a_fast):
    # eq (4.9): E||(I - QQ^T)A||_F <= (1 + k/(h-1))^{1/2} (sum_{j>k} s_j^2)^{1/2}
    # for a Gaussian test matrix with l = k + h columns; mean over 20 seeds.
    k, h = 15, 10
    _, s, _ = np.linalg.svd(a_fast, full_matrices=False)
    bound = math.sqrt(1 + k / (h - 1)) * math.sqrt(np.sum(s[k:] ** 2))
    errs = []
    for seed in range(20):
        prm = FarpcaParams(rank=k + h, block=k + h, power=0, sketch="gaussian", seed=100 + seed)
        r = farpca(a_fast, prm)
        errs.append(math.sqrt(max(r.err_indicator, 0.0)))
    assert np.mean(errs) <= bound


@pytest.mark.parametrize("power", [1, 2])
def test_projection_svd_matches_final_step(a_small, power):
    # for well-conditioned Z the paper's final step (eig(Z), eig(D^T T D))
    # and the plain QR + SVD definition agree
    prm = FarpcaParams(tol=1e-2, block=20, power=power, sketch="sparse_sign", zeta=4, seed=5)
    r = farpca(a_small, prm, keep_bases=True)
    s = projection_svd(a_small, r.Y)
    assert np.allclose(r.S, s, rtol=0, atol=1e-12 * s[0])
