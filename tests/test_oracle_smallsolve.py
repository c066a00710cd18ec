"""Pins for the oracle's projected solve (eqs. (9), (12), (14), (15)).

Every quantity computed from the SVD of H_k is checked against an explicit,
dense evaluation that does not use the SVD: least squares on the stacked
matrix [H_k; lam I], explicit residuals, the trace of I - H_k H_{k,lam}
formed as a matrix, and numerical derivatives of the L-curve.
"""
import math

import numpy as np
import pytest

from oracle import smallsolve as ss


def random_hessenberg(k, seed, decay=0.7):
    r = np.random.default_rng(seed)
    H = np.triu(r.standard_normal((k + 1, k)), -1)
    # ill-conditioned like a Krylov projection of a smoothing operator
    H = H * (decay ** np.arange(k))[None, :]
    for j in range(k):
        H[j + 1, j] = abs(H[j + 1, j]) + 1e-3 * decay ** j
    return H


@pytest.mark.parametrize("k", [1, 2, 5, 17, 40])
def test_givens_residual_equals_least_squares_residual(k):
    H = random_hessenberg(k, k)
    beta = 3.7
    R, g, res = ss.givens_qr(H, beta)
    rhs = np.zeros(k + 1)
    rhs[0] = beta
    y = np.linalg.lstsq(H, rhs, rcond=None)[0]
    assert abs(res - np.linalg.norm(H @ y - rhs)) < 1e-12 * beta
    # the triangular factor solves the same problem
    np.testing.assert_allclose(np.linalg.solve(R, g), y, rtol=1e-9, atol=1e-12 * np.abs(y).max())


@pytest.mark.parametrize("k", [3, 12, 30])
def test_svd_factors(k):
    H = random_hessenberg(k, 100 + k)
    s, uhat, V = ss.svd_proj(H, 2.0)
    U, s2, Vt = np.linalg.svd(H)
    assert np.all(np.diff(s) <= 0)
    np.testing.assert_allclose(np.sort(s ** 2), np.sort(np.linalg.eigvalsh(H.T @ H)),
                               rtol=1e-10, atol=1e-13 * s[0] ** 2)
    recon = U[:, :k] @ np.diag(s) @ Vt
    assert np.linalg.norm(H - recon) < 1e-13 * s[0] * k
    # |uhat|^2 + uhat_{k+1}^2 = beta^2
    _, _, uk1 = ss.givens_qr(H, 2.0)
    assert abs(np.sum(uhat ** 2) + uk1 ** 2 - 4.0) < 1e-12


@pytest.mark.parametrize("lam", [1e-4, 1e-2, 0.3, 5.0])
def test_regularised_solution_equals_stacked_least_squares(lam):
    k = 15
    H = random_hessenberg(k, 7)
    beta = 1.3
    sol = ss.solve_projected(H, beta, "fixed", lam_fixed=lam)
    M = np.vstack([H, lam * np.eye(k)])
    rhs = np.zeros(2 * k + 1)
    rhs[0] = beta
    y = np.linalg.lstsq(M, rhs, rcond=None)[0]
    np.testing.assert_allclose(sol["y"], y, rtol=1e-9, atol=1e-12 * np.abs(y).max())
    r = H @ y
    r[0] -= beta
    assert abs(sol["rho_hat"] - np.linalg.norm(r)) < 1e-12 * beta


def test_gcv_formula_equals_dense_trace_form():
    k = 12
    H = random_hessenberg(k, 11)
    beta = 2.5
    s, uhat, V = ss.svd_proj(H, beta)
    _, _, uk1 = ss.givens_qr(H, beta)
    rhs = np.zeros(k + 1)
    rhs[0] = beta
    for lam in s[0] * np.logspace(-8, 0, 37):
        Hl = np.linalg.solve(H.T @ H + lam ** 2 * np.eye(k), H.T)      # H_{k,lam}
        y = Hl @ rhs
        num = np.linalg.norm(H @ y - rhs) ** 2
        den = np.trace(np.eye(k + 1) - H @ Hl) ** 2
        ref = num / den
        assert abs(ss.gcv(lam, s, uhat, uk1) - ref) < 1e-9 * ref


@pytest.mark.parametrize("seed", range(6))
def test_gcv_choice_is_global_grid_minimum_and_not_worse(seed):
    k = 8 + 3 * seed
    H = random_hessenberg(k, 40 + seed)
    beta = 1.0
    s, uhat, _ = ss.svd_proj(H, beta)
    _, _, uk1 = ss.givens_qr(H, beta)
    lam = ss.choose_gcv(s, uhat, uk1)
    grid = s[0] * np.logspace(-8, 0, 256)
    vals = np.array([ss.gcv(l, s, uhat, uk1) for l in grid])
    assert ss.gcv(lam, s, uhat, uk1) <= vals.min() * (1 + 1e-12)
    g = int(np.argmin(vals))
    assert grid[max(g - 1, 0)] * (1 - 1e-12) <= lam <= grid[min(g + 1, 255)] * (1 + 1e-12)


def test_dp_lambda_hits_target_and_limits():
    k = 20
    H = random_hessenberg(k, 5)
    beta = 4.0
    s, uhat, _ = ss.svd_proj(H, beta)
    _, _, uk1 = ss.givens_qr(H, beta)
    for frac in (0.2, 0.5, 0.9):
        target = uk1 + frac * (beta - uk1)
        lam = ss.choose_dp(s, uhat, uk1, beta, target)
        sol = ss.solve_projected(H, beta, "fixed", lam_fixed=lam)
        assert abs(sol["rho_hat"] - target) < 1e-10 * target
    assert ss.choose_dp(s, uhat, uk1, beta, 0.5 * uk1) == 0.0
    assert math.isinf(ss.choose_dp(s, uhat, uk1, beta, 1.01 * beta))
    sol = ss.solve_projected(H, beta, "dp", dp_target=1.01 * beta)
    assert np.all(sol["y"] == 0) and abs(sol["rho_hat"] - beta) < 1e-14


def test_lambda_limits():
    k = 10
    H = random_hessenberg(k, 9, decay=0.9)
    beta = 1.0
    rhs = np.zeros(k + 1)
    rhs[0] = beta
    # lam = 0: plain GMRES least-squares solution
    y0 = ss.solve_projected(H, beta, "none")["y"]
    np.testing.assert_allclose(y0, np.linalg.lstsq(H, rhs, rcond=None)[0], rtol=1e-9)
    # lam -> inf: y -> 0 like beta * H^T e1 / lam^2
    s1 = np.linalg.norm(H, 2)
    big = 1e6 * s1
    y = ss.solve_projected(H, beta, "fixed", lam_fixed=big)["y"]
    np.testing.assert_allclose(y * big ** 2, H.T @ rhs, rtol=1e-9)


def test_lcurve_curvature_matches_numerical_derivatives():
    k = 14
    H = random_hessenberg(k, 21)
    beta = 1.0
    s, uhat, _ = ss.svd_proj(H, beta)
    _, _, uk1 = ss.givens_qr(H, beta)

    def curve(t):
        lam = math.exp(t)
        sol = ss.solve_projected(H, beta, "fixed", lam_fixed=lam)
        return math.log(sol["rho_hat"]), math.log(np.linalg.norm(sol["y"]))

    for lam in s[0] * np.array([1e-5, 1e-3, 1e-2, 0.1, 0.5]):
        t, h = math.log(lam), 1e-3
        (a0, b0), (am, bm), (ap, bp) = curve(t), curve(t - h), curve(t + h)
        a1, b1 = (ap - am) / (2 * h), (bp - bm) / (2 * h)
        a2, b2 = (ap - 2 * a0 + am) / h ** 2, (bp - 2 * b0 + bm) / h ** 2
        kap_num = (a1 * b2 - a2 * b1) / (a1 ** 2 + b1 ** 2) ** 1.5
        kap = ss._lcurve_curvature(lam, s, uhat, uk1)
        assert abs(kap - kap_num) < 1e-4 * max(1.0, abs(kap)), (lam, kap, kap_num)
