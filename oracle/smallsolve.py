"""The small projected problem of hybrid AB-/BA-GMRES (oracle, FP64).

At iteration k the Arnoldi process gives the (k+1) x k upper Hessenberg
matrix H_k with M W_k = W_{k+1} H_k (eq. (8)).  The hybrid step solves the
Tikhonov-regularised projected problem of eq. (12)

    y_k = argmin_y || [H_k; lam I] y - beta [e_1; 0] ||,   beta = ||r_0||,

with lam chosen per iteration (Sec. 3.1).  With the SVD H_k = U S V^T,
uhat = beta U^T e_1 (first k entries) and uhat_{k+1} the component of
beta e_1 outside range(H_k):

    y_k     = sum_i sigma_i uhat_i / (sigma_i^2 + lam^2) v_i
    rho^2   = sum_i (lam^2/(sigma_i^2+lam^2))^2 uhat_i^2 + uhat_{k+1}^2
    GCV(lam) = rho^2 / (1 + sum_i lam^2/(sigma_i^2+lam^2))^2       (eq. (15))

The denominator is trace(I_{k+1} - H_k H_{k,lam}) with
H_{k,lam} = (H_k^T H_k + lam^2 I)^{-1} H_k^T, as printed in eq. (15).

Readings where the paper is silent (shared with the GPU path by definition,
not by code):
  * GCV minimiser: 256-point log grid on [1e-8 sigma_1, sigma_1], the global
    grid minimum (first index on ties), then 60 golden-section steps in
    log(lam) on [grid_{g-1}, grid_{g+1}] (clamped to the grid); the refined
    point is kept unless its GCV value exceeds the grid minimum.
  * Discrepancy principle as a lambda rule (AB mode): find lam with
    rho(lam) = tau ||e||.  rho is increasing in lam; lam = 0 if
    rho(0) >= tau ||e||, lam = inf (y = 0) if beta <= tau ||e||, otherwise
    100 bisection steps in log(lam) on [1e-12 sigma_1, 1e8 sigma_1].
  * No regularisation (plain AB/BA-GMRES, eqs. (6)-(7)): the minimum-norm
    least-squares y, dropping sigma_i < 1e-14 sigma_1.
"""
from __future__ import annotations

import math

import numpy as np

RULE_NONE, RULE_FIXED, RULE_GCV, RULE_DP, RULE_LCURVE = "none", "fixed", "gcv", "dp", "lcurve"

GCV_GRID = 256
GCV_LO = 1e-8
GOLDEN_STEPS = 60
DP_STEPS = 100
DP_LO, DP_HI = 1e-12, 1e8
RANK_CUT = 1e-14


def givens_qr(H: np.ndarray, beta: float):
    """Givens QR of the (k+1) x k Hessenberg H applied to beta*e_1.

    Returns (R, g, res): R is k x k upper triangular, g the first k entries of
    Q^T beta e_1 and res = |last entry| = min_y ||H y - beta e_1||
    (the GMRES residual of eq. (9)).
    """
    kp1, k = H.shape
    assert kp1 == k + 1
    R = np.array(H, dtype=np.float64, copy=True)
    g = np.zeros(k + 1)
    g[0] = beta
    for j in range(k):
        a, b = R[j, j], R[j + 1, j]
        r = math.hypot(a, b)
        if r == 0.0:
            c, s = 1.0, 0.0
        else:
            c, s = a / r, b / r
        for col in range(j, k):
            u, v = R[j, col], R[j + 1, col]
            R[j, col] = c * u + s * v
            R[j + 1, col] = -s * u + c * v
        u, v = g[j], g[j + 1]
        g[j] = c * u + s * v
        g[j + 1] = -s * u + c * v
    return np.triu(R[:k, :k]), g[:k].copy(), abs(g[k])


def svd_proj(H: np.ndarray, beta: float):
    """sigma (descending), uhat = beta U^T e_1 (k entries) and V of H_k."""
    U, s, Vt = np.linalg.svd(H, full_matrices=True)
    k = H.shape[1]
    uhat = beta * U[0, :k]
    return s, uhat, Vt.T


def filt(sigma, lam):
    """Tikhonov filter pieces: phi_i = lam^2/(sigma_i^2+lam^2)."""
    s2 = sigma * sigma
    l2 = lam * lam
    return l2 / (s2 + l2)


def resid2(lam, sigma, uhat, uk1):
    """rho(lam)^2 = ||H_k y_lam - beta e_1||^2."""
    if lam == 0.0:
        return float(uk1 * uk1)
    if math.isinf(lam):
        return float(np.sum(uhat * uhat) + uk1 * uk1)
    ph = filt(sigma, lam)
    return float(np.sum((ph * uhat) ** 2) + uk1 * uk1)


def gcv(lam, sigma, uhat, uk1):
    """GCV function of eq. (15) for the projected problem."""
    ph = filt(sigma, lam)
    den = 1.0 + float(np.sum(ph))
    return resid2(lam, sigma, uhat, uk1) / (den * den)


def choose_gcv(sigma, uhat, uk1):
    s1 = float(np.max(sigma))
    if s1 == 0.0:
        return 0.0
    # the grid points are sigma_1 * 10^(-8 + 8 g/255), written out
    grid = np.array([s1 * 10.0 ** (math.log10(GCV_LO) * (1.0 - g / (GCV_GRID - 1.0)))
                     for g in range(GCV_GRID)])
    vals = np.array([gcv(l, sigma, uhat, uk1) for l in grid])
    g = int(np.argmin(vals))                     # first index on ties
    lo = math.log(grid[max(g - 1, 0)])
    hi = math.log(grid[min(g + 1, GCV_GRID - 1)])
    invphi = (math.sqrt(5.0) - 1.0) / 2.0
    c = hi - invphi * (hi - lo)
    d = lo + invphi * (hi - lo)
    fc = gcv(math.exp(c), sigma, uhat, uk1)
    fd = gcv(math.exp(d), sigma, uhat, uk1)
    for _ in range(GOLDEN_STEPS):
        if fc <= fd:
            hi, d, fd = d, c, fc
            c = hi - invphi * (hi - lo)
            fc = gcv(math.exp(c), sigma, uhat, uk1)
        else:
            lo, c, fc = c, d, fd
            d = lo + invphi * (hi - lo)
            fd = gcv(math.exp(d), sigma, uhat, uk1)
    lam = math.exp(0.5 * (lo + hi))
    if gcv(lam, sigma, uhat, uk1) <= vals[g]:
        return lam
    return float(grid[g])


def choose_dp(sigma, uhat, uk1, beta, target):
    """lam with rho(lam) = target (= tau ||e||), see the module docstring."""
    t2 = target * target
    if uk1 * uk1 >= t2:
        return 0.0
    if beta * beta <= t2:
        return math.inf
    s1 = float(np.max(sigma))
    lo, hi = math.log(DP_LO * s1), math.log(DP_HI * s1)
    for _ in range(DP_STEPS):
        mid = 0.5 * (lo + hi)
        if resid2(math.exp(mid), sigma, uhat, uk1) < t2:
            lo = mid
        else:
            hi = mid
    return math.exp(0.5 * (lo + hi))


def lcurve_corner(sigma, uhat, uk1):
    """Corner of the L-curve (eq. (14)): maximum curvature on the GCV grid.

    The curve is (a, b) = (log ||H_k y_lam - beta e_1||, log ||y_lam||) as a
    function of t = ln(lam).  Its signed curvature
    (a' b'' - a'' b') / (a'^2 + b'^2)^{3/2} is evaluated in closed form on the
    same 256-point log grid as GCV and the global maximum (first index on
    ties) is returned.
    """
    s1 = float(np.max(sigma))
    if s1 == 0.0:
        return 0.0
    grid = np.array([s1 * 10.0 ** (math.log10(GCV_LO) * (1.0 - g / (GCV_GRID - 1.0)))
                     for g in range(GCV_GRID)])
    best, arg = -math.inf, 0
    for gi, lam in enumerate(grid):
        kap = _lcurve_curvature(lam, sigma, uhat, uk1)
        if kap > best:
            best, arg = kap, gi
    return float(grid[arg])


def _lcurve_curvature(lam, sigma, uhat, uk1):
    # phi_i = sigma_i^2/(sigma_i^2+lam^2); with t = ln(lam), d phi/dt = -2 phi (1-phi).
    # R = ||r||^2 = sum (1-phi)^2 u^2 + uk1^2,   E = ||y||^2 = sum phi u^2/(sigma^2+lam^2)
    # R'  =  4 sum phi (1-phi)^2 u^2            R'' = -8 sum phi (1-phi)^2 (1-3 phi) u^2
    # E'  = -4 sum phi (1-phi) u^2/(s^2+l^2)    E'' =  8 sum phi (1-phi) (2-3 phi) u^2/(s^2+l^2)
    s2 = sigma * sigma
    l2 = lam * lam
    phi = s2 / (s2 + l2)
    u2 = uhat * uhat
    w = u2 / (s2 + l2)
    R = float(np.sum((1.0 - phi) ** 2 * u2) + uk1 * uk1)
    E = float(np.sum(phi * w))
    R1 = float(4.0 * np.sum(phi * (1.0 - phi) ** 2 * u2))
    R2 = float(-8.0 * np.sum(phi * (1.0 - phi) ** 2 * (1.0 - 3.0 * phi) * u2))
    E1 = float(-4.0 * np.sum(phi * (1.0 - phi) * w))
    E2 = float(8.0 * np.sum(phi * (1.0 - phi) * (2.0 - 3.0 * phi) * w))
    if R <= 0.0 or E <= 0.0:
        return -math.inf
    a1, b1 = R1 / (2.0 * R), E1 / (2.0 * E)
    a2 = (R2 * R - R1 * R1) / (2.0 * R * R)
    b2 = (E2 * E - E1 * E1) / (2.0 * E * E)
    den = (a1 * a1 + b1 * b1) ** 1.5
    if den == 0.0:
        return -math.inf
    return (a1 * b2 - a2 * b1) / den


def solve_projected(H: np.ndarray, beta: float, rule: str, lam_fixed: float = 0.0,
                    dp_target: float | None = None):
    """Regularised projected solve of eq. (12) with the chosen lambda rule.

    Returns dict(lam, y, rho_hat, sigma, uhat, uk1).
    """
    k = H.shape[1]
    _, _, uk1 = givens_qr(H, beta)
    sigma, uhat, V = svd_proj(H, beta)
    s1 = float(sigma[0]) if k > 0 else 0.0
    if rule == RULE_NONE:
        lam = 0.0
    elif rule == RULE_FIXED:
        lam = float(lam_fixed)
    elif rule == RULE_GCV:
        lam = choose_gcv(sigma, uhat, uk1)
    elif rule == RULE_DP:
        assert dp_target is not None
        lam = choose_dp(sigma, uhat, uk1, beta, dp_target)
    elif rule == RULE_LCURVE:
        lam = lcurve_corner(sigma, uhat, uk1)
    else:
        raise ValueError(rule)
    if math.isinf(lam):
        y = np.zeros(k)
        rho2 = float(beta * beta)
    elif lam == 0.0:
        keep = sigma >= RANK_CUT * s1
        coef = np.where(keep, uhat / np.where(keep, sigma, 1.0), 0.0)
        y = V @ coef
        rho2 = float(np.sum(np.where(keep, 0.0, uhat) ** 2) + uk1 * uk1)
    else:
        coef = sigma * uhat / (sigma * sigma + lam * lam)
        y = V @ coef
        rho2 = resid2(lam, sigma, uhat, uk1)
    return dict(lam=lam, y=y, rho_hat=math.sqrt(max(rho2, 0.0)), sigma=sigma,
                uhat=uhat, uk1=uk1)
