"""Hybrid AB-GMRES and BA-GMRES (Algorithms 1 and 2), oracle in FP64.

Given a forward projector A: R^n -> R^m, an unmatched backprojector
B: R^m -> R^n and data b, the method runs the Arnoldi process on M = AB
(AB mode, eq. (5)) or M = BA (BA mode, eq. (4)), and at every iteration k

  1. forms q = M w_k and orthogonalises it against W_k (eq. (8));
  2. chooses lam_k and solves the regularised projected problem (eq. (12));
  3. forms x_k = x_0 + B W_k y_k (AB) or x_0 + W_k y_k (BA) (eq. (13));
  4. forms the residual r_k = b - A x_k (AB) or B(b - A x_k) (BA);
  5. applies the stopping rule (Sec. 3.2).

The paper's loop orthogonalises one basis vector at a time (modified
Gram-Schmidt).  The GPU path uses classical Gram-Schmidt with one
re-orthogonalisation pass (CGS2), either as two passes per step or with the
second pass delayed by one step ("dcgs2", below); in exact arithmetic all
give the same W_{k+1} and H_k, so the oracle offers all three.

Delayed CGS2 (dcgs2).  The operator is applied to the once-orthogonalised
next vector v (the first pass of step k leaves v = M w_k - W_k h1), and the
second pass of step k is carried out together with the first pass of step
k+1: with z = M v, one sweep gives a = W_k^T v, gamma = v.v, b = W_k^T z and
delta = v.z.  Then
  * column k of H is completed: H[:k, k-1] += a, H[k, k-1] = alpha with
    alpha^2 = gamma - |a|^2 (a is small), and w_{k+1} = (v - W_k a)/alpha;
  * M w_{k+1} = (z - M W_k a)/alpha = (z - W_{k+1} t)/alpha with t = H_k a
    (the Arnoldi relation M W_k = W_{k+1} H_k), so its first-pass
    coefficients are h1 = W_{k+1}^T M w_{k+1}
    = ([b ; (delta - a.b)/alpha] - t)/alpha, and the next once-orthogonalised
    vector is z/alpha - W_{k+1} (t/alpha + h1).
Each step reads the basis twice instead of four times; the projected problem
of iteration k is known one operator application later, so a run that stops
at iteration k has applied M k+1 times.

Readings of points the paper leaves open:
  * x_0 = 0 unless given (u_0 = 0 in Algorithm 1).
  * Breakdown when h_{k+1,k} <= 1e-14 ||M w_k||: h_{k+1,k} is set to 0, the
    k-th iterate is formed and the run ends.
  * rho_k = ||b - A x_k|| (the data residual) is what the discrepancy
    principle and residual-norm stagnation test, in both modes.  The printed
    DP inequality is reversed; the run stops at the first k with
    rho_k <= tau ||e||.  RNS stops at the first k with
    |rho_{k-1} - rho_k| / rho_{k-1} < eps, with rho_0 = ||b - A x_0||.
  * The returned x is x_k at the stopping iteration (or at K).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import learned as lrn
from . import smallsolve as ss

STATUS_KMAX = 1
STATUS_STOP_DP = 2
STATUS_STOP_RNS = 4
STATUS_BREAKDOWN = 8
STATUS_NONFINITE = 16
STATUS_STOP_LEARNED = 32
STATUS_STOP_NCP = 64

NCP_KS = 1.36      # 5 % Kolmogorov-Smirnov band: +-1.36 / sqrt(q)

BREAKDOWN_TOL = 1e-14


@dataclass
class Result:
    x: np.ndarray
    iters: int
    status: int
    lam: list = field(default_factory=list)        # lam_k, k = 1..iters
    rho: list = field(default_factory=list)        # rho_k, k = 0..iters
    rho_hat: list = field(default_factory=list)    # projected residual, k = 1..iters
    sigma: np.ndarray | None = None                # singular values of H_iters
    H: np.ndarray | None = None                    # (iters+1) x iters
    W: np.ndarray | None = None                    # (iters+1) x len basis (rows)
    beta: float = 0.0
    xs: list = field(default_factory=list)         # x_k history when requested
    Mw_norms: list = field(default_factory=list)
    small: list = field(default_factory=list)      # per-iteration (sigma, uhat, u_{k+1}) when requested
    ncp: list = field(default_factory=list)        # NCP distance of r_k, k = 1..iters (stop "ncp")


def ncp_distance(r, det: int) -> float:
    """Distance of the residual's normalised cumulative periodogram (NCP) from
    that of white noise (Sec. 3.2; Hansen 2010).  r is read as rows of `det`
    detector bins (a sinogram); each row's periodogram |DFT|^2 at frequencies
    1..q = det // 2 (the mean excluded) is summed over the rows, the NCP is
    c_f = sum_{j<=f} P_j / sum_{j<=q} P_j, and the distance is
    max_f |c_f - f/q| (0 when the spectrum is empty)."""
    R = np.asarray(r, dtype=np.float64).reshape(-1, det)
    q = det // 2
    P = (np.abs(np.fft.fft(R, axis=1)) ** 2)[:, 1:q + 1].sum(axis=0)
    tot = float(P.sum())
    if q < 1 or tot == 0.0:
        return 0.0
    c = np.cumsum(P) / tot
    return float(np.max(np.abs(c - np.arange(1, q + 1) / q)))


def ncp_white(r, det: int) -> bool:
    """The NCP stopping test: the residual passes as white noise when its NCP
    stays within the 5 % Kolmogorov-Smirnov band around the straight line."""
    q = det // 2
    return q >= 1 and ncp_distance(r, det) <= NCP_KS / math.sqrt(q)


def hybrid_gmres(A, B, b, mode: str = "AB", K: int = 30, rule: str = "gcv",
                 lam: float = 0.0, stop: str | None = None, tau: float = 1.01,
                 noise_norm: float | None = None, rns_eps: float = 1e-3,
                 x0=None, ortho: str = "cgs2", keep_x: bool = False,
                 keep_basis: bool = False, keep_small: bool = False, mlp=None,
                 judge_delta: float = 0.05, det: int | None = None, learned_gate: float = 0.0) -> Result:
    """Run hybrid AB- or BA-GMRES for at most K iterations.

    A, B     -- callables on flat FP64 vectors (R^n -> R^m and R^m -> R^n)
    rule     -- lambda rule: "none", "fixed" (uses lam), "gcv", "dp", "lcurve",
                or "learned" (the network `mlp` proposes lambda, judged against
                GCV with margin judge_delta; see oracle.learned)
    stop     -- None (run K iterations), "dp", "rns", "ncp" (the residual,
                read as rows of `det` bins, passes the NCP white-noise test)
                or "learned" (the network's stop index, with the discrepancy
                principle first when noise_norm is given; with learned_gate
                c > 0 and noise_norm the stop index is accepted only once the
                data residual is within the factor c of tau ||e||)
    """
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    if x0 is None:
        # x_0 = B u_0 with u_0 = 0
        n = np.asarray(B(np.zeros_like(b))).size
        x0 = np.zeros(n)
    x0 = np.asarray(x0, dtype=np.float64).reshape(-1)
    Ax0 = np.asarray(A(x0)).reshape(-1)
    res0 = b - Ax0
    if mode == "AB":
        r0 = res0
    elif mode == "BA":
        r0 = np.asarray(B(res0)).reshape(-1)
    else:
        raise ValueError(mode)
    rho0 = float(np.linalg.norm(res0))
    beta = float(np.linalg.norm(r0))
    out = Result(x=x0.copy(), iters=0, status=0, rho=[rho0], beta=beta)
    if not np.all(np.isfinite(b)) or not math.isfinite(beta):
        out.status = STATUS_NONFINITE
        return out
    if beta == 0.0:
        out.status = STATUS_BREAKDOWN
        return out
    if rule == "learned" and mlp is None:
        raise ValueError("the learned rule needs the network parameters")
    if stop == "ncp" and not det:
        raise ValueError("the NCP test needs the detector row length det")
    if stop == "learned" and rule != "learned":
        raise ValueError("the learned stop shares the learned rule's network")
    gres = [beta]
    k_hat = float(K)
    if (rule == "dp" or stop == "dp") and noise_norm is None:
        raise ValueError("the discrepancy principle needs ||e||")
    target = None if noise_norm is None else tau * noise_norm

    W = [r0 / beta]
    H = np.zeros((K + 1, K))
    status = STATUS_KMAX
    k_done = 0
    x = x0.copy()

    def apply_M(w):
        if mode == "AB":
            return np.asarray(A(np.asarray(B(w)).reshape(-1))).reshape(-1)
        return np.asarray(B(np.asarray(A(w)).reshape(-1))).reshape(-1)

    if ortho == "dcgs2":
        # first pass of step 1: v = M w_1 - (w_1 . M w_1) w_1
        z = apply_M(W[0])
        H[0, 0] = float(np.dot(W[0], z))
        v = z - H[0, 0] * W[0]
    for k in range(1, K + 1):
        if ortho == "dcgs2":
            Wk = np.stack(W)                  # k x len
            z = apply_M(v)
            a, b_ = Wk @ v, Wk @ z
            gamma, delta = float(np.dot(v, v)), float(np.dot(v, z))
            H[:k, k - 1] += a
            hk = math.sqrt(max(gamma - float(np.dot(a, a)), 0.0))
            H[k, k - 1] = hk
            mw = float(np.linalg.norm(H[:k + 1, k - 1]))   # ||M w_k|| by the Arnoldi relation
            out.Mw_norms.append(mw)
            broke = hk <= BREAKDOWN_TOL * mw
            if broke:
                H[k, k - 1] = 0.0
            else:
                W.append((v - Wk.T @ a) / hk)
                if k < K:
                    t = H[:k + 1, :k] @ a
                    h1 = (np.append(b_, (delta - float(np.dot(a, b_))) / hk) - t) / hk
                    H[:k + 1, k] = h1
                    v = z / hk - np.stack(W).T @ (t / hk + h1)
        else:
            w = W[k - 1]
            q = apply_M(w)
            mw = float(np.linalg.norm(q))
            out.Mw_norms.append(mw)
        if ortho == "dcgs2":
            pass
        elif ortho == "cgs2":
            Wk = np.stack(W)                  # k x len
            h = Wk @ q
            q = q - Wk.T @ h
            c = Wk @ q
            q = q - Wk.T @ c
            H[:k, k - 1] = h + c
        elif ortho == "mgs":
            for i in range(k):
                H[i, k - 1] = float(np.dot(q, W[i]))
                q = q - H[i, k - 1] * W[i]
        else:
            raise ValueError(ortho)
        if ortho != "dcgs2":
            hk = float(np.linalg.norm(q))
            broke = hk <= BREAKDOWN_TOL * mw
            if broke:
                H[k, k - 1] = 0.0
            else:
                H[k, k - 1] = hk
                W.append(q / hk)
        Hk = H[:k + 1, :k]
        if rule == "learned":
            base = ss.solve_projected(Hk, beta, "gcv")
            gres.append(base["uk1"])
            f = lrn.features(base["sigma"], gres, None if noise_norm is None or rho0 <= 0.0 else noise_norm / rho0)
            lam_l, _, _, o1 = lrn.judge(mlp, f, base["sigma"], base["uhat"], base["uk1"], judge_delta)
            # the stop index: the largest prediction made so far
            k_new = min(max(K * o1, 1.0), float(K))
            k_hat = k_new if k == 1 else max(k_hat, k_new)
            sol = ss.solve_projected(Hk, beta, "fixed", lam_fixed=lam_l)
        else:
            sol = ss.solve_projected(Hk, beta, rule, lam_fixed=lam, dp_target=target)
        y = sol["y"]
        Wk = np.stack(W[:k])
        if mode == "AB":
            x = x0 + np.asarray(B(Wk.T @ y)).reshape(-1)
        else:
            x = x0 + Wk.T @ y
        rk = b - np.asarray(A(x)).reshape(-1)
        rho = float(np.linalg.norm(rk))
        out.lam.append(sol["lam"])
        out.rho.append(rho)
        out.rho_hat.append(sol["rho_hat"])
        out.sigma = sol["sigma"]
        if keep_x:
            out.xs.append(x.copy())
        if keep_small:
            out.small.append((sol["sigma"], sol["uhat"], sol["uk1"]))
        k_done = k
        if not (np.all(np.isfinite(x)) and math.isfinite(rho)):
            status = STATUS_NONFINITE
            break
        if broke:
            status = STATUS_BREAKDOWN
            break
        if (stop == "dp" or (stop == "learned" and target is not None)) and rho <= target:
            status = STATUS_STOP_DP
            break
        if stop == "rns" and abs(out.rho[-2] - rho) / out.rho[-2] < rns_eps:
            status = STATUS_STOP_RNS
            break
        if stop == "ncp":
            out.ncp.append(ncp_distance(rk, det))
            if ncp_white(rk, det):
                status = STATUS_STOP_NCP
                break
        if stop == "learned" and k >= k_hat and (learned_gate <= 0 or target is None
                                                 or rho <= learned_gate * target):
            status = STATUS_STOP_LEARNED
            break
    out.x = x
    out.iters = k_done
    out.status = status
    out.H = H[:k_done + 1, :k_done].copy()
    if keep_basis:
        out.W = np.stack(W)
    return out


def hybrid_gmres_restarted(A, B, b, p: int, mode: str = "AB", K: int = 30, rule: str = "gcv",
                           lam: float = 0.0, stop: str | None = None, tau: float = 1.01,
                           noise_norm: float | None = None, rns_eps: float = 1e-3, x0=None,
                           ortho: str = "cgs2", det: int | None = None) -> Result:
    """Restarted hybrid AB-/BA-GMRES (Sec. 3.3): cycles of at most p iterations,
    each started from the final iterate of the previous cycle, K iterations
    in all.  lambda and the stopping rule act on every iteration of every
    cycle; a cycle ended by a stopping rule, a breakdown or non-finite data
    ends the run.  Histories are concatenated: lam_k for k = 1..iters and
    rho_k for k = 0..iters, rho_0 of each cycle being the last rho of the
    previous one (the same data residual)."""
    if p < 1:
        raise ValueError("the cycle length p must be >= 1")
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    x = None if x0 is None else np.asarray(x0, dtype=np.float64).reshape(-1)
    lam_h, rho_h, done, status = [], None, 0, STATUS_KMAX
    out = None
    while done < K:
        pc = min(p, K - done)
        out = hybrid_gmres(A, B, b, mode=mode, K=pc, rule=rule, lam=lam, stop=stop, tau=tau,
                           noise_norm=noise_norm, rns_eps=rns_eps, x0=x, ortho=ortho, det=det)
        if rho_h is None:
            rho_h = [out.rho[0]]
        rho_h += out.rho[1:]
        lam_h += out.lam
        x = out.x
        done += out.iters
        if out.status != STATUS_KMAX:
            status = out.status
            break
    return Result(x=x, iters=done, status=status, lam=lam_h, rho=rho_h, beta=out.beta)
