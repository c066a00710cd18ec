"""ORACLE (test infrastructure only): the learned lambda / stop-index model in FP64.

The paper chooses lambda by GCV, the discrepancy principle or the L-curve
(Sec. 3.1) and stops by DP, NCP or residual stagnation (Sec. 3.2).  This
module defines an optional learned alternative that keeps those rules as
fallback and judge:

* Features (64 per slice and iteration k), from quantities the method itself
  produces and that do not depend on any lambda choice:
    f[i],      i < 32: log10(sigma_(i) / sigma_(1)) for the singular values of
                       H_k sorted in decreasing order, -16 where i >= k or the
                       ratio is below 1e-16;
    f[32],             log10(||e|| / rho_0): the known noise norm relative to
                       the initial data residual rho_0 = ||b - A x_0|| (the
                       level the discrepancy principle stops at), -16 when
                       ||e|| is not given;
    f[32 + t], 1 <= t < 32: log10(r_j / r_0) with j = k - 31 + t, where r_j
                       is the plain GMRES residual of iteration j (the
                       component of beta e_1 outside range(H_j), eq. (9)) and
                       r_0 = beta; 0 where j < 1, -16 below 1e-16.
  All 64 values are scaled by 1/8 (to about [-2, 0]).
* Network: 64 -> 128 -> 128 -> 128 -> 2, ReLU after each hidden layer, linear
  output.  Parameters are one flat vector: W1 [128][64], b1 [128],
  W2 [128][128], b2, W3 [128][128], b3, W4 [2][128], b4 [2] (41,602 values).
* Outputs: o0 = log10(lam / sigma_1) / 8 and o1 = k_stop / K.
* Loss: mean over samples of the summed squared output error.
* Adam: Kingma and Ba (2015), Algorithm 1, with bias-corrected moments.
* Labels (AB mode, from the true image): for each iteration k and each lam on
  the grid lam_g = sigma_1 10^(-8 + 8 g / 63), g < 64, the relative error
  RRE_k(lam) = ||x_k(lam) - x_true|| / ||x_true||, x_k(lam) = x_0 + B W_k y_lam
  with y_lam the solution of eq. (12); lam*_k is the grid argmin (first index
  on ties) and k* the iteration of the smallest RRE_k(lam*_k).
* Judge: the predicted lam^ is used when GCV(lam^) <= (1 + delta) GCV(lam_GCV),
  else lam_GCV (eq. (15)); the run stops at the first k >= max_{j <= k} K o1(j),
  the largest stop prediction made so far (and earlier if the discrepancy
  principle fires).
"""
from __future__ import annotations

import math

import numpy as np

from . import smallsolve as ss

NF, NH, NO = 64, 128, 2
NSIG, NRES = 32, 32
PAD = -16.0
SCALE = 1.0 / 8.0
LGRID = 64
LAYERS = [(NH, NF), (NH, NH), (NH, NH), (NO, NH)]
N_PARAMS = sum(o * i + o for o, i in LAYERS)
# limits of the predicted log10(lam / sigma_1) (keeps lam^ finite and > 0)
LOG_LAM_MIN, LOG_LAM_MAX = -12.0, 4.0


def unpack(theta):
    """[(W, b)] views of the flat parameter vector, in layer order."""
    theta = np.asarray(theta)
    out, off = [], 0
    for o, i in LAYERS:
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    assert off == theta.size
    return out


def features(sigma, gres, noise_rel=None):
    """The 64 features of one slice at iteration k = len(sigma).

    sigma     -- singular values of H_k (any order)
    gres      -- [r_0, r_1, ..., r_k]: beta, then the GMRES residual of each iteration
    noise_rel -- ||e|| / ||b - A x_0||, or None when ||e|| is not known
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    k = sigma.size
    assert len(gres) == k + 1
    f = np.full(NF, 0.0)
    s = np.sort(sigma)[::-1]
    s1 = s[0] if k else 0.0
    for i in range(NSIG):
        v = PAD
        if i < k and s1 > 0.0 and s[i] > 0.0:
            v = max(math.log10(s[i] / s1), PAD)
        f[i] = v
    r0 = gres[0]
    for t in range(1, NRES):
        j = k - (NRES - 1) + t
        v = 0.0
        if j >= 1:
            v = math.log10(gres[j] / r0) if gres[j] > 0.0 else PAD
            v = max(v, PAD)
        f[NSIG + t] = v
    f[NSIG] = max(math.log10(noise_rel), PAD) if noise_rel is not None and noise_rel > 0.0 else PAD
    return f * SCALE


def forward(theta, X):
    """Y = net(X) for X [n][64]; also returns the activations."""
    X = np.asarray(X, dtype=np.float64)
    acts = [X]
    a = X
    layers = unpack(theta)
    for li, (W, b) in enumerate(layers):
        z = a @ W.T + b
        a = np.maximum(z, 0.0) if li < len(layers) - 1 else z
        acts.append(a)
    return a, acts


def loss_grad(theta, X, T):
    """L = (1/n) sum_s sum_o (Y_so - T_so)^2 and dL/dtheta (flat, same layout)."""
    T = np.asarray(T, dtype=np.float64)
    Y, acts = forward(theta, X)
    n = Y.shape[0]
    E = Y - T
    loss = float(np.sum(E * E) / n)
    layers = unpack(theta)
    grads = [None] * len(layers)
    d = 2.0 * E / n                             # dL/dz of the output layer
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a_in = acts[li]
        grads[li] = (d.T @ a_in, d.sum(axis=0))
        if li > 0:
            d = (d @ W) * (acts[li] > 0.0)      # through the ReLU of layer li-1's output
    flat = np.concatenate([np.concatenate([g.ravel(), gb]) for g, gb in grads])
    return loss, flat


def adam(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t >= 1): returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def lambda_grid(s1):
    return np.array([s1 * 10.0 ** (-8.0 + 8.0 * g / (LGRID - 1)) for g in range(LGRID)])


def rre_grid(B, H, beta, W, x0, x_true):
    """RRE_k(lam_g) for every k <= H.shape[1] (AB mode): [K][LGRID].

    y_lam is the least-squares solution of [H_k; lam I] y = [beta e_1; 0]
    (eq. (12)), computed directly (not through the SVD the solver uses), and
    x_k(lam) = x_0 + B(W_k^T y) by its definition.
    """
    K = H.shape[1]
    nt = float(np.linalg.norm(x_true))
    out = np.zeros((K, LGRID))
    for k in range(1, K + 1):
        Hk = H[:k + 1, :k]
        s1 = float(np.linalg.svd(Hk, compute_uv=False)[0])
        rhs = np.zeros(2 * k + 1)
        rhs[0] = beta
        for g, lam in enumerate(lambda_grid(s1)):
            M = np.vstack([Hk, lam * np.eye(k)])
            y = np.linalg.lstsq(M, rhs, rcond=None)[0]
            x = x0 + np.asarray(B(W[:k].T @ y)).reshape(-1)
            out[k - 1, g] = np.linalg.norm(x - x_true) / nt
    return out


def labels(rre, K):
    """Targets per iteration from an RRE grid [k][LGRID] of one run:
    [k][2] = (log10(lam*_k / sigma_1) / 8, k* / K), and k*."""
    g_star = np.argmin(rre, axis=1)                 # first index on ties
    best = rre[np.arange(rre.shape[0]), g_star]
    k_star = int(np.argmin(best)) + 1
    lg = -8.0 + 8.0 * g_star / (LGRID - 1)
    T = np.stack([lg * SCALE, np.full(rre.shape[0], k_star / K)], axis=1)
    return T, k_star


def judge(theta, f, sigma, uhat, uk1, delta):
    """The lambda the learned rule uses at one iteration, and the stop index.

    Returns (lam, lam_hat, accepted, k_hat) where k_hat = K-free o1 (the caller
    multiplies by K)."""
    y, _ = forward(theta, np.asarray(f)[None, :])
    o0, o1 = float(y[0, 0]), float(y[0, 1])
    s1 = float(np.max(sigma))
    lam_gcv = ss.choose_gcv(sigma, uhat, uk1)
    lg = min(max(o0 / SCALE, LOG_LAM_MIN), LOG_LAM_MAX)
    lam_hat = s1 * 10.0 ** lg
    ok = s1 > 0.0 and ss.gcv(lam_hat, sigma, uhat, uk1) <= (1.0 + delta) * ss.gcv(lam_gcv, sigma, uhat, uk1)
    return (lam_hat if ok else lam_gcv), lam_hat, ok, o1
