"""Pins of the learned lambda / stop-index oracle (oracle.learned).

* features: a hand-worked example (values computed by hand below);
* forward: weights chosen so that the network is a known affine map of the
  positive part of its input (closed form);
* backward: central finite differences of the forward (h = 1e-6);
* Adam: with a constant gradient the bias-corrected moments are exact, so
  every step moves each parameter by lr g / (|g| + eps) (Kingma and Ba 2015);
* RRE grid: lam -> x_k(lam) by a direct least-squares solve of eq. (12) and
  x = B W_k y, against the solver's own iterate at the same fixed lambda
  (SVD route) and the plain GMRES iterate at tiny lambda;
* labels: argmin bookkeeping on a constructed grid;
* the learned solve: with the judge never accepting it equals the GCV run,
  and a constant stop output stops at ceil(K o1).
"""
import math

import numpy as np
import pytest

from oracle import learned as L
from oracle import smallsolve as ss
from oracle import solver as osv
from oracle.geometry import Par2D
from oracle.operators import Par2DOps

pytestmark = pytest.mark.usefixtures("oracle_lib")


def rand_theta(seed, scale=1.0):
    r = np.random.default_rng(seed)
    parts = []
    for o, i in L.LAYERS:
        parts.append(r.standard_normal(o * i) * scale * math.sqrt(2.0 / i))
        parts.append(r.standard_normal(o) * 0.1)
    return np.concatenate(parts)


def test_parameter_count():
    assert L.N_PARAMS == 41602


def test_features_hand_example():
    f = L.features([0.5, 2.0, 0.02], [4.0, 2.0, 0.4, 0.04])
    want = np.full(64, -2.0)
    want[0], want[1], want[2] = 0.0, math.log10(0.25) / 8, -2.0 / 8
    want[33:] = 0.0
    want[32] = -2.0                       # no noise norm given
    want[61], want[62], want[63] = math.log10(0.5) / 8, -1.0 / 8, -2.0 / 8
    assert np.allclose(f, want, rtol=0, atol=1e-15)
    # with ||e|| = 1 % of the initial data residual only feature 32 changes
    g = L.features([0.5, 2.0, 0.02], [4.0, 2.0, 0.4, 0.04], noise_rel=0.01)
    want[32] = -2.0 / 8
    assert np.allclose(g, want, rtol=0, atol=1e-15)
    assert L.features([1.0], [1.0, 0.5], noise_rel=1e-20)[32] == -2.0   # clamped at -16 / 8


def test_features_padding_and_zeros():
    f = L.features([3.0, 0.0], [1.0, 0.0, 1e-20])
    assert f[0] == 0.0 and f[1] == -2.0 and np.all(f[2:32] == -2.0)
    assert f[62] == -2.0 and f[63] == -2.0 and np.all(f[33:62] == 0.0) and f[32] == -2.0
    # more than 32 iterations: only the 32 largest sigma and the last 32 residuals
    k = 40
    sig = 2.0 ** -np.arange(k)
    g = [1.0] + [10.0 ** -(j / 10) for j in range(1, k + 1)]
    f = L.features(sig[::-1], g)
    assert np.allclose(f[:32] * 8, np.log10(2.0 ** -np.arange(32)))
    assert np.allclose(f[33:] * 8, [-(j / 10) for j in range(10, 41)])


def test_forward_closed_form():
    theta = np.zeros(L.N_PARAMS)
    (W1, b1), (W2, b2), (W3, b3), (W4, b4) = L.unpack(theta)
    W1[:64, :64] = np.eye(64)
    W2[:] = np.eye(128)
    W3[:] = np.eye(128)
    W4[0, :64] = 1.0
    W4[1, :64] = np.arange(64)
    b4[:] = [1.0, -1.0]
    X = np.random.default_rng(1).standard_normal((5, 64))
    Y, _ = L.forward(theta, X)
    P = np.maximum(X, 0.0)
    assert np.allclose(Y[:, 0], 1.0 + P.sum(1), rtol=1e-14)
    assert np.allclose(Y[:, 1], -1.0 + P @ np.arange(64), rtol=1e-14)


def test_gradient_matches_central_differences():
    theta = rand_theta(3)
    r = np.random.default_rng(4)
    X = r.standard_normal((6, 64))
    T = r.standard_normal((6, 2))
    loss, g = L.loss_grad(theta, X, T)
    Y, _ = L.forward(theta, X)
    assert abs(loss - np.sum((Y - T) ** 2) / 6) <= 1e-14 * loss
    h = 1e-6
    idx = r.choice(L.N_PARAMS, 400, replace=False)
    # every bias and the last layer completely, plus a sample of the rest
    off, extra = 0, []
    for o, i in L.LAYERS:
        extra += list(range(off + o * i, off + o * i + o))
        off += o * i + o
    idx = np.unique(np.concatenate([idx, extra, np.arange(L.N_PARAMS - 258, L.N_PARAMS)]))
    fd = np.empty(idx.size)
    for n, p in enumerate(idx):
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd[n] = (L.loss_grad(tp, X, T)[0] - L.loss_grad(tm, X, T)[0]) / (2 * h)
    err = np.abs(fd - g[idx])
    assert np.max(err) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_adam_constant_gradient_steps():
    r = np.random.default_rng(5)
    theta0 = r.standard_normal(50)
    g = r.standard_normal(50)
    g[3] = 0.0
    m, v, th = np.zeros(50), np.zeros(50), theta0.copy()
    lr, eps = 1e-3, 1e-8
    for t in range(1, 6):
        th, m, v = L.adam(th, g, m, v, t, lr, eps=eps)
    want = theta0 - 5 * lr * g / (np.abs(g) + eps)
    assert np.allclose(th, want, rtol=0, atol=1e-15)
    assert th[3] == theta0[3]


def small_problem(n=16, na=20, seed=0, eta=0.01):
    og = Par2DOps(Par2D(n, n, na, 23))
    r = np.random.default_rng(seed)
    x = np.zeros((n, n))
    x[4:11, 3:9] = 1.0
    x[7:13, 9:14] = 0.5
    x = x.ravel()
    bt = og.A(x)
    b = bt + eta * np.linalg.norm(bt) / math.sqrt(bt.size) * r.standard_normal(bt.size)
    return og, x, b


def test_rre_grid_against_the_solver_iterates():
    og, xt, b = small_problem()
    K = 8
    o = osv.hybrid_gmres(og.A, og.B, b, mode="AB", K=K, rule="none", keep_basis=True, keep_x=True)
    grid = L.rre_grid(og.B, o.H, o.beta, o.W, np.zeros_like(xt), xt)
    nt = np.linalg.norm(xt)
    for k in (1, 4, K):
        # tiny lambda: the plain GMRES iterate
        assert abs(grid[k - 1, 0] - np.linalg.norm(o.xs[k - 1] - xt) / nt) <= 1e-6
        # a grid lambda: the solver run with that lambda fixed (SVD route)
        s1 = float(np.linalg.svd(o.H[:k + 1, :k], compute_uv=False)[0])
        for g in (20, 45, 63):
            lam = L.lambda_grid(s1)[g]
            of = osv.hybrid_gmres(og.A, og.B, b, mode="AB", K=k, rule="fixed", lam=lam)
            assert abs(grid[k - 1, g] - np.linalg.norm(of.x - xt) / nt) <= 1e-10


def test_labels_bookkeeping():
    K = 10
    kk, gg = np.meshgrid(np.arange(1, K + 1), np.arange(L.LGRID), indexing="ij")
    rre = (gg - 10 - kk) ** 2 + 0.5 * (kk - 3) ** 2 + 1.0
    T, k_star = L.labels(rre, K)
    assert k_star == 3
    g_star = 10 + np.arange(1, K + 1)
    assert np.allclose(T[:, 0], (-8 + 8 * g_star / 63) / 8)
    assert np.all(T[:, 1] == 0.3)


def test_learned_solve_falls_back_to_gcv_and_stops_at_k_hat():
    og, xt, b = small_problem(seed=2)
    theta = np.zeros(L.N_PARAMS)
    (_, _), (_, _), (_, _), (_, b4) = L.unpack(theta)
    b4[:] = [-0.25, 0.3]
    K = 20
    # delta = -1: the judge never accepts, so lambda is GCV's; stop at ceil(0.3 K) = 6
    ol = osv.hybrid_gmres(og.A, og.B, b, mode="AB", K=K, rule="learned", stop="learned", mlp=theta,
                          judge_delta=-1.0)
    og6 = osv.hybrid_gmres(og.A, og.B, b, mode="AB", K=6, rule="gcv")
    assert ol.iters == 6 and ol.status == osv.STATUS_STOP_LEARNED
    assert np.array_equal(ol.x, og6.x) and ol.lam == og6.lam
    # a huge margin: lambda^ = sigma_1 10^-2 always
    oh = osv.hybrid_gmres(og.A, og.B, b, mode="AB", K=4, rule="learned", mlp=theta, judge_delta=1e300)
    for k in range(1, 5):
        s1 = float(np.linalg.svd(oh.H[:k + 1, :k], compute_uv=False)[0])
        assert abs(oh.lam[k - 1] - 1e-2 * s1) <= 1e-13 * s1


def test_judge_accepts_within_margin():
    sig = np.array([3.0, 1.0, 0.2, 0.01])
    uh = np.array([1.0, -0.5, 0.3, 0.2])
    uk1 = 0.05
    lg = ss.choose_gcv(sig, uh, uk1)
    theta = np.zeros(L.N_PARAMS)
    b4 = L.unpack(theta)[3][1]
    b4[0] = math.log10(lg / 3.0) / 8 + 0.05       # a little off the GCV minimum
    lam, lam_hat, ok, _ = L.judge(theta, np.zeros(64), sig, uh, uk1, 1.0)
    assert ok and lam == lam_hat and abs(lam_hat / lg - 10 ** 0.4) < 1e-12
    lam, lam_hat, ok, _ = L.judge(theta, np.zeros(64), sig, uh, uk1, 0.0)
    assert not ok and lam == lg


def test_learned_stop_index_is_the_running_maximum():
    """The learned stop fires at the first k >= max_{j <= k} K o1(j): with a
    network whose stop prediction falls as the residual falls, the run goes on
    past the iterations at which k >= K o1(k) alone would have stopped it."""
    og, xt, b = small_problem(seed=3)
    theta = np.zeros(L.N_PARAMS)
    (W1, _), (W2, _), (W3, _), (W4, b4) = L.unpack(theta)
    W1[0, 63] = -1.0          # h = relu(-f_63) with f_63 = log10(r_k / r_0) / 8 <= 0
    W2[0, 0] = 1.0
    W3[0, 0] = 1.0
    W4[1, 0] = -4.0           # o1 = 0.6 - 4 h falls with the residual
    b4[:] = [-0.25, 0.6]
    K = 20
    o = osv.hybrid_gmres(og.A, og.B, b, mode="AB", K=K, rule="learned", stop="learned", mlp=theta,
                         judge_delta=-1.0, keep_small=True)
    # the predictions from the run's own small-solve quantities
    gres = [float(np.linalg.norm(b))] + [sm[2] for sm in o.small]
    preds = []
    for j, sm in enumerate(o.small, start=1):
        y, _ = L.forward(theta, L.features(sm[0], gres[:j + 1])[None, :])
        preds.append(min(max(K * float(y[0, 1]), 1.0), float(K)))
    k_rm = next(k for k in range(1, len(preds) + 1) if k >= max(preds[:k]))
    k_pt = next(k for k in range(1, len(preds) + 1) if k >= preds[k - 1])
    assert o.status == osv.STATUS_STOP_LEARNED and o.iters == k_rm
    assert k_pt < k_rm and preds[0] > preds[-1]
