"""A batch solved as concurrent sub-batches (exec.streams): each sub-batch of
consecutive slices on a stream and host thread of its own inside the library.
The slices are independent (Sec. 2: one reconstruction per slice), so every
output of every slice must equal, bit for bit, what the one-stream solve
gives: x, iterations, status, lambda and residual histories, NCP distances,
learned-rule features and RRE label grids, for both modes, the learned rule,
and restarted cycles; ragged splits (7 slices in 2 or 3 parts) included.
"""
import numpy as np
import pytest

import synth
from oracle.geometry import Par2D
from oracle.operators import Par2DOps

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2602_17892_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pk


@pytest.fixture(scope="module")
def batch(pk):
    n, na, nd, S = 96, 60, 137, 7
    g = pk.Geometry(n, n, na, nd)
    A = pk.Operator("joseph", g, "f32", "f32")
    B = pk.Operator("pixel", g, "f32", "f32")
    og = Par2DOps(Par2D(n, n, na, nd))
    bs, xs, ens = [], [], []
    for s in range(S):
        x, _ = synth.phantom2d(0, 10 + s, n)
        eta = 10 ** (-3 + 1.7 * s / (S - 1))
        b, en = synth.add_relative_noise(og.A(x).reshape(-1), synth.noise_direction(0, 10 + s, og.m), eta)
        bs.append(b)
        xs.append(x)
        ens.append(en)
    bd = torch.as_tensor(np.stack(bs), dtype=torch.float32, device="cuda").reshape(S, na, nd).contiguous()
    xt = torch.as_tensor(np.stack(xs), dtype=torch.float32, device="cuda").reshape(S, n, n).contiguous()
    en = torch.as_tensor(np.array(ens), dtype=torch.float64, device="cuda")
    return A, B, bd, xt, en


def same(a, b):
    """Bitwise equality of two result dicts (NaN entries, e.g. past a stop, equal too)."""
    for k in a:
        if a[k] is None:
            assert b[k] is None, k
            continue
        x, y = a[k], b[k]
        if x.dtype.is_floating_point:
            assert torch.equal(torch.nan_to_num(x, nan=1e300), torch.nan_to_num(y, nan=1e300)), k
        else:
            assert torch.equal(x, y), k


def run(pk, A, B, bd, streams, **kw):
    x, info = pk.solve(A, B, bd, streams=streams, **kw)
    torch.cuda.synchronize()
    out = {k: v for k, v in info.items() if k != "phase_ms"}
    out["x"] = x
    return out


@pytest.mark.parametrize("mode", ["AB", "BA"])
def test_streams_match_one_stream(pk, batch, mode):
    A, B, bd, xt, en = batch
    kw = dict(mode=mode, k=20, reg="gcv", tau=1.01, noise_norm=en, stop="dp", use_graph=True, poll_every=2,
              features=True)
    if mode == "AB":
        kw["x_true"] = xt
    ref = run(pk, A, B, bd, 1, **kw)
    its = ref["iters"].tolist()
    print(f"{mode}: iterations {its}")
    assert len(set(its)) > 1   # the slices stop at different iterations
    for st in (2, 3, 7, 9):
        same(ref, run(pk, A, B, bd, st, **kw))


def test_streams_learned_ncp_restart(pk, batch):
    A, B, bd, xt, en = batch
    mlp = torch.as_tensor(synth.mlp_init(0), dtype=torch.float32, device="cuda")
    for kw in (dict(mode="AB", k=20, reg="learned", mlp=mlp, noise_norm=en, stop="learned", features=True),
               dict(mode="AB", k=20, reg="gcv", stop="ncp"),
               dict(mode="BA", k=24, reg="gcv", noise_norm=en, stop="dp", restart=8)):
        ref = run(pk, A, B, bd, 1, **kw)
        for st in (2, 3):
            same(ref, run(pk, A, B, bd, st, **kw))


def test_streams_arguments(pk, batch):
    A, B, bd, xt, en = batch
    w1 = pk.workspace_bytes(A, B, 7, "AB", 20, stop="dp")
    w3 = pk.workspace_bytes(A, B, 7, "AB", 20, stop="dp", streams=3)
    parts = sum(-(-pk.workspace_bytes(A, B, c, "AB", 20, stop="dp") // 256) * 256 for c in (3, 2, 2))
    assert w3 == parts and w3 >= w1
    with pytest.raises(pk.AbbaError):
        pk.solve(A, B, bd, k=5, streams=2, phases=True)
    with pytest.raises(pk.AbbaError):
        pk.solve(A, B, bd, k=5, streams=-1)
    with pytest.raises(pk.AbbaError):   # a one-stream workspace is too small for three
        pk.solve(A, B, bd, k=20, noise_norm=en, stop="dp", streams=3,
                 workspace=torch.empty(w1 // 2, dtype=torch.uint8, device="cuda"))
