"""Host-side logic of the benchmark: the algorithmic work counts that the
roofline figures divide by.

The Joseph forward projector (Sec. 2, the ray-driven A) makes one
interpolation per row of the dominant axis that a ray crosses inside the
image.  The count is pinned by brute force on the oracle's explicit matrix:
for every ray, the number of distinct marched rows holding a non-zero entry.
"""
import numpy as np
import pytest

import bench


@pytest.mark.parametrize("n,na,nd", [(12, 10, 17), (9, 7, 13), (16, 12, 23)])
def test_joseph_ray_steps_brute_force(oracle_lib, n, na, nd):
    from oracle.geometry import Par2D
    from oracle.operators import Par2DOps
    g = Par2D(n, n, na, nd)
    M = Par2DOps(g).explicit("A").reshape(na, nd, n, n)  # [angle, bin, y, x]
    count = 0
    for a in range(na):
        for d in range(nd):
            nz = M[a, d] != 0
            rows = nz.any(axis=1) if g.rowmarch[a] else nz.any(axis=0)
            count += int(rows.sum())
    assert bench.joseph_ray_steps(n, na, nd) == count


def test_ray_steps_scale_like_the_mean_chord():
    # every ray through the disk crosses about (2 sqrt2 / pi) n rows on average
    n, na, nd = 256, 360, 363
    est = 2 * np.sqrt(2) / np.pi * n * n * na
    assert abs(bench.joseph_ray_steps(n, na, nd) / est - 1) < 0.02


def test_recorded_traffic_ignores_stale_summaries(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    f = tmp_path / "k_traffic.md"
    f.write_text("- source_digest = `deadbeef`\n- hbm_bytes_per_launch = 123.0\n")
    assert bench.recorded_traffic("k") is None
    f.write_text(f"- source_digest = `{bench.kernel_source_digest()}`\n- hbm_bytes_per_launch = 123.0\n")
    assert bench.recorded_traffic("k") == 123.0
    assert bench.recorded_issue("k") is None
    assert bench.recorded_traffic("absent") is None
    f.write_text(f"- source_digest = `{bench.kernel_source_digest()}`\n- hbm_bytes_per_launch = 123.0\n"
                 "- valu_instructions_per_launch = 2048\n- busy_cu_cycles_per_launch = 1024\n")
    assert bench.recorded_issue("k") == {"valu_instructions": 2048.0, "busy_cu_cycles": 1024.0,
                                         "cycles_per_valu_per_simd": 2.0}
    f.write_text("- source_digest = `deadbeef`\n- valu_instructions_per_launch = 2048\n"
                 "- busy_cu_cycles_per_launch = 1024\n")
    assert bench.recorded_issue("k") is None


@pytest.mark.parametrize("n,views,nu,nv,pitch,sid,sdd", [(8, 6, 12, 10, 1.0, 30.0, 60.0),
                                                         (10, 5, 14, 18, 1.5, 16.0, 26.0)])
def test_cone_ray_steps_brute_force(n, views, nu, nv, pitch, sid, sdd):
    # every ray, every plane of its dominant axis: count the planes where both
    # in-plane coordinates of the crossing lie in (-1, n)
    import math
    c = 0.5 * (n - 1)
    want = 0
    for v in range(views):
        b = 2 * math.pi * v / views
        S = (sid * math.cos(b), sid * math.sin(b), 0.0)
        for r in range(nv):
            for col in range(nu):
                ou, ov = (col - 0.5 * (nu - 1)) * pitch, (r - 0.5 * (nv - 1)) * pitch
                P = (-(sdd - sid) * math.cos(b) - ou * math.sin(b), -(sdd - sid) * math.sin(b) + ou * math.cos(b), ov)
                d = [P[t] - S[t] for t in range(3)]
                a = max(range(3), key=lambda t: (abs(d[t]), -t))
                for j in range(n):
                    t = ((j - c) - S[a]) / d[a]
                    crd = [S[o] + t * d[o] + c for o in range(3) if o != a]
                    want += all(-1 < q < n for q in crd)
    assert bench.cone_ray_steps(n, views, nu, nv, pitch, sid, sdd) == want


def test_dcgs2_byte_count():
    """The delayed-CGS2 byte count: steps j = 0..k_s per slice, each moving
    (j + 2) vectors in the dot-product sweep and (j + 4) in the update sweep
    (counted here step by step)."""
    import bench
    iters = [0, 1, 5, 100]
    length = 1000
    want = sum(sum((j + 2) + (j + 4) for j in range(k + 1)) for k in iters) * length * 4
    assert bench.dcgs2_bytes(iters, length) == want


def test_sub_batch_tuning_covers_every_sub_batch_size():
    """The sub-batches of S slices in p parts differ in size by at most one
    (the library's split); their projector launches are tuned at exactly
    those sizes, besides the whole batch and single slices."""
    calls = []

    class Stub:
        @staticmethod
        def autotune(op, batch):
            calls.append((op, batch))
            return {"batch": batch}

    for S, p, sizes in ((256, 3, {85, 86}), (256, 2, {128}), (7, 3, {2, 3}), (5, 9, set()), (256, 1, set()),
                        (4, 2, {2})):
        calls.clear()
        out = bench.tune_sub_batches(Stub, "A", "B", S, p)
        assert {b for _, b in calls} == sizes, (S, p)
        assert sorted(out) == sorted([f"A_sub{z}" for z in sizes] + [f"B_sub{z}" for z in sizes])
