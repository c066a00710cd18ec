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
    assert bench.recorded_traffic("absent") is None
