"""Host checks of two index arguments the 2D projector kernels rely on.

Both emulate the kernels' FP32 arithmetic exactly in numpy (IEEE single
precision, round to nearest even) and need no GPU.

* B (pixel-driven backprojector) fills the windows of a chunk of angles over
  one flat index e = al*W + c and recovers the angle as floor((e + 1/2) *
  fl(1/W)) in FP32.  This must equal e div W for every e < G*W <= 8192
  (the windows of one chunk fit in 64 KB of LDS as 8-byte pairs).
* A (Joseph forward projector) clamps a ray's coordinate once per band of
  H rows to [H-1-PAD, C+PAD-H-1] (PAD zeros on each side of a padded row).
  With |slope| <= 1 every tap of the band must then lie inside the padded row,
  and where the clamp moves the coordinate the taps before and after the clamp
  must all be pad zeros, so the band's sum equals that of the zero-extended
  rows.
"""
import numpy as np
import pytest

PAD = 16   # zeros on each side of a padded row (the library's constant)
H = 8      # rows per band (FP32 and FP64)


def test_flat_window_index_recovers_the_angle():
    e = np.arange(8192, dtype=np.int64)
    ef = e.astype(np.float32) + np.float32(0.5)
    for W in range(1, 8193):
        winv = np.float32(1.0) / np.float32(W)
        n = 8192 // W * W   # entries of the largest chunk that fits
        if n == 0:
            continue
        al = (ef[:n] * winv).astype(np.int64)   # truncation = floor (positive)
        assert np.array_equal(al, e[:n] // W), W


def fma32(a, b, c):
    """Correctly rounded FP32 fma: a*b is exact in FP64 for FP32 a and small
    integer b, the sum is exact in FP64 for the magnitudes used here, and one
    rounding to FP32 gives the fused result."""
    return (a.astype(np.float64) * b + c.astype(np.float64)).astype(np.float32)


@pytest.mark.parametrize("C", [1, 7, 64, 512, 1000])
def test_one_clamp_per_band_keeps_taps_in_the_padded_row(C):
    rng = np.random.default_rng(C)
    L = C + 2 * PAD
    n = 200_000
    slope = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    slope[:4] = np.float32([1.0, -1.0, 0.0, np.nextafter(np.float32(1.0), np.float32(0.0))])
    # band-start coordinates from far left of the image to far right of it
    ub = rng.uniform(-3.0 * C - 40, 4.0 * C + 40, n).astype(np.float32)
    lo, hi = np.float32(H - 1 - PAD), np.float32(L - PAD - H - 1)
    ubc = np.minimum(np.maximum(ub, lo), hi)
    moved = ubc != ub
    for q in range(H):
        u = fma32(-slope, float(q), ubc)
        idx = np.floor(u).astype(np.int64) + PAD   # entry of the left tap in the padded row
        assert idx.min() >= 0 and idx.max() <= L - 2
        # where the clamp moved the coordinate, both taps are pads, before and after
        def in_image(col):   # padded-row entry -> holds an image value?
            return (col >= PAD) & (col < PAD + C)
        u_true = fma32(-slope, float(q), ub)
        idx_true = np.floor(u_true).astype(np.int64) + PAD
        for i in (idx, idx_true):
            touched = in_image(i) | in_image(i + 1)
            assert not np.any(touched & moved)
    assert moved.any() and (~moved).any()
