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


# B's tile: 32 columns x 8*RM rows (the library's constants)
BT, RM = 32, 8


def window_extremes(nx, ny, na, nd, ds=1.0, angles=None):
    """For every tile and angle of B's launch, the smallest t - w0 and the
    largest floor(t - w0) over the tile's pixels, and the window length W the
    host picks.  The window start w0 comes from the operator's table (FP64
    from the FP32 cos/ds and sin/ds at the tile's corners); t - w0 is the
    kernel's FP32 arithmetic, monotone in each pixel coordinate (fma is
    monotone in its operands), so its extremes lie at the tile's corner
    pixels."""
    th = np.asarray(angles, dtype=np.float64) if angles is not None else np.arange(na) * np.pi / na
    cs, sn = np.cos(th), np.sin(th)
    BTY = 8 * RM
    W = int(np.ceil(np.max((BT - 1) * np.abs(cs) + (BTY - 1) * np.abs(sn)) / ds)) + 5
    cb = (cs / ds).astype(np.float32)[None, :]
    sb = (sn / ds).astype(np.float32)[None, :]
    f = np.float32
    cx, cy, cd = f(0.5) * f(nx - 1), f(0.5) * f(ny - 1), f(0.5 * (nd - 1))
    btx, bty = -(-nx // BT), -(-ny // BTY)
    tx, ty = np.meshgrid(np.arange(btx), np.arange(bty), indexing="ij")
    X0 = ((tx * BT).astype(np.float32) - cx).reshape(-1, 1)
    Y0 = ((ty * BTY).astype(np.float32) - cy).reshape(-1, 1)
    X1, Y1 = X0 + f(BT - 1), Y0 + f(BTY - 1)
    X0d, X1d, Y0d, Y1d = (v.astype(np.float64) for v in (X0, X1, Y0, Y1))
    cbd, sbd = cb.astype(np.float64), sb.astype(np.float64)
    tmin = (0.5 * (nd - 1) + np.minimum(X0d * cbd, X1d * cbd)) + np.minimum(Y0d * sbd, Y1d * sbd)
    w0 = np.floor(tmin).astype(np.int64) - 1
    par2 = cd - w0.astype(np.float32)
    lo, hi = None, None
    for X in (X0, X1):
        base = fma32(np.broadcast_to(X, par2.shape), cb.astype(np.float64), par2)
        for Y in (Y0, Y1):
            t = fma32(np.broadcast_to(Y, par2.shape), sb.astype(np.float64), base)
            lo = t if lo is None else np.minimum(lo, t)
            hi = t if hi is None else np.maximum(hi, t)
    return float(lo.min()), int(np.floor(hi).max()), W


@pytest.mark.parametrize("geom", [
    (512, 512, 720, 725, 1.0), (256, 256, 360, 363, 1.0), (96, 96, 60, 137, 1.0), (64, 64, 90, 91, 1.0),
    (128, 128, 180, 183, 1.0), (37, 50, 33, 71, 1.0), (30, 30, 40, 61, 0.7), (8, 8, 12, 13, 1.0),
    (512, 512, 720, 1024, 0.7), (1024, 1024, 900, 1449, 1.0)])
def test_backprojector_window_holds_every_tap(geom):
    """B reads entry floor(t - w0) of the window (the pair of taps
    floor(t - w0) and the next one) without a clamp: every pixel of a tile,
    its overhang included, must have t - w0 >= 0 (truncation is floor) and
    floor(t - w0) <= W - 1.  Checked with margins: t - w0 >= 0.99 and
    floor(t - w0) <= W - 4."""
    nx, ny, na, nd, ds = geom
    lo, hi, W = window_extremes(nx, ny, na, nd, ds)
    assert lo >= 0.99 and hi <= W - 4, (lo, hi, W)


def test_backprojector_window_holds_every_tap_at_uneven_angles():
    rng = np.random.default_rng(5)
    for _ in range(20):
        na = int(rng.integers(3, 200))
        angles = np.sort(rng.uniform(-np.pi, 2 * np.pi, na))
        nx, ny = (int(v) for v in rng.integers(5, 300, 2))
        nd = int(rng.integers(8, 500))
        ds = float(rng.uniform(0.4, 2.5))
        lo, hi, W = window_extremes(nx, ny, na, nd, ds, angles)
        assert lo >= 0.99 and hi <= W - 4, (nx, ny, na, nd, ds, lo, hi, W)


@pytest.mark.parametrize("ny", [1, 37, 64, 65, 512, 1000])
def test_backprojector_tile_rows_are_covered_once(ny):
    """B's workgroups over a tile of BTH = 64 rows: a whole tile (RM = 8 rows
    per thread, rows r + 8m for thread row r < 8) or one of two halves (RM = 4,
    rows 32 h + r + 8m).  Either way every image row is written by exactly one
    (workgroup, thread row, m), and by the same row index, so the two launch
    forms write the same pixels."""
    BTH = 64
    bty = -(-ny // BTH)
    for RM in (8, 4):
        NH = BTH // (8 * RM)
        rows = []
        for ty in range(bty):
            for half in range(NH):
                for r in range(8):
                    i0 = ty * BTH + half * (8 * RM) + r
                    rows += [i0 + 8 * m for m in range(RM) if i0 + 8 * m < ny]
        assert sorted(rows) == list(range(ny)), RM
