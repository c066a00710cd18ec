"""FP64 operator wrappers over the oracle's plain-C definitions.

A is the forward projector of eq. (1); B the unmatched backprojector of
eqs. (4)-(5); At the exact transpose of A (the matched pair used for the
equivalences with LSQR / LSMR in Sec. 3).  Arrays may carry any number of
leading batch dimensions.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .build import load_oracle
from .geometry import Cone3D, Par2D

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _p(a):
    return a.ctypes.data_as(_dp)


def _pi(a):
    return a.ctypes.data_as(_ip)


class Par2DOps:
    """A, At and B for a 2D parallel-beam geometry."""

    def __init__(self, geom: Par2D):
        self.g = geom
        self.lib = load_oracle()
        self._cos = np.ascontiguousarray(geom.cos, dtype=np.float64)
        self._sin = np.ascontiguousarray(geom.sin, dtype=np.float64)
        self._rm = np.ascontiguousarray(geom.rowmarch, dtype=np.int32)

    @property
    def n(self):
        return self.g.n

    @property
    def m(self):
        return self.g.m

    def _img_in(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        lead = x.shape[:-2] if x.ndim >= 2 and x.shape[-2:] == (self.g.ny, self.g.nx) else x.shape[:-1]
        batch = int(np.prod(lead)) if lead else 1
        assert x.size == batch * self.g.n, "image size mismatch"
        return x.reshape(batch, self.g.n), lead

    def _sino_in(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        g = self.g
        lead = y.shape[:-2] if y.ndim >= 2 and y.shape[-2:] == (g.n_angles, g.n_det) else y.shape[:-1]
        batch = int(np.prod(lead)) if lead else 1
        assert y.size == batch * g.m, "sinogram size mismatch"
        return y.reshape(batch, g.m), lead

    def A(self, x):
        g = self.g
        xb, lead = self._img_in(x)
        y = np.zeros((xb.shape[0], g.m))
        self.lib.oracle_joseph2d(_p(xb), _p(y), xb.shape[0], g.nx, g.ny, g.n_angles, g.n_det,
                                 g.det_pitch, _p(self._cos), _p(self._sin), _pi(self._rm))
        return y.reshape(*lead, g.n_angles, g.n_det) if np.ndim(x) >= 2 else y.reshape(-1)

    def At(self, y):
        g = self.g
        yb, lead = self._sino_in(y)
        x = np.zeros((yb.shape[0], g.n))
        self.lib.oracle_joseph2d_t(_p(yb), _p(x), yb.shape[0], g.nx, g.ny, g.n_angles, g.n_det,
                                   g.det_pitch, _p(self._cos), _p(self._sin), _pi(self._rm))
        return x.reshape(*lead, g.ny, g.nx) if np.ndim(y) >= 2 else x.reshape(-1)

    def B(self, y):
        g = self.g
        yb, lead = self._sino_in(y)
        x = np.zeros((yb.shape[0], g.n))
        self.lib.oracle_pixbp2d(_p(yb), _p(x), yb.shape[0], g.nx, g.ny, g.n_angles, g.n_det,
                                g.det_pitch, _p(self._cos), _p(self._sin))
        return x.reshape(*lead, g.ny, g.nx) if np.ndim(y) >= 2 else x.reshape(-1)

    def explicit(self, which: str) -> np.ndarray:
        """Dense matrix of A ('A'), A^T ('At') or B ('B') by applying it to unit vectors."""
        g = self.g
        if which == "A":
            eye = np.eye(g.n).reshape(g.n, g.ny, g.nx)
            return self.A(eye).reshape(g.n, g.m).T.copy()
        eye = np.eye(g.m).reshape(g.m, g.n_angles, g.n_det)
        f = self.At if which == "At" else self.B
        return f(eye).reshape(g.m, g.n).T.copy()


class Cone3DOps:
    """A (Joseph, bilinear) and B (voxel driven, bilinear) for a cone beam."""

    def __init__(self, geom: Cone3D):
        self.g = geom
        self.lib = load_oracle()
        self._src = np.ascontiguousarray(geom.src)
        self._det = np.ascontiguousarray(geom.det)
        self._eu = np.ascontiguousarray(geom.eu)
        self._ev = np.ascontiguousarray(geom.ev)

    @property
    def n(self):
        return self.g.n

    @property
    def m(self):
        return self.g.m

    def A(self, x):
        g = self.g
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(g.n)
        y = np.zeros(g.m)
        self.lib.oracle_cone_fwd(_p(x), _p(y), g.nx, g.ny, g.nz, g.n_views, g.nu, g.nv,
                                 g.pu, g.pv, _p(self._src), _p(self._det), _p(self._eu), _p(self._ev))
        return y

    def B_points(self, y, idx):
        """(B y) at the flat voxel indices idx (the same sum as B)."""
        g = self.g
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(g.m)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.zeros(idx.size)
        self.lib.oracle_cone_bp_points(_p(y), idx.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), _p(out),
                                       idx.size, g.nx, g.ny, g.nz, g.n_views, g.nu, g.nv, g.pu, g.pv,
                                       _p(self._src), _p(self._det), _p(self._eu), _p(self._ev))
        return out

    def B(self, y):
        g = self.g
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(g.m)
        x = np.zeros(g.n)
        self.lib.oracle_cone_bp(_p(y), _p(x), g.nx, g.ny, g.nz, g.n_views, g.nu, g.nv,
                                g.pu, g.pv, _p(self._src), _p(self._det), _p(self._eu), _p(self._ev))
        return x


class FanFlat2DOps:
    """A (Joseph) and B (pixel driven, weight M / pu) of the 2D fan beam with a
    flat detector, over the plain-C definitions in projectors.c."""

    def __init__(self, geom):
        self.g = geom
        self.lib = load_oracle()
        self._src = np.ascontiguousarray(geom.src)
        self._det = np.ascontiguousarray(geom.det)
        self._eu = np.ascontiguousarray(geom.eu)

    @property
    def n(self):
        return self.g.n

    @property
    def m(self):
        return self.g.m

    def A(self, x):
        g = self.g
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(g.n)
        y = np.zeros(g.m)
        self.lib.oracle_fan_fwd(_p(x), _p(y), g.nx, g.ny, g.n_views, g.nu, g.pu, _p(self._src), _p(self._det),
                                _p(self._eu))
        return y

    def B(self, y):
        g = self.g
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(g.m)
        x = np.zeros(g.n)
        self.lib.oracle_fan_bp(_p(y), _p(x), g.nx, g.ny, g.n_views, g.nu, g.pu, _p(self._src), _p(self._det),
                               _p(self._eu))
        return x
