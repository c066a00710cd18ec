"""Geometry tables for the oracle (FP64), computed from their definitions.

2D parallel beam: angle a is t_a = a*pi/n_angles unless angles are given.
A ray marches over rows ("row-march") when |cos t| is the larger direction
cosine.  For the default uniform angles this is decided by the integer test
4a <= n_angles or 4a >= 3*n_angles, which resolves the 45-degree tie without
floating point; for user angles by |cos t| >= |sin t| in FP64.

3D circular cone beam: view v at beta_v = 2*pi*v/n_views (unless given);
source S = sid*(cos b, sin b, 0); flat detector centred at
D = -(sdd - sid)*(cos b, sin b, 0) with column axis eu = (-sin b, cos b, 0)
and row axis ev = (0, 0, 1).

2D fan beam, flat detector: the image plane of the cone geometry -- view v
at beta_v = 2*pi*v/n_views (unless given), source sid*(cos b, sin b),
detector centre -(sdd - sid)*(cos b, sin b), column axis (-sin b, cos b).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Par2D:
    nx: int
    ny: int
    n_angles: int
    n_det: int
    det_pitch: float = 1.0
    angles: np.ndarray | None = None
    cos: np.ndarray = field(init=False)
    sin: np.ndarray = field(init=False)
    rowmarch: np.ndarray = field(init=False)

    def __post_init__(self):
        na = self.n_angles
        if self.angles is None:
            a = np.arange(na)
            theta = a * math.pi / na
            self.cos = np.cos(theta)
            self.sin = np.sin(theta)
            self.rowmarch = ((4 * a <= na) | (4 * a >= 3 * na)).astype(np.int32)
        else:
            theta = np.asarray(self.angles, dtype=np.float64)
            assert theta.shape == (na,)
            self.cos = np.cos(theta)
            self.sin = np.sin(theta)
            self.rowmarch = (np.abs(self.cos) >= np.abs(self.sin)).astype(np.int32)

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def m(self) -> int:
        return self.n_angles * self.n_det


@dataclass
class Cone3D:
    nx: int
    ny: int
    nz: int
    n_views: int
    nu: int
    nv: int
    pu: float
    pv: float
    sid: float
    sdd: float
    angles: np.ndarray | None = None
    src: np.ndarray = field(init=False)
    det: np.ndarray = field(init=False)
    eu: np.ndarray = field(init=False)
    ev: np.ndarray = field(init=False)

    def __post_init__(self):
        if self.angles is None:
            beta = 2.0 * math.pi * np.arange(self.n_views) / self.n_views
        else:
            beta = np.asarray(self.angles, dtype=np.float64)
        c, s = np.cos(beta), np.sin(beta)
        z = np.zeros_like(c)
        self.src = np.stack([self.sid * c, self.sid * s, z], axis=1)
        self.det = np.stack([-(self.sdd - self.sid) * c, -(self.sdd - self.sid) * s, z], axis=1)
        self.eu = np.stack([-s, c, z], axis=1)
        self.ev = np.stack([z, z, np.ones_like(c)], axis=1)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def m(self) -> int:
        return self.n_views * self.nu * self.nv


@dataclass
class FanFlat2D:
    nx: int
    ny: int
    n_views: int
    nu: int
    pu: float
    sid: float
    sdd: float
    angles: np.ndarray | None = None
    src: np.ndarray = field(init=False)
    det: np.ndarray = field(init=False)
    eu: np.ndarray = field(init=False)

    def __post_init__(self):
        if self.angles is None:
            beta = 2.0 * math.pi * np.arange(self.n_views) / self.n_views
        else:
            beta = np.asarray(self.angles, dtype=np.float64)
        c, s = np.cos(beta), np.sin(beta)
        self.src = np.stack([self.sid * c, self.sid * s], axis=1)
        self.det = np.stack([-(self.sdd - self.sid) * c, -(self.sdd - self.sid) * s], axis=1)
        self.eu = np.stack([-s, c], axis=1)

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def m(self) -> int:
        return self.n_views * self.nu
