"""Python binding of libabba.so: hybrid AB-/BA-GMRES for CT on MI355X (gfx950).

The binding only marshals arguments: every step of the method runs in the
HIP kernels of libabba.so.  PyTorch supplies device memory and the current
HIP stream.  Importing this module fails loudly if the library is not built
(``python paper_2602_17892_amd/build.py``).

Low-level names mirror the C ABI (include/abba.h): abba_op_create,
abba_project, abba_backproject, abba_solve_workspace, abba_solve, ...
The helpers ``Operator``, ``project``, ``backproject`` and ``solve`` wrap
them for torch tensors.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

__all__ = [
    "LIB_PATH", "lib", "AbbaError", "Geometry", "Operator", "project", "backproject", "solve",
    "workspace_bytes", "project_workspace_bytes", "backproject_workspace_bytes", "project_noalloc",
    "mlp_loss_grad_workspace_bytes", "solve_layout", "basis_views", "ST_KMAX", "ST_STOP_DP", "ST_STOP_RNS", "ST_BREAKDOWN", "ST_NONFINITE",
    "ST_STOP_LEARNED", "ST_STOP_NCP", "autotune", "set_tuning", "get_tuning", "mlp_forward", "mlp_loss_grad", "mlp_adam", "mlp_labels", "MLP_PARAMS",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libabba.so")

# enums of include/abba.h
F64, F32, BF16 = 0, 1, 2
GEOM_PAR2D, GEOM_CONE3D, GEOM_FAN2D = 0, 1, 2
OP_JOSEPH, OP_PIXEL, OP_JOSEPH_T = 0, 1, 2
MODE_AB, MODE_BA = 0, 1
REG = {"none": 0, "fixed": 1, "gcv": 2, "dp": 3, "lcurve": 4, "learned": 5}
STOP = {None: 0, "none": 0, "dp": 1, "rns": 2, "learned": 3, "ncp": 4}
ST_KMAX, ST_STOP_DP, ST_STOP_RNS, ST_BREAKDOWN, ST_NONFINITE, ST_STOP_LEARNED = 1, 2, 4, 8, 16, 32
ST_STOP_NCP = 64


class AbbaError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib.abba_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib.abba_status_str(status).decode()} ({status}): {msg}")


class _Geometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("n_angles", ctypes.c_int), ("det_u", ctypes.c_int), ("det_v", ctypes.c_int),
                ("det_pitch_u", ctypes.c_double), ("det_pitch_v", ctypes.c_double),
                ("sid", ctypes.c_double), ("sdd", ctypes.c_double),
                ("angles", ctypes.POINTER(ctypes.c_double))]


class _Reg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("lam", ctypes.c_double), ("tau", ctypes.c_double),
                ("noise_norm", ctypes.c_void_p), ("mlp", ctypes.c_void_p), ("judge_delta", ctypes.c_double)]


class _Stop(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("tau", ctypes.c_double), ("rns_eps", ctypes.c_double),
                ("noise_norm", ctypes.c_void_p), ("learned_gate", ctypes.c_double)]


class _Out(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_void_p), ("status", ctypes.c_void_p), ("lam", ctypes.c_void_p),
                ("resid", ctypes.c_void_p), ("features", ctypes.c_void_p), ("x_true", ctypes.c_void_p),
                ("ncp", ctypes.c_void_p), ("rre", ctypes.c_void_p)]


class _Tune(ctypes.Structure):
    _fields_ = [("a_path", ctypes.c_int), ("a_jb", ctypes.c_int), ("b_g", ctypes.c_int), ("czt", ctypes.c_int),
                ("a_rb", ctypes.c_int), ("a_occ", ctypes.c_int), ("ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("candidates", ctypes.c_int), ("a_tile", ctypes.c_int), ("a_vg", ctypes.c_int)]


class _Layout(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_size_t), ("basis", ctypes.c_size_t), ("hessenberg", ctypes.c_size_t),
                ("singular_values", ctypes.c_size_t), ("ldw", ctypes.c_int64), ("len", ctypes.c_int64), ("basis_dtype", ctypes.c_int),
                ("basis_slots", ctypes.c_int), ("k", ctypes.c_int)]


class _Exec(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int), ("poll_every", ctypes.c_int), ("restart", ctypes.c_int),
                ("features", ctypes.c_int), ("ortho", ctypes.c_int), ("phase_ms", ctypes.c_void_p),
                ("streams", ctypes.c_int)]


# phases timed by abba_exec.phase_ms
PHASES = ("A", "B", "ortho", "small", "other")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2602_17892_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i = ctypes.c_void_p, ctypes.c_int
    L.abba_version.restype = ctypes.c_char_p
    L.abba_last_error.restype = ctypes.c_char_p
    L.abba_status_str.restype = ctypes.c_char_p
    L.abba_status_str.argtypes = [i]
    L.abba_op_create.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(_Geometry), i, i]
    L.abba_op_create.restype = i
    L.abba_op_destroy.argtypes = [vp]
    L.abba_op_destroy.restype = None
    L.abba_op_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.abba_op_sizes.restype = i
    sz, szp = ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)
    L.abba_project_workspace.argtypes = [vp, i, szp]
    L.abba_project_workspace.restype = i
    L.abba_backproject_workspace.argtypes = [vp, i, szp]
    L.abba_backproject_workspace.restype = i
    L.abba_project.argtypes = [vp, vp, vp, i, vp, sz, vp]
    L.abba_project.restype = i
    L.abba_backproject.argtypes = [vp, vp, vp, i, vp, sz, vp]
    L.abba_backproject.restype = i
    L.abba_project_noalloc.argtypes = [vp, vp, vp, i, vp]
    L.abba_project_noalloc.restype = i
    L.abba_autotune_workspace.argtypes = [vp, i, szp]
    L.abba_autotune_workspace.restype = i
    L.abba_mlp_loss_grad_workspace.argtypes = [i, szp]
    L.abba_mlp_loss_grad_workspace.restype = i
    L.abba_solve_workspace.argtypes = [vp, vp, i, i, i, ctypes.POINTER(_Stop), ctypes.POINTER(_Exec),
                                       ctypes.POINTER(ctypes.c_size_t)]
    L.abba_solve_workspace.restype = i
    L.abba_solve_layout.argtypes = [vp, vp, i, i, i, ctypes.POINTER(_Stop), ctypes.POINTER(_Exec),
                                    ctypes.POINTER(_Layout)]
    L.abba_solve_layout.restype = i
    L.abba_solve.argtypes = [vp, vp, vp, vp, i, i, i, ctypes.POINTER(_Reg), ctypes.POINTER(_Stop),
                             ctypes.POINTER(_Out), ctypes.POINTER(_Exec), vp, ctypes.c_size_t, vp]
    L.abba_solve.restype = i
    L.abba_autotune.argtypes = [vp, i, i, vp, sz, vp, ctypes.POINTER(_Tune)]
    L.abba_autotune.restype = i
    L.abba_op_set_tuning.argtypes = [vp, i, ctypes.POINTER(_Tune)]
    L.abba_op_set_tuning.restype = i
    L.abba_op_get_tuning.argtypes = [vp, i, ctypes.POINTER(_Tune)]
    L.abba_op_get_tuning.restype = i
    L.abba_mlp_forward.argtypes = [vp, vp, i, vp, vp]
    L.abba_mlp_forward.restype = i
    L.abba_mlp_loss_grad.argtypes = [vp, vp, vp, i, vp, i, vp, vp, vp, sz, vp]
    L.abba_mlp_loss_grad.restype = i
    L.abba_mlp_adam.argtypes = [vp, vp, vp, vp, i, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, vp]
    L.abba_mlp_adam.restype = i
    L.abba_mlp_labels.argtypes = [vp, i, i, vp, vp, vp, vp]
    L.abba_mlp_labels.restype = i
    return L


lib = _load()

# C-ABI names, re-exported
abba_version = lib.abba_version
abba_last_error = lib.abba_last_error
abba_status_str = lib.abba_status_str
abba_op_create = lib.abba_op_create
abba_op_destroy = lib.abba_op_destroy
abba_op_sizes = lib.abba_op_sizes
abba_project = lib.abba_project
abba_backproject = lib.abba_backproject
abba_project_noalloc = lib.abba_project_noalloc
abba_project_workspace = lib.abba_project_workspace
abba_backproject_workspace = lib.abba_backproject_workspace
abba_autotune_workspace = lib.abba_autotune_workspace
abba_mlp_loss_grad_workspace = lib.abba_mlp_loss_grad_workspace
abba_solve_workspace = lib.abba_solve_workspace
abba_solve = lib.abba_solve
abba_solve_layout = lib.abba_solve_layout
abba_autotune = lib.abba_autotune
abba_op_set_tuning = lib.abba_op_set_tuning
abba_op_get_tuning = lib.abba_op_get_tuning
abba_mlp_forward = lib.abba_mlp_forward
abba_mlp_loss_grad = lib.abba_mlp_loss_grad
abba_mlp_adam = lib.abba_mlp_adam
abba_mlp_labels = lib.abba_mlp_labels

MLP_FEATURES, MLP_PARAMS, LABEL_GRID = 64, 41602, 64
FEAT_OUT, FEAT_LABELS = 1, 2


def _check(rc, where):
    if rc != 0:
        raise AbbaError(rc, where)


@dataclass
class Geometry:
    """Scan geometry (see include/abba.h for the conventions)."""
    nx: int
    ny: int
    n_angles: int
    det_u: int
    det_pitch_u: float = 1.0
    kind: str = "par2d"
    nz: int = 1
    det_v: int = 1
    det_pitch_v: float = 1.0
    sid: float = 0.0
    sdd: float = 0.0
    angles: object = None

    def _c(self):
        g = _Geometry()
        g.kind = {"par2d": GEOM_PAR2D, "cone3d": GEOM_CONE3D, "fan2d": GEOM_FAN2D}[self.kind]
        g.nx, g.ny, g.nz = self.nx, self.ny, self.nz
        g.n_angles, g.det_u, g.det_v = self.n_angles, self.det_u, self.det_v
        g.det_pitch_u, g.det_pitch_v = self.det_pitch_u, self.det_pitch_v
        g.sid, g.sdd = self.sid, self.sdd
        keep = None
        if self.angles is not None:
            keep = (ctypes.c_double * self.n_angles)(*[float(a) for a in self.angles])
            g.angles = ctypes.cast(keep, ctypes.POINTER(ctypes.c_double))
        return g, keep

    @property
    def image_shape(self):
        return (self.nz, self.ny, self.nx) if self.kind == "cone3d" else (self.ny, self.nx)

    @property
    def sino_shape(self):
        return (self.n_angles, self.det_v, self.det_u) if self.kind == "cone3d" else (self.n_angles, self.det_u)


_DT = {"f64": F64, "f32": F32, "bf16": BF16}


def _torch_dtype(code):
    import torch
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}[code]


class Operator:
    """A projector handle: kind 'joseph' (A), 'pixel' (unmatched B) or 'joseph_t' (exact A^T)."""

    _KINDS = {"joseph": OP_JOSEPH, "pixel": OP_PIXEL, "joseph_t": OP_JOSEPH_T}

    def __init__(self, kind: str, geom: Geometry, img: str = "f32", sino: str = "f32"):
        self.geom = geom
        self.kind = kind
        self.img_dt, self.sino_dt = _DT[img], _DT[sino]
        g, keep = geom._c()
        h = ctypes.c_void_p()
        _check(lib.abba_op_create(ctypes.byref(h), self._KINDS[kind], ctypes.byref(g), self.img_dt,
                                  self.sino_dt), "abba_op_create")
        del keep
        self.handle = h
        n, m = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.abba_op_sizes(h, ctypes.byref(n), ctypes.byref(m)), "abba_op_sizes")
        self.n, self.m = n.value, m.value

    @property
    def img_dtype(self):
        return _torch_dtype(self.img_dt)

    @property
    def sino_dtype(self):
        return _torch_dtype(self.sino_dt)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:
            lib.abba_op_destroy(h)
            self.handle = None


def _stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, numel, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() % numel:
        raise ValueError(f"{name} has {t.numel()} elements, not a multiple of {numel}")
    return t.numel() // numel


def _need_exact(t, dtype, numel, name):
    _need(t, dtype, 1, name)
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def _bytes(fn, *a) -> int:
    nb = ctypes.c_size_t()
    _check(fn(*a, ctypes.byref(nb)), fn.__name__)
    return nb.value


def project_workspace_bytes(A: Operator, batch: int) -> int:
    """Device scratch bytes abba_project needs for `batch` slices."""
    return _bytes(lib.abba_project_workspace, A.handle, int(batch))


def backproject_workspace_bytes(B: Operator, batch: int) -> int:
    """Device scratch bytes abba_backproject needs for `batch` slices."""
    return _bytes(lib.abba_backproject_workspace, B.handle, int(batch))


def _workspace(nbytes, workspace, device):
    """The caller's workspace tensor (checked), or a new one from torch's
    allocator when none is given; None when nothing is needed."""
    import torch
    if workspace is None:
        return torch.empty(nbytes, dtype=torch.uint8, device=device) if nbytes else None
    if not workspace.is_cuda or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 device tensor")
    return workspace


def _wsptr(ws):
    return (None, 0) if ws is None else (_ptr(ws), ws.numel())


def project(A: Operator, x, out=None, workspace=None):
    """y = A x (batched over leading dimensions).  workspace: a uint8 device
    tensor of at least project_workspace_bytes(A, batch) bytes, or None for
    one from torch's allocator."""
    import torch
    batch = _need(x, A.img_dtype, A.n, "x")
    if out is None:
        out = torch.empty((batch, *A.geom.sino_shape), dtype=A.sino_dtype, device=x.device)
    _need_exact(out, A.sino_dtype, batch * A.m, "out")
    ws = _workspace(project_workspace_bytes(A, batch), workspace, x.device)
    _check(lib.abba_project(A.handle, _ptr(x), _ptr(out), batch, *_wsptr(ws), _stream_ptr()), "abba_project")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def project_noalloc(A: Operator, x, out):
    """y = A x through abba_project_noalloc: no workspace and no allocation in
    the call (the caller passes `out`); its scratch is the library's static
    device buffer of NOALLOC_SCRATCH_BYTES, shared by every such call on the
    device."""
    batch = _need(x, A.img_dtype, A.n, "x")
    _need_exact(out, A.sino_dtype, batch * A.m, "out")
    _check(lib.abba_project_noalloc(A.handle, _ptr(x), _ptr(out), batch, _stream_ptr()), "abba_project_noalloc")
    return out


def backproject(B: Operator, y, out=None, workspace=None):
    """x = B y (batched over leading dimensions); workspace as for project."""
    import torch
    batch = _need(y, B.sino_dtype, B.m, "y")
    if out is None:
        out = torch.empty((batch, *B.geom.image_shape), dtype=B.img_dtype, device=y.device)
    _need_exact(out, B.img_dtype, batch * B.n, "out")
    ws = _workspace(backproject_workspace_bytes(B, batch), workspace, y.device)
    _check(lib.abba_backproject(B.handle, _ptr(y), _ptr(out), batch, *_wsptr(ws), _stream_ptr()),
           "abba_backproject")
    return out


def _tune_dict(t):
    return dict(a_path=t.a_path, a_jb=t.a_jb, b_g=t.b_g, czt=t.czt, a_rb=t.a_rb, a_occ=t.a_occ, a_tile=t.a_tile,
                a_vg=t.a_vg)


def autotune(op: Operator, batch: int, reps: int = 3, workspace=None):
    """Time the launch choices of `op` at `batch` and keep the fastest for that
    batch size (abba_autotune).  Returns the choice with its time and the
    built-in rules' time in ms."""
    import torch
    t = _Tune()
    ws = _workspace(_bytes(lib.abba_autotune_workspace, op.handle, int(batch)), workspace,
                    torch.device("cuda", torch.cuda.current_device()))
    _check(lib.abba_autotune(op.handle, int(batch), int(reps), *_wsptr(ws), _stream_ptr(), ctypes.byref(t)),
           "abba_autotune")
    return dict(_tune_dict(t), ms=t.ms, default_ms=t.default_ms, candidates=t.candidates)


def set_tuning(op: Operator, batch: int, a_path=-1, a_jb=0, b_g=0, czt=0, a_rb=0, a_occ=0, a_tile=0, a_vg=0,
               clear=False):
    """Fix the launch choices of `op` for `batch` (clear=True forgets them)."""
    if clear:
        _check(lib.abba_op_set_tuning(op.handle, int(batch), None), "abba_op_set_tuning")
        return
    t = _Tune(a_path, a_jb, b_g, czt, a_rb, a_occ, 0.0, 0.0, 0, a_tile, a_vg)
    _check(lib.abba_op_set_tuning(op.handle, int(batch), ctypes.byref(t)), "abba_op_set_tuning")


def get_tuning(op: Operator, batch: int):
    """The launch choices `op` keeps for `batch`, or None."""
    t = _Tune()
    r = lib.abba_op_get_tuning(op.handle, int(batch), ctypes.byref(t))
    if r < 0:
        _check(r, "abba_op_get_tuning")
    return _tune_dict(t) if r == 1 else None


ORTHO = {"dcgs2": 0, "cgs2": 1}


def _structs(reg, lam, tau, noise_norm, mlp, judge_delta, stop, stop_tau, rns_eps, use_graph, poll_every,
             restart, features, ortho="dcgs2", learned_gate=0.0, streams=1):
    r = _Reg()
    r.kind = REG[reg]
    r.lam = float(lam)
    r.tau = float(tau)
    r.noise_norm = None if noise_norm is None else noise_norm.data_ptr()
    r.mlp = None if mlp is None else mlp.data_ptr()
    r.judge_delta = float(judge_delta)
    s = _Stop()
    s.kind = STOP[stop]
    s.tau = float(stop_tau)
    s.rns_eps = float(rns_eps)
    s.noise_norm = None if noise_norm is None else noise_norm.data_ptr()
    s.learned_gate = float(learned_gate)
    e = _Exec()
    e.use_graph = int(bool(use_graph))
    e.poll_every = int(poll_every)
    e.restart = int(restart)
    e.features = int(features)
    e.ortho = ORTHO[ortho]
    e.streams = int(streams)
    return r, s, e


def workspace_bytes(A: Operator, B: Operator, batch: int, mode: str, k: int, stop=None, labels=False,
                    restart: int = 0, streams: int = 1) -> int:
    _, s, e = _structs("none", 0, 0, None, None, 0, stop, 1.01, 1e-3, 0, 1, restart, FEAT_LABELS if labels else 0,
                       streams=streams)
    nb = ctypes.c_size_t()
    _check(lib.abba_solve_workspace(A.handle, B.handle, batch, MODE_AB if mode == "AB" else MODE_BA, k,
                                    ctypes.byref(s), ctypes.byref(e), ctypes.byref(nb)), "abba_solve_workspace")
    return nb.value


def solve_layout(A: Operator, B: Operator, batch: int, mode: str, k: int, stop=None, labels=False,
                 restart: int = 0) -> dict:
    """Where abba_solve keeps the basis W and the Hessenberg matrix H inside
    its workspace (abba_solve_layout): byte offsets and strides."""
    _, s, e = _structs("none", 0, 0, None, None, 0, stop, 1.01, 1e-3, 0, 1, restart, FEAT_LABELS if labels else 0)
    L = _Layout()
    _check(lib.abba_solve_layout(A.handle, B.handle, batch, MODE_AB if mode == "AB" else MODE_BA, k,
                                 ctypes.byref(s), ctypes.byref(e), ctypes.byref(L)), "abba_solve_layout")
    return dict(bytes=L.bytes, basis=L.basis, hessenberg=L.hessenberg, singular_values=L.singular_values,
                ldw=L.ldw, len=L.len,
                basis_dtype=L.basis_dtype, basis_slots=L.basis_slots, k=L.k)


def basis_views(workspace, layout: dict, batch: int, sigma: bool = False):
    """(W, H) views into a solve's workspace tensor: W [batch, slots, ldw] in the
    basis dtype, H [batch, k, k+1] float64 (column j of H_k is H[s, j]); with
    sigma, also the singular values of H_k, float64 [batch, k], descending."""
    import torch
    dt = _torch_dtype(layout["basis_dtype"])
    esz = torch.empty((), dtype=dt).element_size()
    nW = batch * layout["basis_slots"] * layout["ldw"]
    W = workspace[layout["basis"]:layout["basis"] + nW * esz].view(dt).view(batch, layout["basis_slots"],
                                                                            layout["ldw"])
    k = layout["k"]
    nH = batch * k * (k + 1)
    H = workspace[layout["hessenberg"]:layout["hessenberg"] + nH * 8].view(torch.float64).view(batch, k, k + 1)
    if not sigma:
        return W, H
    o = layout["singular_values"]
    sv = workspace[o:o + batch * k * 8].view(torch.float64).view(batch, k)
    return W, H, sv


def solve(A: Operator, B: Operator, b, mode: str = "AB", k: int = 30, reg: str = "gcv", lam: float = 0.0,
          tau: float = 1.01, noise_norm=None, stop=None, rns_eps: float = 1e-3, x0=None, use_graph=False,
          poll_every: int = 1, restart: int = 0, mlp=None, judge_delta: float = 0.05, history: bool = True,
          workspace=None, features: bool = False, ortho: str = "dcgs2", x_true=None, phases: bool = False,
          learned_gate: float = 0.0, streams: int = 1):
    """Hybrid AB-/BA-GMRES on a batch of slices; returns (x, info).

    streams > 1 runs the batch as that many sub-batches of consecutive slices
    concurrently, each on a stream and host thread of its own inside the
    library (the same bits per slice; the workspace is workspace_bytes(...,
    streams=streams)).

    ortho: "dcgs2" (CGS2 with the second pass delayed to the next step's
    sweep, the default) or "cgs2" (both passes in each step).

    b: device tensor [batch, *sino_shape] in A's sinogram dtype.  noise_norm:
    device float64 [batch] (||e|| per slice) for the discrepancy principle.
    info holds device tensors iters [batch], status [batch] and, with
    history, lam [batch, k] and resid [batch, k+1].  features=True adds the
    learned-rule features [batch, k, 64] (float32); x_true (device, image
    dtype, AB mode) adds the RRE label grid rre [batch, k, 64].  mlp: device
    float32 [MLP_PARAMS] for reg="learned".  learned_gate = c > 0: the learned
    stop (with noise_norm) fires only once rho_k <= c tau ||e||.  phases=True times the phases of
    the solve with HIP events (the iterations then run without a graph and the
    call waits for the stream) and adds info["phase_ms"], a dict over PHASES.
    """
    import torch
    batch = _need(b, A.sino_dtype, A.m, "b")
    dev = b.device
    if x0 is None:
        x = torch.zeros((batch, *A.geom.image_shape), dtype=A.img_dtype, device=dev)
    else:
        x = x0.clone()
    _need_exact(x, A.img_dtype, batch * A.n, "x0")
    if noise_norm is not None:
        noise_norm = noise_norm.to(device=dev, dtype=torch.float64).contiguous()
        if noise_norm.numel() != batch:
            raise ValueError(f"noise_norm has {noise_norm.numel()} entries, expected one per slice ({batch})")
    fbits = (FEAT_OUT if features else 0) | (FEAT_LABELS if x_true is not None else 0)
    r, s, e = _structs(reg, lam, tau, noise_norm, mlp, judge_delta, stop, tau, rns_eps, use_graph, poll_every,
                       restart, fbits, ortho, learned_gate, streams)
    pms = (ctypes.c_double * len(PHASES))() if phases else None
    e.phase_ms = None if pms is None else ctypes.addressof(pms)
    m = MODE_AB if mode == "AB" else MODE_BA
    iters = torch.zeros(batch, dtype=torch.int32, device=dev)
    status = torch.zeros(batch, dtype=torch.int32, device=dev)
    lamh = torch.empty((batch, k), dtype=torch.float64, device=dev) if history else None
    resh = torch.empty((batch, k + 1), dtype=torch.float64, device=dev) if history else None
    o = _Out()
    o.iters, o.status = iters.data_ptr(), status.data_ptr()
    o.lam = None if lamh is None else lamh.data_ptr()
    o.resid = None if resh is None else resh.data_ptr()
    ncph = torch.empty((batch, k), dtype=torch.float64, device=dev) if (history and stop == "ncp") else None
    o.ncp = None if ncph is None else ncph.data_ptr()
    feats = torch.zeros((batch, k, MLP_FEATURES), dtype=torch.float32, device=dev) if features else None
    o.features = None if feats is None else feats.data_ptr()
    rre = None
    if x_true is not None:
        _need_exact(x_true, A.img_dtype, batch * A.n, "x_true")
        rre = torch.full((batch, k, LABEL_GRID), float("nan"), dtype=torch.float64, device=dev)
        o.x_true = x_true.data_ptr()
        o.rre = rre.data_ptr()
    if mlp is not None:
        _need_exact(mlp, torch.float32, MLP_PARAMS, "mlp")
    nb = ctypes.c_size_t()
    _check(lib.abba_solve_workspace(A.handle, B.handle, batch, m, k, ctypes.byref(s), ctypes.byref(e),
                                    ctypes.byref(nb)), "abba_solve_workspace")
    if workspace is None:
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    elif not workspace.is_cuda or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 device tensor")
    _check(lib.abba_solve(A.handle, B.handle, _ptr(b), _ptr(x), batch, m, k, ctypes.byref(r), ctypes.byref(s),
                          ctypes.byref(o), ctypes.byref(e), _ptr(workspace), workspace.numel(), _stream_ptr()),
           "abba_solve")
    info = dict(iters=iters, status=status, lam=lamh, resid=resh, features=feats, rre=rre, ncp=ncph)
    if pms is not None:
        info["phase_ms"] = {name: float(pms[i]) for i, name in enumerate(PHASES)}
    return x, info


def mlp_forward(params, X):
    """Y [n, 2] = network(X [n, 64]) (float32 device tensors)."""
    import torch
    n = _need(X, torch.float32, MLP_FEATURES, "X")
    _need_exact(params, torch.float32, MLP_PARAMS, "params")
    Y = torch.empty((n, 2), dtype=torch.float32, device=X.device)
    _check(lib.abba_mlp_forward(_ptr(params), _ptr(X), n, _ptr(Y), _stream_ptr()), "abba_mlp_forward")
    return Y


def mlp_loss_grad_workspace_bytes(n: int) -> int:
    """Device bytes of per-tile partial gradients for n samples."""
    return _bytes(lib.abba_mlp_loss_grad_workspace, int(n))


def mlp_loss_grad(params, X, T, idx=None, grad=None, loss=None, workspace=None):
    """(loss, grad) of the mean squared error over rows idx of (X, T) (all rows if None)."""
    import torch
    nrows = _need(X, torch.float32, MLP_FEATURES, "X")
    if _need(T, torch.float32, 2, "T") != nrows:
        raise ValueError("X and T need the same number of rows")
    _need_exact(params, torch.float32, MLP_PARAMS, "params")
    n = nrows
    if idx is not None:
        n = _need(idx, torch.int32, 1, "idx")
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device) if grad is None else grad
    loss = torch.empty(1, dtype=torch.float64, device=X.device) if loss is None else loss
    _need_exact(grad, torch.float32, MLP_PARAMS, "grad")
    _need_exact(loss, torch.float64, 1, "loss")
    ws = _workspace(mlp_loss_grad_workspace_bytes(n), workspace, X.device)
    _check(lib.abba_mlp_loss_grad(_ptr(params), _ptr(X), _ptr(T), nrows, None if idx is None else _ptr(idx), n,
                                  _ptr(grad), _ptr(loss), *_wsptr(ws), _stream_ptr()), "abba_mlp_loss_grad")
    return loss, grad


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on params (m, v: moment buffers)."""
    import torch
    for t, name in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _need_exact(t, torch.float32, MLP_PARAMS, name)
    _check(lib.abba_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                             float(beta2), float(eps), _stream_ptr()), "abba_mlp_adam")


def mlp_labels(rre, iters=None):
    """Training targets [batch, k, 2] and k* [batch] from solve(..., x_true=...)'s rre."""
    import torch
    if rre.dim() != 3 or rre.shape[2] != LABEL_GRID:
        raise ValueError(f"rre must be [batch, k, {LABEL_GRID}]")
    batch, k = rre.shape[0], rre.shape[1]
    _need_exact(rre, torch.float64, batch * k * LABEL_GRID, "rre")
    tgt = torch.empty((batch, k, 2), dtype=torch.float32, device=rre.device)
    ks = torch.empty(batch, dtype=torch.int32, device=rre.device)
    if iters is not None:
        _need_exact(iters, torch.int32, batch, "iters")
    _check(lib.abba_mlp_labels(_ptr(rre), batch, k, None if iters is None else _ptr(iters), _ptr(tgt), _ptr(ks),
                               _stream_ptr()), "abba_mlp_labels")
    return tgt, ks


def mlp_train(params, X, T, epochs, batch=4096, lr=1e-3, seed=0, log=None):
    """Adam on the mean squared error over minibatches of (X, T), in place on
    params; the sample order of each epoch is a seeded permutation drawn on
    the host.  Returns the mean loss of each epoch."""
    import numpy as np
    import torch
    nrows = _need(X, torch.float32, MLP_FEATURES, "X")
    m = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=X.device)
    v = torch.zeros_like(m)
    grad = torch.empty_like(m)
    loss = torch.empty(1, dtype=torch.float64, device=X.device)
    rng = np.random.default_rng(seed)
    ws = torch.empty(mlp_loss_grad_workspace_bytes(min(batch, nrows)), dtype=torch.uint8, device=X.device)
    step, hist = 0, []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(nrows).astype(np.int32), device=X.device)
        tot = torch.zeros(1, dtype=torch.float64, device=X.device)
        nb = 0
        for i0 in range(0, nrows, batch):
            idx = perm[i0:i0 + batch]
            mlp_loss_grad(params, X, T, idx=idx, grad=grad, loss=loss, workspace=ws)
            step += 1
            mlp_adam(params, grad, m, v, step, lr)
            tot += loss
            nb += 1
        hist.append(float(tot) / nb)
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return hist


def status_names(code: int):
    names = {ST_KMAX: "kmax", ST_STOP_DP: "dp", ST_STOP_RNS: "rns", ST_BREAKDOWN: "breakdown",
             ST_NONFINITE: "nonfinite", ST_STOP_LEARNED: "learned", ST_STOP_NCP: "ncp"}
    return [v for b_, v in names.items() if code & b_]


def relative_l2(a, b) -> float:
    """||a - b|| / ||b|| in float64 (a convenience for reports)."""
    import torch
    a = a.to(torch.float64)
    b = b.to(torch.float64)
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

