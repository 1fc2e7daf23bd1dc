"""ctypes binding of libbgk.so (argument marshalling only).

Every computation runs in the HIP library; this module turns problem dicts
into ``bgk_problem`` structs, passes device pointers of torch tensors and the
current torch stream, and raises on non-zero status codes.  It fails loudly
when the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbgk.so")

OK, E_INVALID, E_CFL, E_UNSUPPORTED, E_HIP, E_NONFINITE, E_NEGATIVE, E_ALIAS = range(8)
KINDS = {"shock": 0, "cavity": 1, "periodic1d": 2, "periodic2d": 3, "cavity3d": 4, "periodic3d": 5}
FP64, FP32 = 0, 1


class BGKError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bgk error {code}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double),
        ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("nv", ctypes.c_int * 3),
        ("vlo", ctypes.c_double * 3), ("vhi", ctypes.c_double * 3),
        ("kn", ctypes.c_double), ("omega", ctypes.c_double),
        ("cfl", ctypes.c_double), ("dt", ctypes.c_double),
        ("mach", ctypes.c_double), ("lid_mach", ctypes.c_double),
        ("t_wall", ctypes.c_double),
        ("splitting", ctypes.c_int), ("limiter", ctypes.c_int),
        ("maxwellian", ctypes.c_int),
        ("reduced", ctypes.c_int),
        ("nz", ctypes.c_int),
        ("z0", ctypes.c_double), ("z1", ctypes.c_double),
    ]


EXPORTS = ("bgk_init", "bgk_free", "bgk_last_error", "bgk_sizes", "bgk_instance_info",
           "bgk_initial_state", "bgk_step", "bgk_moments", "bgk_check", "bgk_set_timing",
           "bgk_timing", "bgk_autotune", "bgk_get_launch", "bgk_set_launch", "bgk_set_graph",
           "bgk_step_adjoint", "bgk_lid_shear", "bgk_lid_shear_grad", "bgk_set_rounding_seed",
           "bgk_get_rounding_seed", "bgk_cavity_metrics", "bgk_step_noalloc", "bgk_record_bytes",
           "bgk_step_record", "bgk_step_adjoint_record", "bgk_adjoint_sweep_record")

TUNED_PATH = os.path.join(HERE, "tuned.json")

_lib = None


def load(path: str = LIB_PATH):
    """Load libbgk.so and declare its signatures (no GPU work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_0903_4044_amd.build`")
    L = ctypes.CDLL(path)
    vp, sz, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_double), \
        ctypes.POINTER(ctypes.c_int)
    L.bgk_init.argtypes = [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    L.bgk_free.argtypes = [vp]
    L.bgk_last_error.argtypes = [vp]
    L.bgk_last_error.restype = ctypes.c_char_p
    L.bgk_sizes.argtypes = [vp, sz, sz, sz, sz]
    L.bgk_instance_info.argtypes = [vp, ctypes.c_int, sz, sz, dp]
    L.bgk_initial_state.argtypes = [vp, vp, vp]
    L.bgk_step.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp]
    L.bgk_moments.argtypes = [vp, vp, vp, vp]
    L.bgk_check.argtypes = [vp, vp, vp]
    L.bgk_set_timing.argtypes = [vp, ctypes.c_int]
    L.bgk_set_rounding_seed.argtypes = [vp, ctypes.c_uint]
    L.bgk_get_rounding_seed.argtypes = [vp, ctypes.POINTER(ctypes.c_uint)]
    L.bgk_timing.argtypes = [vp, dp, ip]
    L.bgk_autotune.argtypes = [vp, vp, vp, vp, vp]
    L.bgk_get_launch.argtypes = [vp, ip, ip, ip, ip, dp]
    L.bgk_set_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.bgk_set_graph.argtypes = [vp, ctypes.c_int]
    L.bgk_step_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.bgk_lid_shear.argtypes = [vp, vp, vp, vp]
    L.bgk_lid_shear_grad.argtypes = [vp, vp, vp, vp, vp]
    L.bgk_cavity_metrics.argtypes = [vp, vp, dp, vp]
    L.bgk_step_noalloc.argtypes = [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, vp, vp]
    L.bgk_record_bytes.argtypes = [vp, sz]
    L.bgk_step_record.argtypes = [vp, vp, vp, vp, vp]
    L.bgk_step_adjoint_record.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.bgk_adjoint_sweep_record.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp, vp, vp,
                                           vp]
    for name in EXPORTS:
        getattr(L, name).restype = getattr(L, name).restype or ctypes.c_int
    L.bgk_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def to_struct(cfg: dict) -> Problem:
    p = Problem()
    p.kind = KINDS[cfg["kind"]]
    p.nx = int(cfg["nx"])
    p.ny = int(cfg.get("ny", 1))
    p.x0, p.x1 = float(cfg["x0"]), float(cfg["x1"])
    p.y0, p.y1 = float(cfg.get("y0", 0.0)), float(cfg.get("y1", 1.0))
    for a in range(3):
        p.nv[a] = int(cfg["nv"][a])
        p.vlo[a] = float(cfg["vlo"][a])
        p.vhi[a] = float(cfg["vhi"][a])
    p.kn, p.omega = float(cfg["kn"]), float(cfg["omega"])
    p.cfl, p.dt = float(cfg.get("cfl", 0.5)), float(cfg.get("dt", 0.0))
    p.mach = float(cfg.get("mach", 0.0))
    p.lid_mach = float(cfg.get("lid_mach", 0.0))
    p.t_wall = float(cfg.get("t_wall", 1.0))
    p.splitting = 0 if cfg.get("splitting", "strang") == "strang" else 1
    p.limiter = {"minmod": 0, "none": 1, "shift": 2}[cfg.get("limiter", "minmod")]
    p.maxwellian = {"point": 0, "conservative": 1}[cfg.get("maxwellian", "point")]
    p.reduced = 1 if cfg.get("reduced", False) else 0
    p.nz = int(cfg.get("nz", 1))
    p.z0, p.z1 = float(cfg.get("z0", 0.0)), float(cfg.get("z1", 1.0))
    return p


def size_class(problems, precision: str) -> str:
    """Key of the tuned-shape table: dimension (the highest of a batch that
    mixes them), precision, velocity grid and the power-of-two bucket of the
    total cell count."""
    import math
    p0 = problems[0]
    cells = sum(inputs.ncells(p) for p in problems)
    bucket = 1 << max(0, math.ceil(math.log2(max(cells, 1))))
    nv = "x".join(str(int(v)) for v in p0["nv"])
    dim = max(inputs.ndim(p) for p in problems)
    return f"{dim}d/{precision}/nv{nv}/cells<={bucket}"


def load_tuned() -> dict:
    import json
    if os.path.exists(TUNED_PATH):
        with open(TUNED_PATH) as fh:
            return json.load(fh)
    return {}


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: torch.Tensor) -> int:
    assert t.is_cuda and t.is_contiguous()
    return int(t.data_ptr())


def step_noalloc(problems, precision: str, f_in: torch.Tensor, f_out: torch.Tensor, n: int,
                 ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """bgk_step_noalloc: n steps of `problems` (a dict or a list of dicts)
    without a context; the library allocates nothing.  ws: a device buffer of
    at least f_in's bytes (needed for n >= 2), the caller's."""
    if isinstance(problems, dict):
        problems = [problems]
    L = load()
    arr = (Problem * len(problems))(*[to_struct(p) for p in problems])
    code = FP64 if precision == "fp64" else FP32
    rc = L.bgk_step_noalloc(arr, len(problems), code, _ptr(f_in), _ptr(f_out), int(n),
                            _ptr(ws) if ws is not None else None, _stream_handle(stream))
    if rc != OK:
        raise BGKError(rc, L.bgk_last_error(None).decode())
    return f_out


class Context:
    """Owns a bgk_ctx for one or more instances stepped together.

    tune: "table" applies the launch shape recorded for this size class in
    tuned.json (if any), "off" keeps the library default; call autotune() to
    time all shapes on the current device.
    """

    def __init__(self, problems, precision: str | None = None, tune: str = "table"):
        if isinstance(problems, dict):
            problems = [problems]
        self.problems = [dict(p) for p in problems]
        prec = precision or self.problems[0].get("precision", "fp64")
        self.precision = prec
        self.code = FP64 if prec == "fp64" else FP32
        self.dtype = torch.float64 if prec == "fp64" else torch.float32
        self.L = load()
        arr = (Problem * len(self.problems))(*[to_struct(p) for p in self.problems])
        h = ctypes.c_void_p()
        rc = self.L.bgk_init(arr, len(self.problems), self.code, ctypes.byref(h))
        if rc != OK:
            raise BGKError(rc, self.L.bgk_last_error(None).decode())
        self.h = h
        fe, nc, ws, wa = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        self._check(self.L.bgk_sizes(self.h, ctypes.byref(fe), ctypes.byref(nc), ctypes.byref(ws), ctypes.byref(wa)))
        self.f_elems, self.ncells = fe.value, nc.value
        self.ws_step_bytes, self.ws_adjoint_bytes = ws.value, wa.value
        rb = ctypes.c_size_t()
        self._check(self.L.bgk_record_bytes(self.h, ctypes.byref(rb)))
        self.record_bytes = rb.value
        self._ws = {}  # caller-owned workspaces (torch), made at first use
        self.nvel = inputs.nvel(self.problems[0])
        self.offsets, self.cell_offsets, self.dts = [], [], []
        for i in range(len(self.problems)):
            fo, co, dt = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_double()
            self._check(self.L.bgk_instance_info(self.h, i, ctypes.byref(fo), ctypes.byref(co), ctypes.byref(dt)))
            self.offsets.append(fo.value)
            self.cell_offsets.append(co.value)
            self.dts.append(dt.value)
        self.key = size_class(self.problems, self.precision)
        if tune == "table":
            shape = load_tuned().get(self.key)
            if shape:
                try:  # a shape recorded for another streaming form of the same size class may not apply
                    self.set_launch(shape["vec"], shape["unroll"], shape["vsplit"], shape.get("persist", 0))
                except BGKError:
                    pass

    def _check(self, rc):
        if rc != OK:
            raise BGKError(rc, self.L.bgk_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.L.bgk_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers --------------------------------------------------------
    def empty(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.f_elems, dtype=self.dtype, device=device)

    def workspace(self, kind: str = "step", device="cuda") -> torch.Tensor:
        """The workspace of bgk_step ("step") or bgk_step_adjoint ("adjoint"):
        a torch byte tensor of the size bgk_sizes reports, kept for later calls."""
        ws = self._ws.get(kind)
        if ws is None:
            n = self.ws_step_bytes if kind == "step" else self.ws_adjoint_bytes
            ws = self._ws[kind] = torch.empty(n, dtype=torch.uint8, device=device)
        return ws

    def release_workspaces(self):
        """Drop the workspaces (the next call that needs one makes it again)."""
        self._ws.clear()

    def instance_view(self, f: torch.Tensor, i: int) -> torch.Tensor:
        n = inputs.ncells(self.problems[i]) * self.nvel
        o = self.offsets[i]
        return f[o:o + n].view(inputs.ncells(self.problems[i]), self.nvel)

    # -- calls ----------------------------------------------------------
    def initial_state(self, f: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        f = self.empty() if f is None else f
        self._check(self.L.bgk_initial_state(self.h, _ptr(f), _stream_handle(stream)))
        return f

    def step(self, f_in: torch.Tensor, f_out: torch.Tensor | None = None, n: int = 1, stream=None) -> torch.Tensor:
        f_out = torch.empty_like(f_in) if f_out is None else f_out
        assert f_in.dtype == self.dtype and f_in.numel() == self.f_elems and f_out.numel() == self.f_elems
        ws = _ptr(self.workspace("step", f_in.device)) if n >= 2 else None
        self._check(self.L.bgk_step(self.h, _ptr(f_in), _ptr(f_out), int(n), ws, _stream_handle(stream)))
        return f_out

    def moments(self, f: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        out = torch.empty((self.ncells, 5), dtype=torch.float64, device=f.device) if out is None else out
        self._check(self.L.bgk_moments(self.h, _ptr(f), _ptr(out), _stream_handle(stream)))
        return out

    # -- reverse sweep ----------------------------------------------------
    def grad_buffer(self, device="cuda") -> torch.Tensor:
        """Per-instance (dL/dKn, dL/dT_w) accumulator, float64 [ninst, 2]."""
        return torch.zeros((len(self.problems), 2), dtype=torch.float64, device=device)

    def step_adjoint(self, f_n: torch.Tensor, lam_next: torch.Tensor, lam_n: torch.Tensor | None = None,
                     grad: torch.Tensor | None = None, stream=None):
        """lam_n = (d step / d f_n)^T lam_next; adds this step's parameter
        gradients to grad (created if None).  Returns (lam_n, grad)."""
        lam_n = torch.empty_like(lam_next) if lam_n is None else lam_n
        grad = self.grad_buffer(f_n.device) if grad is None else grad
        self._check(self.L.bgk_step_adjoint(self.h, _ptr(f_n), _ptr(lam_next), _ptr(lam_n), _ptr(grad),
                                            _ptr(self.workspace("adjoint", f_n.device)), _stream_handle(stream)))
        return lam_n, grad

    def step_record(self, f_in: torch.Tensor, f_out: torch.Tensor | None = None, rec: torch.Tensor | None = None,
                    stream=None):
        """One step f_out = step(f_in) that keeps its record (a byte tensor of
        record_bytes) for step_adjoint_record.  Returns (f_out, rec)."""
        f_out = torch.empty_like(f_in) if f_out is None else f_out
        rec = torch.empty(self.record_bytes, dtype=torch.uint8, device=f_in.device) if rec is None else rec
        self._check(self.L.bgk_step_record(self.h, _ptr(f_in), _ptr(f_out), _ptr(rec), _stream_handle(stream)))
        return f_out, rec

    def step_adjoint_record(self, f_n: torch.Tensor, rec: torch.Tensor, lam_next: torch.Tensor,
                            lam_n: torch.Tensor | None = None, grad: torch.Tensor | None = None, stream=None):
        """step_adjoint at f_n from the record step_record kept for the step
        from f_n (nothing recomputed).  Returns (lam_n, grad)."""
        lam_n = torch.empty_like(lam_next) if lam_n is None else lam_n
        grad = self.grad_buffer(f_n.device) if grad is None else grad
        self._check(self.L.bgk_step_adjoint_record(self.h, _ptr(f_n), _ptr(rec), _ptr(lam_next), _ptr(lam_n),
                                                   _ptr(grad), _ptr(self.workspace("adjoint", f_n.device)),
                                                   _stream_handle(stream)))
        return lam_n, grad

    def adjoint_sweep_record(self, states, records, lam_N: torch.Tensor, lam_0: torch.Tensor | None = None,
                             grad: torch.Tensor | None = None, stream=None):
        """lambda^0 from lambda^N through the recorded steps (states[i], records[i])
        of a rollout, in one call.  Returns (lam_0, grad)."""
        n = len(states)
        if len(records) != n:
            raise ValueError("one record per state")
        lam_0 = torch.empty_like(lam_N) if lam_0 is None else lam_0
        grad = self.grad_buffer(lam_N.device) if grad is None else grad
        fp = (ctypes.c_void_p * max(n, 1))(*[_ptr(t) for t in states])
        rp = (ctypes.c_void_p * max(n, 1))(*[_ptr(t) for t in records])
        self._check(self.L.bgk_adjoint_sweep_record(self.h, n, fp, rp, _ptr(lam_N), _ptr(lam_0), _ptr(grad),
                                                    _ptr(self.workspace("adjoint", lam_N.device)),
                                                    _stream_handle(stream)))
        return lam_0, grad

    def lid_shear(self, f: torch.Tensor, stream=None) -> torch.Tensor:
        """Lid shear of every cavity instance (0 for other kinds), float64 [ninst]."""
        out = torch.empty(len(self.problems), dtype=torch.float64, device=f.device)
        self._check(self.L.bgk_lid_shear(self.h, _ptr(f), _ptr(out), _stream_handle(stream)))
        return out

    def lid_shear_grad(self, f: torch.Tensor, lam: torch.Tensor | None = None, grad: torch.Tensor | None = None,
                       stream=None):
        """dL/df of the lid shear (summed over instances) and its explicit T_w term."""
        lam = torch.empty_like(f) if lam is None else lam
        grad = self.grad_buffer(f.device) if grad is None else grad
        self._check(self.L.bgk_lid_shear_grad(self.h, _ptr(f), _ptr(lam), _ptr(grad), _stream_handle(stream)))
        return lam, grad

    def cavity_metrics(self, f: torch.Tensor, stream=None) -> np.ndarray:
        """(D, G) of every instance (NaN for non-cavities), shape [ninst, 2];
        synchronises the stream."""
        out = np.empty((len(self.problems), 2))
        self._check(self.L.bgk_cavity_metrics(self.h, _ptr(f), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              _stream_handle(stream)))
        return out

    def check(self, f: torch.Tensor, stream=None) -> int:
        return self.L.bgk_check(self.h, _ptr(f), _stream_handle(stream))

    def autotune(self, f: torch.Tensor, stream=None) -> dict:
        """Time every valid streaming-kernel shape on state f; keep the fastest.
        The timed steps write into a temporary torch buffer."""
        scratch = torch.empty_like(f)
        self._check(self.L.bgk_autotune(self.h, _ptr(f), _ptr(scratch), _ptr(self.workspace("step", f.device)),
                                        _stream_handle(stream)))
        del scratch
        return self.launch()

    def launch(self) -> dict:
        v, u, s, p, us = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._check(self.L.bgk_get_launch(self.h, ctypes.byref(v), ctypes.byref(u), ctypes.byref(s), ctypes.byref(p),
                                          ctypes.byref(us)))
        return {"vec": v.value, "unroll": u.value, "vsplit": s.value, "persist": p.value, "tuned_us": us.value}

    def set_launch(self, vec: int, unroll: int, vsplit: int, persist: int = 0):
        self._check(self.L.bgk_set_launch(self.h, int(vec), int(unroll), int(vsplit), int(persist)))

    def set_seed(self, seed: int):
        """Rounding seed of the FP32 path (stochastic rounding of stored values);
        bgk_step advances it by its step count."""
        self._check(self.L.bgk_set_rounding_seed(self.h, int(seed) & 0xFFFFFFFF))

    def seed(self) -> int:
        v = ctypes.c_uint()
        self._check(self.L.bgk_get_rounding_seed(self.h, ctypes.byref(v)))
        return v.value

    def set_graph(self, on: bool):
        """Replay the steady two-step launch sequence from a captured hipGraph."""
        self._check(self.L.bgk_set_graph(self.h, 1 if on else 0))

    def set_timing(self, capacity: int):
        """capacity > 0: time every streaming launch (events made up front); 0: off."""
        self._check(self.L.bgk_set_timing(self.h, int(capacity)))

    def timing(self):
        ms, n = ctypes.c_double(), ctypes.c_int()
        self._check(self.L.bgk_timing(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value
