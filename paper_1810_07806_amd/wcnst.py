"""Python binding of the C ABI in ``include/wcnst.h`` (``libwcnst.so``).

Argument marshalling only: every step of the solver runs in the HIP kernels
of the library.  PyTorch supplies device memory (state arrays, workspace) and
the HIP stream.  Importing works without a GPU; creating a solver requires the
built library and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import math
import os

from .build import LIB_PATH

OK, E_INVALID_ARG, E_NONPHYSICAL, E_MAX_STEPS, E_HIP = 0, 1, 2, 3, 4
_SYSTEM = {"advection": 0, "burgers": 1, "euler": 2}
_BC = {"periodic": 0, "zero_gradient": 1, "reflect": 2, "fixed": 3}
_FLUX = {"roe": 0, "lf": 1, "vanleer": 2}
_SCHEME = {"teno": 0, "linear": 1, "js": 2, "z": 3}
_DIFF = {"mnd": 0, "md": 1, "hwcns": 2}

EXPORTS = ("wcnst_desc_init", "wcnst_workspace_size", "wcnst_create", "wcnst_rhs", "wcnst_step",
           "wcnst_solve", "wcnst_status_sync", "wcnst_reset", "wcnst_set_tuning", "wcnst_stage_shape",
           "wcnst_stage_layout",
           "wcnst_profile_enable",
           "wcnst_profile_read", "wcnst_destroy", "wcnst_last_error",
           "wcnst_batch_workspace_size", "wcnst_batch_create", "wcnst_batch_offsets", "wcnst_batch_solve",
           "wcnst_batch_bad_cells", "wcnst_batch_set_tuning", "wcnst_batch_kernel_ms", "wcnst_batch_stats",
           "wcnst_batch_set_persist",
           "wcnst_batch_destroy",
           "wcnst_pool_workspace_size", "wcnst_pool_create", "wcnst_pool_admit", "wcnst_pool_tick",
           "wcnst_pool_result", "wcnst_pool_release", "wcnst_pool_set_tuning", "wcnst_pool_tick_split",
           "wcnst_pool_tick_ms", "wcnst_pool_destroy", "wcnst_solve_noalloc")


class WcnstError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"wcnst status {status}: {msg}")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("ndim", ctypes.c_int32), ("system", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("flux", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("diff", ctypes.c_int32), ("charwise", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("gamma", ctypes.c_double), ("adv_speed", ctypes.c_double), ("CT", ctypes.c_double),
        ("C", ctypes.c_double), ("eps_teno", ctypes.c_double), ("eps_js", ctypes.c_double),
        ("fixed_x", (ctypes.c_double * 4) * 2), ("fixed_y", (ctypes.c_double * 4) * 2),
        ("gravity", ctypes.c_double),
        ("z_q", ctypes.c_int32), ("eps_z", ctypes.c_double),
    ]


_lib = None


def lib(path: str | None = None):
    """Load ``libwcnst.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: build it with "
                           "`python -m paper_1810_07806_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(path)
    vp, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
    D = ctypes.POINTER(Desc)
    L.wcnst_desc_init.argtypes = [D]
    L.wcnst_workspace_size.argtypes = [D, ctypes.POINTER(ctypes.c_size_t)]
    L.wcnst_create.argtypes = [D, vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.wcnst_rhs.argtypes = [vp, vp, vp, vp]
    L.wcnst_step.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double]
    L.wcnst_solve.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int64, dp, i64p]
    L.wcnst_status_sync.argtypes = [vp, dp, i64p, ctypes.POINTER(ctypes.c_int32), i64p, i64p]
    L.wcnst_reset.argtypes = [vp, ctypes.c_double, ctypes.c_int64]
    L.wcnst_set_tuning.argtypes = [vp, ctypes.c_int32]
    L.wcnst_stage_shape.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int32)] * 5
    L.wcnst_stage_layout.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.wcnst_profile_enable.argtypes = [vp, ctypes.c_int]
    L.wcnst_profile_read.argtypes = [vp, dp, i64p]
    L.wcnst_destroy.argtypes = [vp]
    L.wcnst_last_error.restype = ctypes.c_char_p
    L.wcnst_batch_workspace_size.argtypes = [D, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    L.wcnst_batch_create.argtypes = [D, ctypes.c_int32, vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.wcnst_batch_offsets.argtypes = [vp, i64p]
    L.wcnst_batch_solve.argtypes = [vp, vp, dp, ctypes.c_double, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_int32), dp, i64p]
    L.wcnst_batch_bad_cells.argtypes = [vp, i64p, i64p]
    L.wcnst_batch_set_tuning.argtypes = [vp, ctypes.c_int32]
    L.wcnst_batch_kernel_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.wcnst_batch_stats.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int32)] * 3
    L.wcnst_batch_set_persist.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.wcnst_batch_destroy.argtypes = [vp]
    i32, i32p = ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)
    L.wcnst_pool_workspace_size.argtypes = [i32, ctypes.POINTER(ctypes.c_size_t)]
    L.wcnst_pool_create.argtypes = [D, i32, vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.wcnst_pool_admit.argtypes = [vp, D, vp, vp, vp, ctypes.c_double, ctypes.c_double, i32p]
    L.wcnst_pool_tick.argtypes = [vp, ctypes.c_int64, i32p]
    L.wcnst_pool_result.argtypes = [vp, i32, i32p, i32p, dp, i64p, i64p, i64p]
    L.wcnst_pool_release.argtypes = [vp, i32]
    L.wcnst_pool_set_tuning.argtypes = [vp, i32]
    L.wcnst_pool_tick_split.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]
    L.wcnst_pool_tick_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.wcnst_pool_destroy.argtypes = [vp]
    L.wcnst_solve_noalloc.argtypes = [D, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int64, dp, i64p]
    for name in EXPORTS:
        if name != "wcnst_last_error":
            getattr(L, name).restype = ctypes.c_int32
    _lib = L
    return L


def _check(st: int):
    if st != OK:
        raise WcnstError(st, lib().wcnst_last_error().decode())


def make_desc(desc: dict) -> Desc:
    d = Desc()
    _check(lib().wcnst_desc_init(ctypes.byref(d)))
    d.ndim = int(desc.get("ndim", 1))
    d.system = _SYSTEM[desc.get("system", "euler")]
    d.nx = int(desc["nx"])
    d.ny = int(desc.get("ny", 1)) if d.ndim == 2 else 1
    d.x0, d.x1 = float(desc.get("x0", 0.0)), float(desc.get("x1", 1.0))
    d.y0, d.y1 = float(desc.get("y0", 0.0)), float(desc.get("y1", 1.0))
    d.bc_x = _BC[desc.get("bc_x", "zero_gradient")]
    d.bc_y = _BC[desc.get("bc_y", "zero_gradient")]
    d.flux = _FLUX[desc.get("flux", "roe")]
    d.scheme = _SCHEME[desc.get("scheme", "teno")]
    d.diff = _DIFF[desc.get("diff", "mnd")]
    d.charwise = int(desc.get("charwise", 1))
    d.q = int(desc.get("q", 6))
    d.gamma = float(desc.get("gamma", 1.4))
    d.adv_speed = float(desc.get("adv_speed", 1.0))
    d.CT = float(desc.get("CT", 1e-5))
    d.C = float(desc.get("C", 1.0))
    d.eps_teno = float(desc.get("eps_teno", 1e-40))
    d.eps_js = float(desc.get("eps_js", 1e-6))
    for name in ("fixed_x", "fixed_y"):
        states = desc.get(name)
        if states is not None:
            arr = getattr(d, name)
            for side in range(2):
                for v, val in enumerate(states[side]):
                    arr[side][v] = float(val)
    d.gravity = float(desc.get("gravity", 0.0))
    d.z_q = int(desc.get("z_q", 1))
    d.eps_z = float(desc.get("eps_z", 1e-40))
    return d


def nvar(desc: dict) -> int:
    if desc.get("system", "euler") != "euler":
        return 1
    return 3 if int(desc.get("ndim", 1)) == 1 else 4


def _nfaces_1d(desc: dict) -> int:
    """Midpoints of a 1D line: -2 .. nx for MND, -3 .. nx+1 for MD, -1 .. nx-1
    for HWCNS."""
    return int(desc["nx"]) + {"mnd": 3, "md": 5, "hwcns": 1}[desc.get("diff", "mnd")]


def flag_count(desc: dict) -> int:
    nv, nx = nvar(desc), int(desc["nx"])
    if int(desc.get("ndim", 1)) == 1:
        return nv * _nfaces_1d(desc) * 2
    ny = int(desc["ny"])
    return nv * ny * (nx + 3) * 2 + nv * nx * (ny + 3) * 2


def solve_noalloc(desc: dict, U, t_final: float = math.inf, cfl: float = 0.5, max_steps: int = 1 << 62,
                  stream=None):
    """wcnst_solve_noalloc: solve U (a contiguous float64 CUDA tensor of
    nvar * ny * nx values) in place from t = 0 with the library's static
    scratch (no workspace).  Returns (t, steps); raises WcnstError."""
    import torch
    if not (isinstance(U, torch.Tensor) and U.is_cuda and U.dtype == torch.float64 and U.is_contiguous()):
        raise TypeError("state must be a contiguous float64 CUDA tensor")
    ny = int(desc.get("ny", 1)) if int(desc.get("ndim", 1)) == 2 else 1
    if U.numel() != nvar(desc) * ny * int(desc["nx"]):
        raise ValueError("state size does not match the descriptor")
    d = make_desc(desc)
    st = stream if stream is not None else torch.cuda.current_stream(U.device)
    t = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().wcnst_solve_noalloc(ctypes.byref(d), ctypes.c_void_p(st.cuda_stream), ctypes.c_void_p(U.data_ptr()),
                                     float(t_final), float(cfl), int(max_steps), ctypes.byref(t), ctypes.byref(n)))
    return t.value, n.value


class Solver:
    """One WCNS-T solver bound to a torch CUDA stream and a torch-owned workspace."""

    def __init__(self, desc: dict, stream=None, device: str = "cuda"):
        import torch
        self._torch = torch
        self.desc = dict(desc)
        self.nv = nvar(desc)
        self.ny = int(desc.get("ny", 1)) if int(desc.get("ndim", 1)) == 2 else 1
        self.nx = int(desc["nx"])
        self._d = make_desc(desc)
        n = ctypes.c_size_t(0)
        _check(lib().wcnst_workspace_size(ctypes.byref(self._d), ctypes.byref(n)))
        self.ws_bytes = n.value
        raw = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + n.value]
        self.stream = stream if stream is not None else torch.cuda.current_stream(raw.device)
        h = ctypes.c_void_p()
        _check(lib().wcnst_create(ctypes.byref(self._d), ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.c_void_p(self.ws.data_ptr()), n.value, ctypes.byref(h)))
        self._h = h

    # -- helpers
    def _state(self, U):
        t = self._torch
        if not (isinstance(U, t.Tensor) and U.is_cuda and U.dtype == t.float64 and U.is_contiguous()):
            raise TypeError("state must be a contiguous float64 CUDA tensor")
        if U.numel() != self.nv * self.ny * self.nx:
            raise ValueError(f"state has {U.numel()} values, expected {self.nv}x{self.ny}x{self.nx}")
        return ctypes.c_void_p(U.data_ptr())

    def new_state(self, U_host):
        """Copy a host array (nv, ny, nx) to a new device tensor."""
        t = self._torch
        return t.as_tensor(U_host, dtype=t.float64).reshape(self.nv, self.ny, self.nx).to(
            self.ws.device).contiguous()

    # -- C ABI
    def rhs(self, U, flags: bool = False, out=None):
        t = self._torch
        R = out if out is not None else t.empty_like(U)
        fl = t.zeros(flag_count(self.desc), dtype=t.uint8, device=U.device) if flags else None
        _check(lib().wcnst_rhs(self._h, self._state(U), self._state(R),
                               ctypes.c_void_p(fl.data_ptr()) if fl is not None else None))
        return (R, fl) if flags else R

    def step(self, U, dt: float = 0.0, cfl: float = 0.5):
        _check(lib().wcnst_step(self._h, self._state(U), float(dt), float(cfl)))

    def solve(self, U, t_final: float = math.inf, cfl: float = 0.5, max_steps: int = 1 << 62):
        t = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        st = lib().wcnst_solve(self._h, self._state(U), float(t_final), float(cfl), int(max_steps),
                               ctypes.byref(t), ctypes.byref(n))
        if st not in (OK,):
            raise WcnstError(st, lib().wcnst_last_error().decode())
        return t.value, n.value

    def status(self) -> dict:
        t, n, s = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int32()
        bs, bc = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().wcnst_status_sync(self._h, ctypes.byref(t), ctypes.byref(n), ctypes.byref(s),
                                       ctypes.byref(bs), ctypes.byref(bc)))
        return dict(t=t.value, steps=n.value, status=s.value, bad_stage=bs.value, bad_cell=bc.value)

    def reset(self, t: float = 0.0, steps: int = 0):
        _check(lib().wcnst_reset(self._h, float(t), int(steps)))

    def set_tuning(self, rows_per_segment: int):
        _check(lib().wcnst_set_tuning(self._h, int(rows_per_segment)))

    def stage_shape(self) -> dict:
        """Launch shape of the stage kernels: strips, and segments 0 ..
        nseg1-1 of rows1 rows then rows2 rows up to nseg (2D)."""
        v = [ctypes.c_int32() for _ in range(5)]
        _check(lib().wcnst_stage_shape(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("strips", "rows1", "rows2", "nseg1", "nseg"), (x.value for x in v)))

    def stage_layout(self):
        """Rows of the first-height segments in the next two-height 2D stage
        launch, an int32 array [strips][nseg1 + 1] of boundaries, or None
        where stage launches use fixed heights."""
        import numpy as np
        n = ctypes.c_int32()
        _check(lib().wcnst_stage_layout(self._h, None, 0, ctypes.byref(n)))
        if n.value == 0:
            return None
        out = np.zeros(n.value, dtype=np.int32)
        _check(lib().wcnst_stage_layout(self._h, out.ctypes.data, n.value, ctypes.byref(n)))
        strips = self.stage_shape()["strips"]
        return out.reshape(strips, n.value // strips)

    def profile_enable(self, on: bool = True):
        _check(lib().wcnst_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().wcnst_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().wcnst_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def split_flags(desc: dict, fl):
    """Views of a flat flag buffer as the x (and y) blocks of ``wcnst_rhs``."""
    nv, nx = nvar(desc), int(desc["nx"])
    if int(desc.get("ndim", 1)) == 1:
        return [fl.reshape(nv, 1, _nfaces_1d(desc), 2)]
    ny = int(desc["ny"])
    nxb = nv * ny * (nx + 3) * 2
    return [fl[:nxb].reshape(nv, ny, nx + 3, 2), fl[nxb:].reshape(nv, nx, ny + 3, 2)]


class Batch:
    """Many independent 1D Euler problems advanced together in graph-captured
    ticks of multi-instance stage launches.

    States are packed into one device tensor (``pack``/``unpack``); instance i
    occupies ``offsets[i] : offsets[i] + 3 * nx_i`` with layout [v][nx_i]."""

    def __init__(self, descs, stream=None, device: str = "cuda"):
        import numpy as np
        import torch
        self._torch = torch
        self.descs = [dict(d) for d in descs]
        self.n = len(descs)
        arr = (Desc * self.n)(*[make_desc(d) for d in descs])
        self._arr = arr
        nbytes = ctypes.c_size_t(0)
        _check(lib().wcnst_batch_workspace_size(arr, self.n, ctypes.byref(nbytes)))
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + nbytes.value]
        self.stream = stream if stream is not None else torch.cuda.current_stream(raw.device)
        h = ctypes.c_void_p()
        _check(lib().wcnst_batch_create(arr, self.n, ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.c_void_p(self.ws.data_ptr()), nbytes.value, ctypes.byref(h)))
        self._h = h
        offs = (ctypes.c_int64 * (self.n + 1))()
        _check(lib().wcnst_batch_offsets(self._h, offs))
        self.offsets = np.array(list(offs), dtype=np.int64)

    def pack(self, states):
        """Device tensor holding every instance's (3, 1, nx) state."""
        import numpy as np
        host = np.zeros(int(self.offsets[-1]), dtype=np.float64)
        for i, U in enumerate(states):
            a = np.ascontiguousarray(U, dtype=np.float64).ravel()
            host[self.offsets[i]:self.offsets[i] + a.size] = a
        return self._torch.as_tensor(host).to(self.ws.device)

    def unpack(self, Ug):
        h = Ug.cpu().numpy()
        return [h[self.offsets[i]:self.offsets[i] + 3 * int(d["nx"])].reshape(3, 1, int(d["nx"])).copy()
                for i, d in enumerate(self.descs)]

    def set_tuning(self, steps_per_tick: int = 64):
        _check(lib().wcnst_batch_set_tuning(self._h, int(steps_per_tick)))

    def kernel_ms(self) -> float:
        ms = ctypes.c_double(0.0)
        _check(lib().wcnst_batch_kernel_ms(self._h, ctypes.byref(ms)))
        return ms.value

    def set_persist(self, switch_strips: int = 0, waves_per_group: int = 8, instances_per_group: int = 1):
        """Persistent finish once the running instances hold at most
        switch_strips strips (0: stage launches to the end)."""
        _check(lib().wcnst_batch_set_persist(self._h, int(switch_strips), int(waves_per_group),
                                             int(instances_per_group)))

    def stats(self) -> dict:
        """Ticks of the last solve, graphs captured for them and instances
        finished in the persistent launch."""
        tk, gr, pi = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().wcnst_batch_stats(self._h, ctypes.byref(tk), ctypes.byref(gr), ctypes.byref(pi)))
        return dict(ticks=tk.value, graphs=gr.value, persist_instances=pi.value)

    def solve(self, Ug, t_final, cfl: float = 0.5, max_steps: int = 1 << 40):
        """Returns dict(status, t, steps) arrays; raises only on HIP errors."""
        import numpy as np
        t = self._torch
        if not (isinstance(Ug, t.Tensor) and Ug.is_cuda and Ug.dtype == t.float64 and Ug.is_contiguous()
                and Ug.numel() >= int(self.offsets[-1])):
            raise TypeError("packed state must be a contiguous float64 CUDA tensor of the batch length")
        tf = np.broadcast_to(np.asarray(t_final, dtype=np.float64), (self.n,)).copy()
        st = (ctypes.c_int32 * self.n)()
        to = (ctypes.c_double * self.n)()
        so = (ctypes.c_int64 * self.n)()
        ret = lib().wcnst_batch_solve(self._h, ctypes.c_void_p(Ug.data_ptr()),
                                      tf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(cfl),
                                      int(max_steps), st, to, so)
        if ret == E_HIP or ret == E_INVALID_ARG:
            raise WcnstError(ret, lib().wcnst_last_error().decode())
        return dict(status=np.array(list(st)), t=np.array(list(to)), steps=np.array(list(so)))

    def bad_cells(self):
        import numpy as np
        bs = (ctypes.c_int64 * self.n)()
        bc = (ctypes.c_int64 * self.n)()
        _check(lib().wcnst_batch_bad_cells(self._h, bs, bc))
        return np.array(list(bs)), np.array(list(bc))

    def close(self):
        if getattr(self, "_h", None):
            lib().wcnst_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """Device-resident pool of Euler solves advanced together in ticks
    (continuous batching).  Request buffers are torch float64 CUDA tensors
    owned by the caller (for instance views of one arena)."""

    def __init__(self, scheme: dict | None = None, capacity: int = 256, stream=None, device: str = "cuda"):
        import torch
        self._torch = torch
        sch = dict(scheme or {})
        sch.setdefault("nx", 64)
        self._scheme = make_desc(sch)
        self.capacity = int(capacity)
        nbytes = ctypes.c_size_t(0)
        _check(lib().wcnst_pool_workspace_size(self.capacity, ctypes.byref(nbytes)))
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + nbytes.value]
        self.stream = stream if stream is not None else torch.cuda.current_stream(raw.device)
        h = ctypes.c_void_p()
        _check(lib().wcnst_pool_create(ctypes.byref(self._scheme), self.capacity,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.c_void_p(self.ws.data_ptr()),
                                       nbytes.value, ctypes.byref(h)))
        self._h = h
        self._held = {}

    def admit(self, desc: dict, U, U1, U2, t_final: float, cfl: float = 0.5) -> int:
        t = self._torch
        n = nvar(desc) * int(desc["nx"]) * (int(desc.get("ny", 1)) if int(desc.get("ndim", 1)) == 2 else 1)
        for a in (U, U1, U2):
            if not (isinstance(a, t.Tensor) and a.is_cuda and a.dtype == t.float64 and a.is_contiguous()
                    and a.numel() == n):
                raise TypeError(f"request buffers must be contiguous float64 CUDA tensors of {n} elements")
        d = make_desc(desc)
        slot = ctypes.c_int32(-1)
        _check(lib().wcnst_pool_admit(self._h, ctypes.byref(d), ctypes.c_void_p(U.data_ptr()),
                                      ctypes.c_void_p(U1.data_ptr()), ctypes.c_void_p(U2.data_ptr()),
                                      float(t_final), float(cfl), ctypes.byref(slot)))
        self._held[slot.value] = (U, U1, U2)
        return slot.value

    def tick(self, steps: int, steps_2d: int | None = None) -> int:
        """Advance the 1D requests by up to `steps` steps and the 2D ones by
        up to `steps_2d` (default: the same); returns the requests advanced."""
        n = ctypes.c_int32(0)
        _check(lib().wcnst_pool_tick_split(self._h, int(steps), int(steps if steps_2d is None else steps_2d),
                                           ctypes.byref(n)))
        return n.value

    def tick_ms(self) -> tuple:
        """Device time of the last tick's 1D and 2D launches (ms)."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().wcnst_pool_tick_ms(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def result(self, slot: int) -> dict:
        f, s = ctypes.c_int32(), ctypes.c_int32()
        tt = ctypes.c_double()
        n, bs, bc = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().wcnst_pool_result(self._h, int(slot), ctypes.byref(f), ctypes.byref(s), ctypes.byref(tt),
                                       ctypes.byref(n), ctypes.byref(bs), ctypes.byref(bc)))
        return dict(finished=bool(f.value), status=s.value, t=tt.value, steps=n.value, bad_stage=bs.value,
                    bad_cell=bc.value)

    def release(self, slot: int):
        _check(lib().wcnst_pool_release(self._h, int(slot)))
        self._held.pop(slot, None)

    def set_tuning(self, rows_per_segment: int = 0):
        _check(lib().wcnst_pool_set_tuning(self._h, int(rows_per_segment)))

    def close(self):
        if getattr(self, "_h", None):
            lib().wcnst_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
