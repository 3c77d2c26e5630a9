"""ctypes binding of libdg.so (include/dg.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides device memory (the state, the workspace,
flag and margin buffers) and the stream; the library never allocates.

Raises ``DGLibraryMissing`` when libdg.so is not built -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

DG_ABI_VERSION = 3
DG_OK, DG_ERR_INVALID_ARG, DG_ERR_UNSUPPORTED, DG_ERR_WORKSPACE, DG_ERR_HIP, DG_ERR_NONPHYSICAL = 0, -1, -2, -3, -4, -5
BURGERS, EULER = 0, 1
PERIODIC, TRANSMISSIVE, REFLECTIVE, INFLOW = 0, 1, 2, 3
LIM_NONE, LIM_CSWENO, LIM_CSWENO_CHAR = 0, 1, 2
IND_TVB, IND_ALL, IND_LEARNED, IND_KXRCF = 0, 1, 2, 3
NEGW_SPLIT, NEGW_RAW = 0, 1

# every symbol include/dg.h declares
EXPORTS = ("dg_workspace_bytes", "dg_init", "dg_destroy", "dg_proj_nodes", "dg_project", "dg_residual",
           "dg_limit", "dg_cfl_dt", "dg_step", "dg_status", "dg_strerror", "dg_profile_enable", "dg_profile_read",
           "dg_autotune", "dg_mlp_layout", "dg_mlp_features", "dg_mlp_forward", "dg_mlp_gradient", "dg_mlp_adam", "dg_set_learned",
           "dg_batch_workspace_bytes", "dg_batch_init", "dg_batch_destroy", "dg_batch_autotune", "dg_batch_set_tiles",
           "dg_batch_step", "dg_batch_set_learned", "dg_set_time", "dg_limit_noalloc")
PROF_KINDS = ("stage1", "stage23", "limiter", "dt")


class DGLibraryMissing(ImportError):
    pass


class DGError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("equation", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 4),
        ("limiter", ctypes.c_int32),
        ("indicator", ctypes.c_int32),
        ("negw_mode", ctypes.c_int32),
        ("positivity", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("x0", ctypes.c_double),
        ("x1", ctypes.c_double),
        ("y0", ctypes.c_double),
        ("y1", ctypes.c_double),
        ("tvb_M", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("bc_beyond", ctypes.c_int32 * 4),
        ("pad", ctypes.c_int32),
        ("bc_switch", (ctypes.c_double * 2) * 4),
        ("bc_state", ((ctypes.c_double * 4) * 2) * 4),
        ("x_nodes", ctypes.POINTER(ctypes.c_double)),
        ("y_nodes", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DGLibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                                   "python paper_1904_11147_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, vp = ctypes.POINTER, ctypes.c_void_p
        i32, d = ctypes.c_int32, ctypes.c_double
        sigs = {
            "dg_workspace_bytes": [P(Config), P(ctypes.c_size_t)],
            "dg_init": [P(Config), vp, ctypes.c_size_t, vp, P(vp)],
            "dg_destroy": [vp],
            "dg_proj_nodes": [vp, P(d), P(d), P(i32)],
            "dg_project": [vp, vp, i32, i32, vp],
            "dg_residual": [vp, vp, vp],
            "dg_limit": [vp, vp, vp, vp, vp, P(i32)],
            "dg_cfl_dt": [vp, vp, P(d)],
            "dg_step": [vp, vp, P(d), d, d, i32, P(i32)],
            "dg_status": [vp],
            "dg_profile_enable": [vp, ctypes.c_int],
            "dg_profile_read": [vp, P(d), P(ctypes.c_int64), P(ctypes.c_int64), ctypes.c_int],
            "dg_autotune": [vp, vp, P(i32), P(ctypes.c_float)],
            "dg_mlp_layout": [i32, P(i32), P(ctypes.c_int64), P(ctypes.c_int64)],
            "dg_mlp_features": [vp, vp, vp, vp],
            "dg_mlp_forward": [vp, i32, i32, vp, vp, vp, vp],
            "dg_mlp_gradient": [vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp],
            "dg_mlp_adam": [vp, vp, vp, vp, vp, i32, ctypes.c_float, i32, vp],
            "dg_set_learned": [vp, vp, vp, d, d, vp],
            "dg_batch_workspace_bytes": [P(Config), i32, P(ctypes.c_size_t)],
            "dg_batch_init": [P(Config), i32, vp, ctypes.c_size_t, vp, P(vp)],
            "dg_batch_destroy": [vp],
            "dg_batch_autotune": [vp, vp, P(ctypes.c_int64), P(i32), P(i32), P(ctypes.c_float)],
            "dg_batch_set_tiles": [vp, i32, i32],
            "dg_batch_step": [vp, vp, P(ctypes.c_int64), P(d), P(d), i32, P(i32), P(i32), P(ctypes.c_int64)],
            "dg_batch_set_learned": [vp, i32, vp, vp, d, d, vp],
            "dg_set_time": [vp, d],
            "dg_limit_noalloc": [P(Config), vp, vp, vp, vp, d, P(i32), vp],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.dg_strerror.argtypes = [ctypes.c_int]
        L.dg_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(code):
    try:
        return lib().dg_strerror(int(code)).decode()
    except DGLibraryMissing:
        return str(code)


def make_config(dim=1, equation=BURGERS, order=2, nx=16, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                bc=(PERIODIC,) * 4, gamma=1.4, limiter=LIM_CSWENO, indicator=IND_TVB, negw_mode=NEGW_SPLIT,
                tvb_M=1.0, weno_eps=1e-6, cfl=0.1, positivity=0, bc_beyond=(-1, -1, -1, -1),
                bc_switch=((0.0, 0.0),) * 4, bc_state=None, xn=None, yn=None):
    c = Config()
    c.abi_version = DG_ABI_VERSION
    c.dim, c.equation, c.order = dim, equation, order
    c.nx, c.ny = nx, (1 if dim == 1 else ny)
    for k in range(4):
        c.bc[k] = bc[k]
    c.limiter, c.indicator, c.negw_mode, c.positivity = limiter, indicator, negw_mode, int(positivity)
    c.gamma, c.x0, c.x1, c.y0, c.y1 = gamma, x0, x1, y0, y1
    c.tvb_M, c.weno_eps, c.cfl = tvb_M, weno_eps, cfl
    st = np.zeros((4, 2, 4)) if bc_state is None else np.asarray(bc_state, dtype=np.float64)
    c.pad = 0
    for k in range(4):
        c.bc_beyond[k] = int(bc_beyond[k])
        for a in range(2):
            c.bc_switch[k][a] = float(bc_switch[k][a])
            for v in range(4):
                c.bc_state[k][a][v] = float(st[k, a, v])
    keep = []  # node arrays of a non-uniform mesh, alive as long as the config
    for name, arr, n in (("x_nodes", xn, nx), ("y_nodes", yn, c.ny)):
        if arr is None:
            continue
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        if arr.shape != (n + 1,):
            raise ValueError(f"{name} needs {n + 1} values")
        keep.append(arr)
        setattr(c, name, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    c._keep = keep
    return c


def limit_noalloc(state, t=0.0, flags=None, margin=None, flags_override=None, stream=None, **cfg):
    """dg_limit_noalloc: the limiter on `state` (in place) for the
    configuration `cfg` with the library's static scratch; flags / margin are
    optional output tensors.  Returns (status code, n_troubled)."""
    c = make_config(**cfg)
    st = stream if stream is not None else torch.cuda.current_stream(state.device)
    n = ctypes.c_int32()
    rc = lib().dg_limit_noalloc(ctypes.byref(c), _ptr(state), _ptr(flags), _ptr(margin), _ptr(flags_override),
                                float(t), ctypes.byref(n), ctypes.c_void_p(st.cuda_stream))
    if rc not in (DG_OK, DG_ERR_NONPHYSICAL):
        raise DGError(rc, "dg_limit_noalloc")
    return rc, n.value


def workspace_bytes(cfg: Config) -> int:
    n = ctypes.c_size_t()
    rc = lib().dg_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n))
    if rc:
        raise DGError(rc, "dg_workspace_bytes")
    return n.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Problem:
    """One discretised problem bound to a CUDA/HIP device and stream."""

    def __init__(self, device="cuda", stream=None, **cfg):
        self.cfg = make_config(**cfg)
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.dim, self.order = self.cfg.dim, self.cfg.order
        self.nx, self.ny = self.cfg.nx, self.cfg.ny
        self.nv = 1 if self.cfg.equation == BURGERS else self.dim + 2
        self.nm = (self.order + 1) ** self.dim
        nbytes = workspace_bytes(self.cfg)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            handle = ctypes.c_void_p()
            rc = lib().dg_init(ctypes.byref(self.cfg), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle))
        if rc:
            raise DGError(rc, "dg_init")
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            lib().dg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- shapes -----------------------------------------------------------
    @property
    def shape(self):
        return (self.nv, self.nm, self.ny, self.nx)

    def empty_state(self):
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    def _check_state(self, s):
        if s.dtype != torch.float64 or tuple(s.shape) != self.shape or not s.is_contiguous() or s.device != self.device:
            raise ValueError(f"state must be a contiguous float64 {self.shape} tensor on {self.device}")

    def _rc(self, rc, what, allow_nonphysical=False):
        if rc == DG_ERR_NONPHYSICAL and allow_nonphysical:
            return rc
        if rc:
            raise DGError(rc, what)
        return rc

    # -- calls --------------------------------------------------------------
    def proj_nodes(self):
        r = (ctypes.c_double * 16)()
        w = (ctypes.c_double * 16)()
        nq = ctypes.c_int32()
        self._rc(lib().dg_proj_nodes(self._h, r, w, ctypes.byref(nq)), "dg_proj_nodes")
        return [r[k] for k in range(nq.value)], [w[k] for k in range(nq.value)]

    def project(self, point_values, state=None, j0=0):
        """point_values: device float64 [nv][nq][nq][rows][nx] (1D [nv][nq][1][nx])."""
        state = self.empty_state() if state is None else state
        self._check_state(state)
        pv = point_values.contiguous()
        if pv.dtype != torch.float64 or pv.device != self.device:
            raise ValueError("point_values must be float64 on the problem's device")
        nrows = pv.shape[-2] if self.dim == 2 else 1
        with torch.cuda.stream(self.stream):
            self._rc(lib().dg_project(self._h, _ptr(pv), int(j0), int(nrows), _ptr(state)), "dg_project")
        return state

    def residual(self, state, out=None):
        self._check_state(state)
        out = torch.empty_like(state) if out is None else out
        self._rc(lib().dg_residual(self._h, _ptr(state), _ptr(out)), "dg_residual", True)
        return out

    def limit(self, state, flags_override=None, want_margin=True, allow_nonphysical=True):
        """In place.  Returns (flags uint8 [ny,nx], margin float64 [ny,nx] or None, n_troubled)."""
        self._check_state(state)
        flags = torch.empty((self.ny, self.nx), dtype=torch.uint8, device=self.device)
        margin = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) if want_margin else None
        ovr = None
        if flags_override is not None:
            ovr = flags_override.to(device=self.device, dtype=torch.uint8).contiguous()
        n = ctypes.c_int32()
        rc = lib().dg_limit(self._h, _ptr(state), _ptr(flags), _ptr(margin), _ptr(ovr), ctypes.byref(n))
        self._rc(rc, "dg_limit", allow_nonphysical)
        return flags, margin, n.value

    def set_time(self, t):
        """Time of the boundary data for residual() and limit()."""
        self._rc(lib().dg_set_time(self._h, float(t)), "dg_set_time")

    def cfl_dt(self, state):
        self._check_state(state)
        dt = ctypes.c_double()
        self._rc(lib().dg_cfl_dt(self._h, _ptr(state), ctypes.byref(dt)), "dg_cfl_dt", True)
        return dt.value

    def step(self, state, t, t_end, dt=0.0, max_steps=2**31 - 1, allow_nonphysical=False):
        """Advance in place; returns (t, steps)."""
        self._check_state(state)
        tt = ctypes.c_double(t)
        steps = ctypes.c_int32()
        rc = lib().dg_step(self._h, _ptr(state), ctypes.byref(tt), float(t_end), float(dt), int(max_steps),
                           ctypes.byref(steps))
        self._rc(rc, "dg_step", allow_nonphysical)
        return tt.value, steps.value

    def status(self):
        return lib().dg_status(self._h)

    def autotune(self, state):
        """Tile height of the 2D stage kernels timed on this state: (rows, ms)."""
        self._check_state(state)
        rows = ctypes.c_int32()
        ms = ctypes.c_float()
        self._rc(lib().dg_autotune(self._h, _ptr(state), ctypes.byref(rows), ctypes.byref(ms)), "dg_autotune", True)
        return rows.value, ms.value

    def profile(self, enable=True):
        self._rc(lib().dg_profile_enable(self._h, 1 if enable else 0), "dg_profile_enable")

    def profile_read(self, reset=False):
        """{kind: (ms, launches)} and the troubled-cell total since the last reset."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int64 * 4)()
        tr = ctypes.c_int64()
        self._rc(lib().dg_profile_read(self._h, ms, n, ctypes.byref(tr), 1 if reset else 0), "dg_profile_read")
        return {k: (ms[i], n[i]) for i, k in enumerate(PROF_KINDS)}, tr.value


def problem_from_workload(wl, device="cuda", **over):
    kw = dict(dim=wl.dim, equation=wl.equation, order=wl.order, nx=wl.nx, ny=wl.ny, x0=wl.x0, x1=wl.x1,
              y0=wl.y0, y1=wl.y1, bc=tuple(wl.bc), gamma=wl.gamma, cfl=wl.cfl)
    kw.update(wl.bc_extra)
    kw.update(wl.mesh)
    kw.update(over)
    return Problem(device=device, **kw)


def initial_state(prob, wl, limit=True, rows_per_chunk=None, state=None):
    """Project the workload's initial data (evaluated at this library's nodes)
    and apply the limiter once."""
    r, _ = prob.proj_nodes()
    state = prob.empty_state() if state is None else state
    if prob.dim == 2 and wl.point_values_device(r, 0, 1, prob.device) is not None:
        nq = len(r)
        rows = rows_per_chunk or max(1, min(prob.ny, (1 << 30) // (prob.nv * nq * nq * prob.nx * 8)))
        for j0 in range(0, prob.ny, rows):
            nr = min(rows, prob.ny - j0)
            prob.project(wl.point_values_device(r, j0, nr, prob.device), state, j0=j0)
    elif prob.dim == 1:
        pv = torch.from_numpy(wl.point_values(r)).to(prob.device)
        prob.project(pv, state)
    else:
        nq = len(r)
        per_row = prob.nv * nq * nq * prob.nx * 8
        rows = rows_per_chunk or max(1, min(prob.ny, (1 << 30) // per_row))
        for j0 in range(0, prob.ny, rows):
            nr = min(rows, prob.ny - j0)
            pv = torch.from_numpy(wl.point_values(r, j0, nr)).to(prob.device)
            prob.project(pv, state, j0=j0)
            del pv
    if limit:
        prob.limit(state, want_margin=False)
    return state


class Batch:
    """Independent 2D Euler problems of any sizes and orders advanced together
    (dg_batch_*): one states buffer holds every instance at 32-element aligned
    offsets; `view(i)` is instance i's [4][(N+1)^2][ny][nx] state."""

    def __init__(self, cfgs, device="cuda", stream=None):
        import numpy as np
        self.n = len(cfgs)
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.cfgs = [dict(c) for c in cfgs]
        arr = (Config * self.n)(*[make_config(**c) for c in cfgs])
        self._cfg_arr = arr
        self.shapes = []
        offs, o = [], 0
        for c in arr:
            shp = (4, (c.order + 1) ** 2, c.ny, c.nx)
            self.shapes.append(shp)
            offs.append(o)
            o += (int(np.prod(shp)) + 31) // 32 * 32
        self.offsets = np.array(offs, dtype=np.int64)
        self._off_c = (ctypes.c_int64 * self.n)(*offs)
        nbytes = ctypes.c_size_t()
        rc = lib().dg_batch_workspace_bytes(arr, self.n, ctypes.byref(nbytes))
        if rc:
            raise DGError(rc, "dg_batch_workspace_bytes")
        with torch.cuda.device(self.device):
            self.states = torch.zeros(max(o, 1), dtype=torch.float64, device=self.device)
            self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            handle = ctypes.c_void_p()
            rc = lib().dg_batch_init(arr, self.n, ctypes.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle))
        if rc:
            raise DGError(rc, "dg_batch_init")
        self._h = handle
        self._learned = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().dg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def view(self, i):
        import numpy as np
        shp = self.shapes[i]
        o = int(self.offsets[i])
        return self.states[o:o + int(np.prod(shp))].view(shp)

    def dofs(self, active=None):
        import numpy as np
        idx = range(self.n) if active is None else [i for i in range(self.n) if active[i]]
        return int(sum(np.prod(self.shapes[i]) for i in idx))

    def autotune(self):
        """{order: (rows, tiles, ms)} of the orders present."""
        rows = (ctypes.c_int32 * 4)()
        tiles = (ctypes.c_int32 * 4)()
        ms = (ctypes.c_float * 4)()
        rc = lib().dg_batch_autotune(self._h, _ptr(self.states), self._off_c, rows, tiles, ms)
        if rc:
            raise DGError(rc, "dg_batch_autotune")
        return {o: (rows[o], tiles[o], ms[o]) for o in range(1, 4) if rows[o]}

    def set_tiles(self, order, rows):
        rc = lib().dg_batch_set_tiles(self._h, int(order), int(rows))
        if rc:
            raise DGError(rc, "dg_batch_set_tiles")

    def set_learned(self, order, w_bf16, master, band=(0.2, 0.8), prob=None):
        """prob: optional float tensor with as many elements as `states`;
        every indicator pass writes p of instance i's cell c at
        prob[offsets[i] + c]."""
        self._learned[order] = (w_bf16, master, prob)  # the library keeps the pointers
        rc = lib().dg_batch_set_learned(self._h, int(order), _ptr(w_bf16), _ptr(master), float(band[0]),
                                        float(band[1]), _ptr(prob) if prob is not None else None)
        if rc:
            raise DGError(rc, "dg_batch_set_learned")

    def step(self, t, t_end, max_steps=2**31 - 1, allow_nonphysical=False):
        """Advance every instance from t[i] towards t_end[i] (sequences or
        scalars); returns (t, steps, status, troubled) as numpy arrays and an
        int."""
        import numpy as np
        tv = np.broadcast_to(np.asarray(t, dtype=np.float64), (self.n,)).copy()
        te = np.broadcast_to(np.asarray(t_end, dtype=np.float64), (self.n,)).copy()
        tc = (ctypes.c_double * self.n)(*tv)
        tec = (ctypes.c_double * self.n)(*te)
        steps = (ctypes.c_int32 * self.n)()
        status = (ctypes.c_int32 * self.n)()
        tr = ctypes.c_int64()
        rc = lib().dg_batch_step(self._h, _ptr(self.states), self._off_c, tc, tec, int(max_steps), steps, status,
                                 ctypes.byref(tr))
        if rc and not (rc == DG_ERR_NONPHYSICAL and allow_nonphysical):
            raise DGError(rc, "dg_batch_step")
        return (np.array(tc[:]), np.array(steps[:], dtype=np.int64), np.array(status[:], dtype=np.int64),
                tr.value)


def batch_from_workloads(wls, device="cuda", limit=True, **over):
    """A Batch of 2D Euler workloads with each instance's initial state
    projected (and limited) through a single-mesh problem of the same
    configuration."""
    cfgs = []
    for wl in wls:
        kw = dict(dim=2, equation=wl.equation, order=wl.order, nx=wl.nx, ny=wl.ny, x0=wl.x0, x1=wl.x1,
                  y0=wl.y0, y1=wl.y1, bc=tuple(wl.bc), gamma=wl.gamma, cfl=wl.cfl)
        kw.update(wl.bc_extra)
        kw.update(over)
        cfgs.append(kw)
    b = Batch(cfgs, device=device)
    for i, wl in enumerate(wls):
        p = Problem(device=device, **cfgs[i])
        initial_state(p, wl, limit=limit, state=b.view(i))
        p.close()
        del p
    torch.cuda.synchronize(b.device)
    return b

