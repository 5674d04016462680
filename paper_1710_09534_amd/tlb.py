"""ctypes binding of ``libtlb.so`` (C ABI in include/tlb.h).

Argument marshalling only: every step of the solver runs in the HIP
library.  PyTorch provides the device workspace and the stream.  Importing
this module raises if the library has not been built -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime before libtlb binds to it)

_HERE = os.path.dirname(os.path.abspath(__file__))
# TLB_LIBRARY selects another build of the same library (the host-sanitized one)
LIB_PATH = os.environ.get("TLB_LIBRARY") or os.path.join(_HERE, "libtlb.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("%s is not built: run python -m paper_1710_09534_amd.build" % LIB_PATH)

TLB_OK, TLB_EINVAL, TLB_EPARAM, TLB_ENOMEM, TLB_EDEVICE, TLB_EDIVERGED, TLB_ESTATE, TLB_EBUSY = (
    0, -1, -2, -3, -4, -5, -6, -7)
TLB_FP64, TLB_FP32, TLB_FP16DEV = 0, 1, 2
PRECISIONS = {"fp64": TLB_FP64, "fp32": TLB_FP32, "fp16dev": TLB_FP16DEV}
FIELDS = ("c1", "c2", "c3", "rho", "ux", "uy", "p", "mu1", "mu2", "mu3")
F_ALL = (1 << len(FIELDS)) - 1


class TlbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("tlb status %d: %s" % (status, msg))
        self.status = status


class tlb_fluid(C.Structure):
    _fields_ = [("sigma12", C.c_double), ("sigma13", C.c_double), ("sigma23", C.c_double),
                ("D", C.c_double), ("M0", C.c_double), ("tau1", C.c_double),
                ("tau2", C.c_double), ("rho", C.c_double * 3), ("nu", C.c_double * 3),
                ("gravity", C.c_double * 2), ("lambda_", C.c_double)]


class tlb_material(C.Structure):
    _fields_ = [("theta13_deg", C.c_double), ("theta23_deg", C.c_double),
                ("wall_u", C.c_double * 2), ("kind", C.c_int)]


TLB_WALL, TLB_VELOCITY = 0, 1


class tlb_request(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("fluid", tlb_fluid),
                ("periodic_x", C.c_int), ("periodic_y", C.c_int),
                ("material", C.POINTER(C.c_uint8)), ("mats", C.POINTER(tlb_material)),
                ("n_mats", C.c_int), ("c1", C.POINTER(C.c_double)), ("c2", C.POINTER(C.c_double)),
                ("ux", C.POINTER(C.c_double)), ("uy", C.POINTER(C.c_double)),
                ("nsteps", C.c_int64), ("result_fields", C.c_uint32)]


class tlb_server_counters(C.Structure):
    _fields_ = [("completed", C.c_int64), ("failed", C.c_int64), ("queued", C.c_int64),
                ("running", C.c_int64), ("busy_seconds", C.c_double),
                ("node_steps", C.c_double), ("arena_free_largest", C.c_size_t)]


TLB_REQ_QUEUED, TLB_REQ_RUNNING, TLB_REQ_DONE, TLB_REQ_FAILED, TLB_REQ_CANCELLED = range(5)

lib = C.CDLL(LIB_PATH)
_vp = C.c_void_p
_D = C.POINTER(C.c_double)
_SIGS = {
    "tlb_workspace_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int]),
    "tlb_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(tlb_fluid), _vp, C.c_size_t,
                             _vp, C.POINTER(_vp)]),
    "tlb_set_geometry": (C.c_int, [_vp, C.c_int, C.c_int, C.POINTER(C.c_uint8),
                                   C.POINTER(tlb_material), C.c_int, _D]),
    "tlb_init_fields": (C.c_int, [_vp, _D, _D, _D, _D]),
    "tlb_step": (C.c_int, [_vp, C.c_int64]),
    "tlb_set_check_interval": (C.c_int, [_vp, C.c_int64]),
    "tlb_step_count": (C.c_int64, [_vp]),
    "tlb_read_fields": (C.c_int, [_vp, C.c_uint32, _D]),
    "tlb_read_populations": (C.c_int, [_vp, _D]),
    "tlb_mass": (C.c_int, [_vp, _D]),
    "tlb_mass_noalloc": (C.c_int, [_vp, _vp]),
    "tlb_checkpoint_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "tlb_checkpoint_save": (C.c_int, [_vp, _vp]),
    "tlb_checkpoint_load": (C.c_int, [_vp, _vp]),
    "tlb_time_steps": (C.c_int, [_vp, C.c_int64, _D]),
    "tlb_probe_bandwidth": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_size_t,
                                      _vp, C.c_int, _D]),
    "tlb_set_tile_rows": (C.c_int, [_vp, C.c_int]),
    "tlb_set_pair_rows": (C.c_int, [_vp, C.c_int]),
    "tlb_autotune_rows": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_int)]),
    "tlb_batch_table_bytes": (C.c_size_t, [C.c_int]),
    "tlb_batch_create": (C.c_int, [C.c_int, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "tlb_batch_set": (C.c_int, [_vp, C.POINTER(_vp), C.c_int]),
    "tlb_batch_use_graph": (C.c_int, [_vp, C.c_int]),
    "tlb_batch_step": (C.c_int, [_vp, C.c_int64]),
    "tlb_batch_autotune_rows": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_int)]),
    "tlb_batch_autotune_pair_rows": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_int)]),
    "tlb_batch_sync": (C.c_int, [_vp]),
    "tlb_batch_set_pair_rows": (C.c_int, [_vp, C.c_int]),
    "tlb_batch_last_error": (C.c_char_p, [_vp]),
    "tlb_batch_destroy": (None, [_vp]),
    "tlb_server_set_check_steps": (C.c_int, [_vp, C.c_int64]),
    "tlb_server_create": (C.c_int, [_vp, C.c_size_t, C.c_int, C.c_int, C.c_int64, _vp,
                                    C.POINTER(_vp)]),
    "tlb_server_submit": (C.c_int, [_vp, C.POINTER(tlb_request), C.POINTER(C.c_uint64)]),
    "tlb_server_poll": (C.c_int, [_vp, C.c_uint64, C.POINTER(C.c_int)]),
    "tlb_server_wait": (C.c_int, [_vp, C.c_uint64, C.c_double]),
    "tlb_server_result": (C.c_int, [_vp, C.c_uint64, C.c_uint32, _D, _D]),
    "tlb_server_release": (C.c_int, [_vp, C.c_uint64]),
    "tlb_server_cancel": (C.c_int, [_vp, C.c_uint64]),
    "tlb_server_stats": (C.c_int, [_vp, C.POINTER(tlb_server_counters)]),
    "tlb_server_last_error": (C.c_char_p, [_vp]),
    "tlb_server_destroy": (None, [_vp]),
    "tlb_last_error": (C.c_char_p, [_vp]),
    "tlb_destroy": (None, [_vp]),
    # three-dimensional (D3Q19) step, include/tlb3d.h
    "tlb3_workspace_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int]),
    "tlb3_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(tlb_fluid),
                              C.c_double, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "tlb3_set_geometry": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_uint8),
                                    C.POINTER(tlb_material), C.c_int, _D]),
    "tlb3_init_fields": (C.c_int, [_vp, _D, _D, _D, _D, _D]),
    "tlb3_step": (C.c_int, [_vp, C.c_int64]),
    "tlb3_set_check_interval": (C.c_int, [_vp, C.c_int64]),
    "tlb3_read_fields": (C.c_int, [_vp, C.c_uint32, _D]),
    "tlb3_read_populations": (C.c_int, [_vp, _D]),
    "tlb3_mass": (C.c_int, [_vp, _D]),
    "tlb3_time_steps": (C.c_int, [_vp, C.c_int64, _D]),
    "tlb3_last_error": (C.c_char_p, [_vp]),
    "tlb3_destroy": (None, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def tlb_last_error(ctx=None) -> str:
    return lib.tlb_last_error(ctx).decode()


def _check(status, ctx=None):
    if status != TLB_OK:
        raise TlbError(status, tlb_last_error(ctx))


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


def make_fluid(fl: dict) -> tlb_fluid:
    f = tlb_fluid()
    f.sigma12, f.sigma13, f.sigma23 = fl["sigma12"], fl["sigma13"], fl["sigma23"]
    f.D, f.M0, f.tau1, f.tau2 = fl["D"], fl["M0"], fl["tau1"], fl["tau2"]
    for i in range(3):
        f.rho[i] = fl["rho"][i]
        f.nu[i] = fl["nu"][i]
    g = fl.get("gravity", (0.0, 0.0))
    f.gravity[0], f.gravity[1] = g[0], g[1]
    f.lambda_ = float(fl.get("lambda", 0.0))
    return f


def make_materials(mats):
    arr = (tlb_material * max(1, len(mats)))()
    for i, m in enumerate(mats):
        arr[i].theta13_deg = m["theta13"]
        arr[i].theta23_deg = m["theta23"]
        wu = m.get("wall_u", (0.0, 0.0))
        arr[i].wall_u[0], arr[i].wall_u[1] = wu[0], wu[1]
        arr[i].kind = int(m.get("kind", TLB_WALL))
    return arr


def tlb_workspace_bytes(nx: int, ny: int, precision: int) -> int:
    return int(lib.tlb_workspace_bytes(nx, ny, precision))


class Solver:
    """One lattice on the current HIP device: owns a torch workspace and the
    C context.  Method names follow the C ABI (tlb_<name>)."""

    def __init__(self, nx, ny, fluid: dict, precision="fp64", device="cuda:0", stream=None):
        import torch
        self.nx, self.ny = int(nx), int(ny)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.device = torch.device(device)
        nbytes = tlb_workspace_bytes(self.nx, self.ny, self.precision)
        if nbytes == 0:
            raise TlbError(TLB_EINVAL, "bad lattice size")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._fluid = make_fluid(fluid)
        h = _vp()
        st = lib.tlb_create(self.nx, self.ny, self.precision, C.byref(self._fluid),
                            _vp(self.workspace.data_ptr()), nbytes,
                            _vp(self.stream.cuda_stream), C.byref(h))
        _check(st, None)
        self.ctx = h

    def __del__(self):
        self.destroy()

    def destroy(self, _lib=lib):
        # _lib is bound at definition time: module globals may already be
        # cleared when this runs during interpreter shutdown
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            _lib.tlb_destroy(ctx)
        self.ctx = None

    @property
    def n(self):
        return self.nx * self.ny

    def _f(self, a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != (self.ny, self.nx):
            raise ValueError("field shape %s != %s" % (a.shape, (self.ny, self.nx)))
        return a

    def set_geometry(self, material, mats, periodic=(1, 1)):
        material = np.ascontiguousarray(material, dtype=np.uint8)
        if material.shape != (self.ny, self.nx):
            raise ValueError("material shape mismatch")
        arr = make_materials(mats)
        th12 = np.zeros(max(1, len(mats)))
        st = lib.tlb_set_geometry(self.ctx, int(periodic[0]), int(periodic[1]),
                                  material.ctypes.data_as(C.POINTER(C.c_uint8)), arr, len(mats),
                                  _dp(th12))
        _check(st, self.ctx)
        return th12[:len(mats)]

    def init_fields(self, c1, c2, ux=None, uy=None):
        c1, c2, ux, uy = (self._f(a) for a in (c1, c2, ux, uy))
        _check(lib.tlb_init_fields(self.ctx, _dp(c1), _dp(c2), _dp(ux), _dp(uy)), self.ctx)

    def step(self, n: int = 1):
        _check(lib.tlb_step(self.ctx, int(n)), self.ctx)

    def set_check_interval(self, n: int):
        _check(lib.tlb_set_check_interval(self.ctx, int(n)), self.ctx)

    def set_tile_rows(self, rows: int):
        _check(lib.tlb_set_tile_rows(self.ctx, int(rows)), self.ctx)

    def set_pair_rows(self, rows: int):
        _check(lib.tlb_set_pair_rows(self.ctx, int(rows)), self.ctx)

    @property
    def step_count(self) -> int:
        return int(lib.tlb_step_count(self.ctx))

    def read_fields(self, mask: int = F_ALL) -> dict:
        names = [f for i, f in enumerate(FIELDS) if mask & (1 << i)]
        out = np.zeros((len(names), self.ny, self.nx))
        _check(lib.tlb_read_fields(self.ctx, mask, _dp(out)), self.ctx)
        return {k: out[i] for i, k in enumerate(names)}

    def read_populations(self) -> np.ndarray:
        out = np.zeros((27, self.ny, self.nx))
        _check(lib.tlb_read_populations(self.ctx, _dp(out)), self.ctx)
        return out

    def mass(self) -> np.ndarray:
        out = np.zeros(3)
        _check(lib.tlb_mass(self.ctx, _dp(out)), self.ctx)
        return out

    def mass_noalloc(self, dev_out):
        """Enqueue the mass sums into dev_out (a float64 device tensor of 4
        elements: sum c1, c2, c3, non-finite count) without synchronizing."""
        import torch
        if dev_out.dtype != torch.float64 or dev_out.numel() < 4 or not dev_out.is_cuda:
            raise ValueError("dev_out must be a float64 device tensor of at least 4 elements")
        _check(lib.tlb_mass_noalloc(self.ctx, C.c_void_p(dev_out.data_ptr())), self.ctx)

    def checkpoint_save(self) -> bytes:
        n = C.c_size_t()
        _check(lib.tlb_checkpoint_bytes(self.ctx, C.byref(n)), self.ctx)
        buf = C.create_string_buffer(n.value)
        _check(lib.tlb_checkpoint_save(self.ctx, buf), self.ctx)
        return buf.raw

    def checkpoint_load(self, blob: bytes):
        n = C.c_size_t()
        _check(lib.tlb_checkpoint_bytes(self.ctx, C.byref(n)), self.ctx)
        if len(blob) != n.value:   # the library reads exactly that many bytes
            raise ValueError("checkpoint of %d bytes for a context that takes %d"
                             % (len(blob), n.value))
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib.tlb_checkpoint_load(self.ctx, buf), self.ctx)

    def time_steps(self, n: int) -> float:
        ms = C.c_double()
        _check(lib.tlb_time_steps(self.ctx, int(n), C.byref(ms)), self.ctx)
        return ms.value

    def autotune_rows(self, steps_per_candidate: int = 20) -> int:
        best = C.c_int()
        _check(lib.tlb_autotune_rows(self.ctx, int(steps_per_candidate), C.byref(best)), self.ctx)
        return best.value


def probe_bandwidth(kind: int, src, dst, nx: int = 0, ny: int = 0, tile_rows: int = 64,
                    reps: int = 10, stream=None) -> float:
    """Average ms per launch of a streaming reference (kind 0: 16-byte copy of
    src to dst; kind 1: the step kernel's 31-plane FP32 access shape on an
    nx x ny lattice); src, dst: torch device tensors."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    ms = C.c_double()
    nbytes = min(src.numel() * src.element_size(), dst.numel() * dst.element_size())
    _check(lib.tlb_probe_bandwidth(int(kind), int(nx), int(ny), int(tile_rows),
                                   C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                   nbytes, C.c_void_p(st.cuda_stream), int(reps), C.byref(ms)))
    return ms.value


class Batch:
    """Independent lattices advanced by shared step launches (tlb_batch_*)."""

    def __init__(self, max_lattices: int, device="cuda:0", stream=None):
        import torch
        nbytes = int(lib.tlb_batch_table_bytes(int(max_lattices)))
        self.table = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        # a stream of its own (default priority): graph capture needs a
        # non-default stream; call sync() before using members on their own
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        h = _vp()
        st = lib.tlb_batch_create(int(max_lattices), _vp(self.table.data_ptr()), nbytes,
                                  _vp(self.stream.cuda_stream), C.byref(h))
        if st != TLB_OK:
            raise TlbError(st, lib.tlb_batch_last_error(None).decode())
        self.h = h
        self.members = []

    def _check(self, st):
        if st != TLB_OK:
            raise TlbError(st, lib.tlb_batch_last_error(self.h).decode())

    def set(self, solvers):
        arr = (_vp * max(1, len(solvers)))(*[s.ctx for s in solvers])
        self._check(lib.tlb_batch_set(self.h, arr, len(solvers)))
        self.members = list(solvers)

    def use_graph(self, steps: int):
        self._check(lib.tlb_batch_use_graph(self.h, int(steps)))

    def set_pair_rows(self, rows: int):
        self._check(lib.tlb_batch_set_pair_rows(self.h, int(rows)))

    def step(self, n: int):
        self._check(lib.tlb_batch_step(self.h, int(n)))

    def autotune_rows(self, steps_per_candidate: int = 20) -> int:
        best = C.c_int()
        self._check(lib.tlb_batch_autotune_rows(self.h, int(steps_per_candidate), C.byref(best)))
        return best.value

    def autotune_pair_rows(self, steps_per_candidate: int = 20) -> int:
        best = C.c_int()
        self._check(lib.tlb_batch_autotune_pair_rows(self.h, int(steps_per_candidate),
                                                     C.byref(best)))
        return best.value

    def sync(self):
        self._check(lib.tlb_batch_sync(self.h))

    def __del__(self, _lib=lib):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            _lib.tlb_batch_destroy(h)
            self.h = None


FIELDS3 = ("c1", "c2", "c3", "rho", "ux", "uy", "uz", "p", "mu1", "mu2", "mu3")


class Solver3D:
    """One three-dimensional (D3Q19) lattice on the current HIP device:
    owns a torch workspace and the C context (tlb3_*)."""

    def __init__(self, nx: int, ny: int, nz: int, fluid: dict, precision="fp64",
                 device="cuda:0"):
        import torch
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        nbytes = int(lib.tlb3_workspace_bytes(self.nx, self.ny, self.nz, self.precision))
        if nbytes == 0:
            raise TlbError(TLB_EINVAL, "unsupported size or precision for the 3-D step")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(device)
        self._fluid = make_fluid(fluid)
        h = _vp()
        st = lib.tlb3_create(self.nx, self.ny, self.nz, self.precision, C.byref(self._fluid),
                             float(fluid.get("gravity_z", 0.0)), _vp(self.workspace.data_ptr()),
                             nbytes, _vp(self.stream.cuda_stream), C.byref(h))
        if st != TLB_OK:
            raise TlbError(st, lib.tlb3_last_error(None).decode())
        self.ctx = h

    def __del__(self):
        self.destroy()

    def destroy(self, _lib=lib):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            _lib.tlb3_destroy(ctx)
        self.ctx = None

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    def _check(self, st):
        if st != TLB_OK:
            raise TlbError(st, lib.tlb3_last_error(self.ctx).decode())

    def _f(self, a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
        if a.size != self.n:
            raise ValueError("field size mismatch")
        return a

    def set_geometry(self, material, mats, periodic=(1, 1, 1)):
        material = np.ascontiguousarray(material, dtype=np.uint8)
        if material.shape != (self.nz, self.ny, self.nx):
            raise ValueError("material shape mismatch")
        arr = make_materials(mats)
        th12 = np.zeros(max(1, len(mats)))
        self._check(lib.tlb3_set_geometry(self.ctx, int(periodic[0]), int(periodic[1]),
                                          int(periodic[2]),
                                          material.ctypes.data_as(C.POINTER(C.c_uint8)), arr,
                                          len(mats), _dp(th12)))
        return th12[:len(mats)]

    def init_fields(self, c1, c2, ux=None, uy=None, uz=None):
        a = [self._f(v) for v in (c1, c2, ux, uy, uz)]
        self._check(lib.tlb3_init_fields(self.ctx, *[_dp(v) for v in a]))

    def step(self, n: int = 1):
        self._check(lib.tlb3_step(self.ctx, int(n)))

    def set_check_interval(self, n: int):
        self._check(lib.tlb3_set_check_interval(self.ctx, int(n)))

    def read_fields(self, names=FIELDS3) -> dict:
        mask = 0
        for nm in names:
            mask |= 1 << FIELDS3.index(nm)
        order = [nm for nm in FIELDS3 if mask & (1 << FIELDS3.index(nm))]
        out = np.zeros(len(order) * self.n)
        self._check(lib.tlb3_read_fields(self.ctx, mask, _dp(out)))
        shape = (self.nz, self.ny, self.nx)
        return {nm: out[i * self.n:(i + 1) * self.n].reshape(shape) for i, nm in enumerate(order)}

    def read_populations(self) -> np.ndarray:
        out = np.zeros(57 * self.n)
        self._check(lib.tlb3_read_populations(self.ctx, _dp(out)))
        return out.reshape(57, self.nz, self.ny, self.nx)

    def mass(self) -> np.ndarray:
        out = np.zeros(3)
        self._check(lib.tlb3_mass(self.ctx, _dp(out)))
        return out

    def time_steps(self, n: int) -> float:
        ms = C.c_double()
        self._check(lib.tlb3_time_steps(self.ctx, int(n), C.byref(ms)))
        return ms.value


def from_problem3(problem: dict, precision="fp64", device="cuda:0", init=True) -> Solver3D:
    """Creates a 3-D solver for a problem dict of ``workloads`` (``*3d``,
    ``random_fields3``) and initialises it."""
    s = Solver3D(problem["nx"], problem["ny"], problem["nz"], problem["fluid"], precision, device)
    s.set_geometry(problem["material"], problem["mats"], problem.get("periodic", (1, 1, 1)))
    if init:
        s.init_fields(problem["c1"], problem["c2"], problem.get("ux"), problem.get("uy"),
                      problem.get("uz"))
    return s


def from_problem(problem: dict, precision="fp64", device="cuda:0", init=True) -> Solver:
    """Creates a solver for a problem dict of ``workloads`` and initialises it."""
    s = Solver(problem["nx"], problem["ny"], problem["fluid"], precision, device)
    s.set_geometry(problem["material"], problem["mats"], problem.get("periodic", (1, 1)))
    if init:
        s.init_fields(problem["c1"], problem["c2"], problem.get("ux"), problem.get("uy"))
    return s


class Server:
    """Continuous-batching solve server (tlb_server_*).  The arena (a torch
    uint8 tensor of arena_bytes) is the server's whole device budget."""

    def __init__(self, arena_bytes: int, max_slots: int, precision="fp32", quantum=200,
                 device="cuda:0"):
        import torch
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self.stream = torch.cuda.Stream(device=device)
        h = _vp()
        st = lib.tlb_server_create(_vp(self.arena.data_ptr()), int(arena_bytes), int(max_slots),
                                   self.precision, int(quantum), _vp(self.stream.cuda_stream),
                                   C.byref(h))
        if st != TLB_OK:
            raise TlbError(st, lib.tlb_server_last_error(None).decode())
        self.h = h
        self._size = {}   # request id -> (nx, ny): the library writes that many nodes per field

    def set_check_steps(self, steps: int):
        self._check(lib.tlb_server_set_check_steps(self.h, int(steps)))

    def _check(self, st):
        if st != TLB_OK:
            raise TlbError(st, lib.tlb_server_last_error(self.h).decode())

    def submit(self, problem: dict, nsteps: int, fields: int = F_ALL) -> int:
        nx, ny = int(problem["nx"]), int(problem["ny"])
        keep = []

        def arr(a, dtype=np.float64):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dtype)
            if a.shape != (ny, nx):
                raise ValueError("array of shape %s for a %d x %d lattice" % (a.shape, nx, ny))
            keep.append(a)
            return a

        mat = arr(problem["material"], np.uint8)
        c1, c2 = arr(problem["c1"]), arr(problem["c2"])
        ux, uy = arr(problem.get("ux")), arr(problem.get("uy"))
        mats = make_materials(problem["mats"])
        r = tlb_request()
        r.nx, r.ny = nx, ny
        r.fluid = make_fluid(problem["fluid"])
        px, py = problem.get("periodic", (1, 1))
        r.periodic_x, r.periodic_y = int(px), int(py)
        r.material = mat.ctypes.data_as(C.POINTER(C.c_uint8))
        r.mats = mats
        r.n_mats = len(problem["mats"])
        r.c1, r.c2 = _dp(c1), _dp(c2)
        r.ux, r.uy = _dp(ux), _dp(uy)
        r.nsteps = int(nsteps)
        r.result_fields = int(fields)
        rid = C.c_uint64()
        self._check(lib.tlb_server_submit(self.h, C.byref(r), C.byref(rid)))
        self._size[rid.value] = (nx, ny)
        return rid.value

    def poll(self, rid: int) -> int:
        st = C.c_int()
        self._check(lib.tlb_server_poll(self.h, rid, C.byref(st)))
        return st.value

    def wait(self, rid: int, timeout: float = -1.0):
        self._check(lib.tlb_server_wait(self.h, rid, float(timeout)))

    def result(self, rid: int, nx: int = None, ny: int = None, mask: int = F_ALL):
        """Fields of a finished request; nx, ny, if given, must be its size."""
        if rid not in self._size:
            raise TlbError(TLB_EINVAL, "unknown request id")
        snx, sny = self._size[rid]
        if (nx is not None and nx != snx) or (ny is not None and ny != sny):
            raise ValueError("request %d is %d x %d, not %s x %s" % (rid, snx, sny, nx, ny))
        names = [f for i, f in enumerate(FIELDS) if mask & (1 << i)]
        out = np.zeros((len(names), sny, snx))
        lat = C.c_double()
        self._check(lib.tlb_server_result(self.h, rid, mask, _dp(out), C.byref(lat)))
        return {k: out[i] for i, k in enumerate(names)}, lat.value

    def latency(self, rid: int) -> float:
        lat = C.c_double()
        self._check(lib.tlb_server_result(self.h, rid, 0, None, C.byref(lat)))
        return lat.value

    def release(self, rid: int):
        self._check(lib.tlb_server_release(self.h, rid))
        self._size.pop(rid, None)

    def cancel(self, rid: int):
        self._check(lib.tlb_server_cancel(self.h, rid))

    def stats(self) -> dict:
        c = tlb_server_counters()
        self._check(lib.tlb_server_stats(self.h, C.byref(c)))
        return {f: getattr(c, f) for f, _ in tlb_server_counters._fields_}

    def close(self, _lib=lib):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            _lib.tlb_server_destroy(h)
            self.h = None

    def __del__(self):
        self.close()
