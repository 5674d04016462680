"""ctypes marshalling for the C oracle in ``tlb_oracle.c`` (test infrastructure
only: see the package docstring).  No arithmetic of the method lives here."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tlb_oracle.c")
_SRC3 = os.path.join(_HERE, "tlb3d_oracle.c")
_LIB = os.path.join(_HERE, "libtlb_oracle.so")

FIELDS = ("c1", "c2", "c3", "rho", "ux", "uy", "p", "mu1", "mu2", "mu3")
STAGES = ("lapc1", "lapc2", "lapc3", "gc1x", "gc1y", "gc2x", "gc2y", "gc3x", "gc3y",
          "grx", "gry", "lapmu1", "lapmu2", "fsx", "fsy", "fax", "fay", "taug", "nu",
          "d1x", "d1y", "d2x", "d2y")

_lock = threading.Lock()
_lib = None


def library_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, FP64, no FMA contraction)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, _SRC3, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Fluid(C.Structure):
    _fields_ = [("sigma12", C.c_double), ("sigma13", C.c_double), ("sigma23", C.c_double),
                ("D", C.c_double), ("M0", C.c_double), ("tau1", C.c_double),
                ("tau2", C.c_double), ("rho", C.c_double * 3), ("nu", C.c_double * 3),
                ("gravity", C.c_double * 2), ("lambda_", C.c_double)]


class _Material(C.Structure):
    _fields_ = [("theta13_deg", C.c_double), ("theta23_deg", C.c_double),
                ("wall_u", C.c_double * 2), ("kind", C.c_int)]


class _Derived(C.Structure):
    _fields_ = [("lambda_", C.c_double * 3), ("lambdaT", C.c_double),
                ("M", C.c_double * 2), ("eta", C.c_double * 2)]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
                os.path.getmtime(_SRC), os.path.getmtime(_SRC3)):
            build()
        lib = C.CDLL(_LIB)
        D = C.POINTER(C.c_double)
        vp = C.c_void_p
        sig = {
            "orc_lattice": (None, [C.POINTER(C.c_int), C.POINTER(C.c_int), D, C.POINTER(C.c_int)]),
            "orc_params": (C.c_int, [C.POINTER(_Fluid), C.POINTER(_Derived)]),
            "orc_cos12": (C.c_int, [C.POINTER(_Fluid), C.c_double, C.c_double, D]),
            "orc_wetting_ghost": (None, [C.c_double] * 6 + [D]),
            "orc_chem_potential": (None, [C.POINTER(_Fluid)] + [C.c_double] * 5 + [D]),
            "orc_equilibria": (None, [C.c_double] * 10 + [D, D, D]),
            "orc_sources": (None, [C.c_double] * 15 + [D, D, D]),
            "orc_create": (C.c_int, [C.c_int, C.c_int, C.POINTER(_Fluid), C.c_int, C.c_int,
                                     C.POINTER(C.c_uint8), C.POINTER(_Material), C.c_int,
                                     C.POINTER(vp)]),
            "orc_destroy": (None, [vp]),
            "orc_last_error": (C.c_char_p, []),
            "orc_init": (C.c_int, [vp, D, D, D, D]),
            "orc_eval": (C.c_int, [vp]),
            "orc_step": (C.c_int, [vp, C.c_int]),
            "orc_fields": (C.c_int, [vp, D]),
            "orc_stage": (C.c_int, [vp, C.c_int, D]),
            "orc_populations": (C.c_int, [vp, D]),
            "orc_set_populations": (C.c_int, [vp, D]),
            "orc_history": (C.c_int, [vp, D]),
            "orc_mass": (C.c_int, [vp, D]),
            "orc_grad_field": (C.c_int, [vp, D, D, D]),
            "orc_lap_field": (C.c_int, [vp, D, D]),
            "orc_num_threads": (C.c_int, []),
            "orc3_lattice": (None, [C.POINTER(C.c_int)] * 3 + [D, C.POINTER(C.c_int)]),
            "orc3_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(_Fluid), C.c_double,
                                      C.c_int, C.c_int, C.c_int, C.POINTER(C.c_uint8),
                                      C.POINTER(_Material), C.c_int, C.POINTER(vp)]),
            "orc3_destroy": (None, [vp]),
            "orc3_last_error": (C.c_char_p, []),
            "orc3_init": (C.c_int, [vp, D, D, D, D, D]),
            "orc3_eval": (C.c_int, [vp]),
            "orc3_step": (C.c_int, [vp, C.c_int]),
            "orc3_fields": (C.c_int, [vp, D]),
            "orc3_populations": (C.c_int, [vp, D]),
            "orc3_mass": (C.c_int, [vp, D]),
            "orc3_grad_field": (C.c_int, [vp, D, D, D, D]),
            "orc3_lap_field": (C.c_int, [vp, D, D]),
            "orc_set_num_threads": (None, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _fluid(fl: dict) -> _Fluid:
    f = _Fluid()
    f.sigma12, f.sigma13, f.sigma23 = fl["sigma12"], fl["sigma13"], fl["sigma23"]
    f.D, f.M0, f.tau1, f.tau2 = fl["D"], fl["M0"], fl["tau1"], fl["tau2"]
    for i in range(3):
        f.rho[i] = fl["rho"][i]
        f.nu[i] = fl["nu"][i]
    g = fl.get("gravity", (0.0, 0.0))
    f.gravity[0], f.gravity[1] = g[0], g[1]
    f.lambda_ = float(fl.get("lambda", 0.0))
    return f


# ------------------------------------------------------------ pure functions
def lattice():
    lib = _load()
    ex = (C.c_int * 9)()
    ey = (C.c_int * 9)()
    w = np.zeros(9)
    opp = (C.c_int * 9)()
    lib.orc_lattice(ex, ey, _dp(w), opp)
    return np.array(ex[:]), np.array(ey[:]), w, np.array(opp[:])


def params(fl: dict):
    lib = _load()
    d = _Derived()
    rc = lib.orc_params(C.byref(_fluid(fl)), C.byref(d))
    return {"lambda": np.array(d.lambda_[:]), "lambdaT": d.lambdaT, "M": np.array(d.M[:]),
            "eta": np.array(d.eta[:]), "admissible": rc == 0}


def cos12(fl: dict, theta13_deg: float, theta23_deg: float):
    lib = _load()
    out = C.c_double()
    rc = lib.orc_cos12(C.byref(_fluid(fl)), theta13_deg, theta23_deg, C.byref(out))
    return out.value, rc == 0


def wetting_ghost(D, cos12_, cos13, cos23, c1, c2):
    lib = _load()
    out = np.zeros(3)
    lib.orc_wetting_ghost(D, cos12_, cos13, cos23, c1, c2, _dp(out))
    return out


def chem_potential(fl: dict, c1, c2, lap1, lap2, lap3):
    lib = _load()
    out = np.zeros(3)
    lib.orc_chem_potential(C.byref(_fluid(fl)), c1, c2, lap1, lap2, lap3, _dp(out))
    return out


def equilibria(c1, c2, eta1, eta2, mu1, mu2, rho, p, ux, uy):
    lib = _load()
    f1, f2, g = np.zeros(9), np.zeros(9), np.zeros(9)
    lib.orc_equilibria(c1, c2, eta1, eta2, mu1, mu2, rho, p, ux, uy, _dp(f1), _dp(f2), _dp(g))
    return f1, f2, g


def sources(tau1, tau2, taug, d1, d2, u, grad_rho, force, fa):
    lib = _load()
    F1, F2, G = np.zeros(9), np.zeros(9), np.zeros(9)
    lib.orc_sources(tau1, tau2, taug, d1[0], d1[1], d2[0], d2[1], u[0], u[1],
                    grad_rho[0], grad_rho[1], force[0], force[1], fa[0], fa[1],
                    _dp(F1), _dp(F2), _dp(G))
    return F1, F2, G


# --------------------------------------------------------------- simulation
class Oracle:
    """Whole-lattice FP64 oracle.  ``problem`` is a dict with keys nx, ny,
    fluid, periodic (px, py), material (uint8 [ny, nx]), mats (list of dicts
    with theta13, theta23, wall_u and kind: 0 wall, 1 velocity boundary)."""

    def __init__(self, problem: dict, threads: int | None = None):
        self._lib = _load()
        if threads:
            self._lib.orc_set_num_threads(int(threads))
        self.nx, self.ny = int(problem["nx"]), int(problem["ny"])
        self.material = np.ascontiguousarray(problem["material"], dtype=np.uint8)
        assert self.material.shape == (self.ny, self.nx)
        mats = problem.get("mats", [])
        arr = (_Material * max(1, len(mats)))()
        for i, m in enumerate(mats):
            arr[i].theta13_deg = m["theta13"]
            arr[i].theta23_deg = m["theta23"]
            wu = m.get("wall_u", (0.0, 0.0))
            arr[i].wall_u[0], arr[i].wall_u[1] = wu[0], wu[1]
            arr[i].kind = int(m.get("kind", 0))
        self._fl = _fluid(problem["fluid"])
        h = C.c_void_p()
        px, py = problem.get("periodic", (1, 1))
        rc = self._lib.orc_create(self.nx, self.ny, C.byref(self._fl), int(px), int(py),
                                  self.material.ctypes.data_as(C.POINTER(C.c_uint8)),
                                  arr, len(mats), C.byref(h))
        if rc != 0:
            raise ValueError("oracle create failed (%d): %s"
                             % (rc, self._lib.orc_last_error().decode()))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.orc_destroy(h)
            self._h = None

    @property
    def n(self):
        return self.nx * self.ny

    def _field(self, a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.shape == (self.ny, self.nx)
        return a

    def init(self, c1, c2, ux=None, uy=None):
        c1, c2, ux, uy = (self._field(a) for a in (c1, c2, ux, uy))
        keep = (c1, c2, ux, uy)  # noqa: F841  (keeps buffers alive across the call)
        rc = self._lib.orc_init(self._h, _dp(c1), _dp(c2),
                                _dp(ux) if ux is not None else None,
                                _dp(uy) if uy is not None else None)
        assert rc == 0

    def step(self, n: int = 1):
        rc = self._lib.orc_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError(self._lib.orc_last_error().decode())

    def eval(self):
        assert self._lib.orc_eval(self._h) == 0

    def fields(self) -> dict:
        out = np.zeros((len(FIELDS), self.ny, self.nx))
        assert self._lib.orc_fields(self._h, _dp(out)) == 0
        return {k: out[i] for i, k in enumerate(FIELDS)}

    def stage(self, name: str) -> np.ndarray:
        out = np.zeros((self.ny, self.nx))
        assert self._lib.orc_stage(self._h, STAGES.index(name), _dp(out)) == 0
        return out

    def populations(self) -> np.ndarray:
        out = np.zeros((27, self.ny, self.nx))
        self._lib.orc_populations(self._h, _dp(out))
        return out

    def set_populations(self, pops: np.ndarray):
        pops = np.ascontiguousarray(pops, dtype=np.float64)
        assert pops.shape == (27, self.ny, self.nx)
        self._lib.orc_set_populations(self._h, _dp(pops))

    def history(self) -> np.ndarray:
        out = np.zeros((4, self.ny, self.nx))
        self._lib.orc_history(self._h, _dp(out))
        return out

    def mass(self) -> np.ndarray:
        out = np.zeros(3)
        self._lib.orc_mass(self._h, _dp(out))
        return out

    def grad(self, chi):
        chi = self._field(chi)
        gx, gy = np.zeros_like(chi), np.zeros_like(chi)
        self._lib.orc_grad_field(self._h, _dp(chi), _dp(gx), _dp(gy))
        return gx, gy

    def lap(self, chi):
        chi = self._field(chi)
        out = np.zeros_like(chi)
        self._lib.orc_lap_field(self._h, _dp(chi), _dp(out))
        return out

    @staticmethod
    def num_threads() -> int:
        return _load().orc_num_threads()

    @staticmethod
    def set_num_threads(n: int) -> None:
        """Threads of the calling thread's later oracle calls."""
        _load().orc_set_num_threads(int(n))


# ------------------------------------------------------------------ 3-D
FIELDS3 = ("c1", "c2", "c3", "rho", "ux", "uy", "uz", "p", "mu1", "mu2", "mu3")


def lattice3():
    lib = _load()
    ex, ey, ez, opp = ((C.c_int * 19)() for _ in range(4))
    w = np.zeros(19)
    lib.orc3_lattice(ex, ey, ez, _dp(w), opp)
    return np.array(ex[:]), np.array(ey[:]), np.array(ez[:]), w, np.array(opp[:])


class Oracle3D:
    """Three-dimensional FP64 oracle (D3Q19).  ``problem`` holds nx, ny, nz,
    fluid (with gravity (gx, gy) and "gravity_z"), periodic (px, py, pz),
    material (uint8 [nz, ny, nx]), mats."""

    def __init__(self, problem: dict, threads: int | None = None):
        self._lib = _load()
        if threads:
            self._lib.orc_set_num_threads(int(threads))
        self.nx, self.ny, self.nz = int(problem["nx"]), int(problem["ny"]), int(problem["nz"])
        self.material = np.ascontiguousarray(problem["material"], dtype=np.uint8)
        assert self.material.shape == (self.nz, self.ny, self.nx)
        mats = problem.get("mats", [])
        arr = (_Material * max(1, len(mats)))()
        for i, m in enumerate(mats):
            arr[i].theta13_deg = m["theta13"]
            arr[i].theta23_deg = m["theta23"]
            wu = m.get("wall_u", (0.0, 0.0))
            arr[i].wall_u[0], arr[i].wall_u[1] = wu[0], wu[1]
            arr[i].kind = int(m.get("kind", 0))
        fl = problem["fluid"]
        self._fl = _fluid(fl)
        h = C.c_void_p()
        px, py, pz = problem.get("periodic", (1, 1, 1))
        rc = self._lib.orc3_create(self.nx, self.ny, self.nz, C.byref(self._fl),
                                   float(fl.get("gravity_z", 0.0)), int(px), int(py), int(pz),
                                   self.material.ctypes.data_as(C.POINTER(C.c_uint8)), arr,
                                   len(mats), C.byref(h))
        if rc != 0:
            raise ValueError("oracle3 create failed (%d): %s"
                             % (rc, self._lib.orc3_last_error().decode()))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.orc3_destroy(h)
            self._h = None

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    def _arr(self, a):
        return None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1)

    def init(self, c1, c2, ux=None, uy=None, uz=None):
        a = [self._arr(v) for v in (c1, c2, ux, uy, uz)]
        rc = self._lib.orc3_init(self._h, *[None if v is None else _dp(v) for v in a])
        assert rc == 0

    def step(self, n: int = 1):
        if self._lib.orc3_step(self._h, int(n)) != 0:
            raise RuntimeError(self._lib.orc3_last_error().decode())

    def fields(self) -> dict:
        out = np.zeros(11 * self.n)
        assert self._lib.orc3_fields(self._h, _dp(out)) == 0
        shape = (self.nz, self.ny, self.nx)
        return {k: out[i * self.n:(i + 1) * self.n].reshape(shape) for i, k in enumerate(FIELDS3)}

    def populations(self) -> np.ndarray:
        out = np.zeros(57 * self.n)
        self._lib.orc3_populations(self._h, _dp(out))
        return out.reshape(57, self.nz, self.ny, self.nx)

    def mass(self) -> np.ndarray:
        out = np.zeros(3)
        self._lib.orc3_mass(self._h, _dp(out))
        return out

    def grad(self, chi):
        chi = self._arr(chi)
        g = [np.zeros(self.n) for _ in range(3)]
        self._lib.orc3_grad_field(self._h, _dp(chi), *[_dp(a) for a in g])
        shape = (self.nz, self.ny, self.nx)
        return tuple(a.reshape(shape) for a in g)

    def lap(self, chi):
        chi = self._arr(chi)
        out = np.zeros(self.n)
        self._lib.orc3_lap_field(self._h, _dp(chi), _dp(out))
        return out.reshape(self.nz, self.ny, self.nx)
