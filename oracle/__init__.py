"""TEST INFRASTRUCTURE: ctypes wrapper of the plain FP64 CPU oracle.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product package never does.

The oracle itself is C (``lbm_oracle.c``); this module builds it with gcc and
exposes a small class, :class:`OracleDomain`, mirroring the oracle's C calls.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")
SOURCES = [os.path.join(HERE, "lbm_oracle.c")]

D2Q9, D3Q19 = 0, 1
EQ_BGK, EQ_HELUO = 0, 1
FACE_PERIODIC, FACE_WALL, FACE_INLET, FACE_OUTLET, FACE_OUTLET_VELOCITY = 0, 1, 2, 3, 4
FACE_ZOUHE_VELOCITY, FACE_ZOUHE_PRESSURE = 5, 6
PROFILE_UNIFORM, PROFILE_PARABOLIC = 0, 1
SHAPE_CIRCLE, SHAPE_ELLIPSE, SHAPE_OUTER_CIRCLE = 0, 1, 2
BC_HALFWAY, BC_MLS = 0, 1
MOTION_STATIC, MOTION_CONST_VEL, MOTION_ROTATE, MOTION_OSCILLATE, MOTION_TABLE, MOTION_FREE = 0, 1, 2, 3, 4, 5
DRIVE_STATIC, DRIVE_LATTICE, DRIVE_COMOVING = 0, 1, 2
INTEGRATOR_EULER, INTEGRATOR_AB2 = 0, 1
REFILL_MEAN, REFILL_AIDUN, REFILL_EXTRAPOLATE = 0, 1, 2
SETS_PREVIOUS, SETS_PREDICTED = 0, 1
REC_LEN = 20
FACE_REC_LEN = 18
MAX_BODIES = 64


def compile_c(sources, out_path) -> str:
    """gcc with the oracle's flags (no FMA contraction, OpenMP on bulk loops):
    the oracle itself, or a variant of its source that a test writes."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-I", HERE, "-o", out_path + ".tmp"] + list(sources) + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out_path + ".tmp", out_path)
    return out_path


def build(force: bool = True) -> str:
    """Compile the oracle."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    return compile_c(SOURCES, LIB_PATH)


class _Desc(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("tau", C.c_double), ("rho0", C.c_double), ("eq_model", C.c_int32),
                ("face", C.c_int32 * 6), ("inlet_profile", C.c_int32), ("inlet_u", C.c_double),
                ("init_rho", C.POINTER(C.c_double)), ("init_u", C.POINTER(C.c_double))]


class _Body(C.Structure):
    _fields_ = [("shape", C.c_int32), ("axes", C.c_double * 3), ("bc", C.c_int32),
                ("motion", C.c_int32), ("c0", C.c_double * 3), ("theta0", C.c_double),
                ("vel", C.c_double * 3), ("omega", C.c_double), ("amp", C.c_double * 3),
                ("period", C.c_double), ("table", C.POINTER(C.c_double)),
                ("table_count", C.c_int64), ("mass", C.c_double), ("inertia", C.c_double),
                ("ext_force", C.c_double * 3), ("ext_torque", C.c_double), ("drive", C.c_int32),
                ("integrator", C.c_int32), ("refill", C.c_int32), ("sets", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load(LIB_PATH)
    return _lib


def load(path):
    """The oracle library at `path` with its argument types declared (the
    built oracle, or a variant of it built by a test)."""
    L = C.CDLL(path)
    L.ora_create.restype = C.c_void_p
    L.ora_create.argtypes = [C.POINTER(_Desc)]
    L.ora_destroy.argtypes = [C.c_void_p]
    L.ora_set_body.argtypes = [C.c_void_p, C.c_int, C.POINTER(_Body)]
    L.ora_step.argtypes = [C.c_void_p, C.c_int64]
    L.ora_time.restype = C.c_int64
    L.ora_time.argtypes = [C.c_void_p]
    L.ora_body_records.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_void_p]
    L.ora_face_records.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]
    L.ora_links.restype = C.c_int64
    L.ora_links.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    L.ora_types.argtypes = [C.c_void_p, C.c_void_p]
    L.ora_get_f.argtypes = [C.c_void_p, C.c_void_p]
    L.ora_fields.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.ora_lattice.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    L.ora_body_pose.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_void_p]
    L.ora_body_drive.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_void_p]
    L.ora_set_threads.argtypes = [C.c_int]
    return L


def lattice(kind: int):
    """(c[Q,3] int, w[Q] float, opp[Q] int) as the oracle numbers them."""
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    o = np.zeros(19, np.int32)
    q = lib().ora_lattice(kind, c.ctypes.data, w.ctypes.data, o.ctypes.data)
    return c[:q].copy(), w[:q].copy(), o[:q].copy()


def nthreads() -> int:
    return lib().ora_nthreads()


def set_threads(n: int) -> int:
    """threads of the oracle's bulk loops from now on; returns the count"""
    return lib().ora_set_threads(int(n))


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleDomain:
    """One oracle domain. Arguments mirror the workload description used by
    the tests (see ``lbm_workloads``)."""

    def __init__(self, lattice, nx, ny, nz=1, tau=0.8, rho0=1.0, eq_model=EQ_BGK,
                 faces=(FACE_PERIODIC,) * 6, inlet_profile=PROFILE_UNIFORM, inlet_u=0.0,
                 init_rho=None, init_u=None, library=None):
        self._L = library if library is not None else lib()
        self.lattice = lattice
        self.nx, self.ny = nx, ny
        self.nz = nz if lattice == D3Q19 else 1
        self.Q = 9 if lattice == D2Q9 else 19
        self.N = self.nx * self.ny * self.nz
        d = _Desc()
        d.lattice, d.nx, d.ny, d.nz = lattice, nx, ny, self.nz
        d.tau, d.rho0, d.eq_model = tau, rho0, eq_model
        for k in range(6):
            d.face[k] = faces[k]
        d.inlet_profile, d.inlet_u = inlet_profile, inlet_u
        self._keep = []
        if init_rho is not None:
            r = np.ascontiguousarray(init_rho, dtype=np.float64).reshape(-1)
            assert r.size == self.N
            self._keep.append(r)
            d.init_rho = _dptr(r)
        if init_u is not None:
            u = np.ascontiguousarray(init_u, dtype=np.float64).reshape(-1)
            assert u.size == 3 * self.N
            self._keep.append(u)
            d.init_u = _dptr(u)
        self._h = self._L.ora_create(C.byref(d))
        if not self._h:
            raise ValueError("oracle rejected the domain description")
        self._keep = []

    def close(self):
        if self._h:
            self._L.ora_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_body(self, body_id, shape, axes, bc=BC_HALFWAY, motion=MOTION_STATIC, c0=(0, 0, 0),
                 theta0=0.0, vel=(0, 0, 0), omega=0.0, amp=(0, 0, 0), period=1.0, table=None,
                 mass=0.0, inertia=0.0, ext_force=(0, 0, 0), ext_torque=0.0, drive=DRIVE_STATIC,
                 integrator=INTEGRATOR_EULER, refill=REFILL_MEAN, sets=SETS_PREVIOUS):
        b = _Body()
        b.mass, b.inertia, b.ext_torque = mass, inertia, ext_torque
        for a in range(3):
            b.ext_force[a] = ext_force[a] if a < len(ext_force) else 0.0
        b.drive, b.integrator, b.refill, b.sets = drive, integrator, refill, sets
        b.shape = shape
        ax = list(axes) + [0.0] * (3 - len(axes))
        for a in range(3):
            b.axes[a] = ax[a]
            b.c0[a] = c0[a] if a < len(c0) else 0.0
            b.vel[a] = vel[a] if a < len(vel) else 0.0
            b.amp[a] = amp[a] if a < len(amp) else 0.0
        b.bc, b.motion, b.theta0, b.omega, b.period = bc, motion, theta0, omega, period
        keep = None
        if table is not None:
            keep = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 8)
            b.table = _dptr(keep)
            b.table_count = keep.shape[0]
        rc = self._L.ora_set_body(self._h, body_id, C.byref(b))
        if rc != 0:
            raise ValueError(f"oracle rejected body {body_id}")

    def step(self, n=1):
        rc = self._L.ora_step(self._h, n)
        if rc != 0:
            raise RuntimeError(f"oracle step failed ({rc})")

    @property
    def t(self):
        return self._L.ora_time(self._h)

    def records(self, body_id, first=0, count=None):
        if count is None:
            count = self.t - first
        out = np.zeros((count, REC_LEN))
        if self._L.ora_body_records(self._h, body_id, first, count, out.ctypes.data) != 0:
            raise ValueError("bad record range")
        return out

    def face_records(self, first=0, count=None):
        if count is None:
            count = self.t - first
        out = np.zeros((count, FACE_REC_LEN))
        if self._L.ora_face_records(self._h, first, count, out.ctypes.data) != 0:
            raise ValueError("bad record range")
        return out

    def links(self, body_id):
        n = self._L.ora_links(self._h, body_id, 0, None, None, None)
        if n < 0:
            raise ValueError("no such body")
        node = np.zeros(n, np.int64)
        d = np.zeros(n, np.int32)
        delta = np.zeros(n)
        self._L.ora_links(self._h, body_id, n, node.ctypes.data, d.ctypes.data, delta.ctypes.data)
        return node, d, delta

    def pose(self, body_id, t):
        """prescribed pose at step t: X[3], theta, V[3], Omega_z"""
        out = np.zeros(8)
        if self._L.ora_body_pose(self._h, body_id, t, out.ctypes.data) != 0:
            raise ValueError("no such body or step")
        return out

    def drive(self, body_id, t):
        """flow force (3) and torque z that moved a free body from t to t+1"""
        out = np.zeros(4)
        if self._L.ora_body_drive(self._h, body_id, t, out.ctypes.data) != 0:
            raise ValueError("no such free body or step")
        return out

    def types(self):
        t = np.zeros(self.N, np.int32)
        self._L.ora_types(self._h, t.ctypes.data)
        return t

    def populations(self):
        f = np.zeros(self.N * self.Q)
        self._L.ora_get_f(self._h, f.ctypes.data)
        return f.reshape(self.N, self.Q)

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        self._L.ora_fields(self._h, rho.ctypes.data, u.ctypes.data)
        return rho, u.reshape(self.N, 3)
