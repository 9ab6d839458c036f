"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the lattice-Boltzmann update and the momentum-exchange sums
runs in the HIP library ``liblbm.so``; this module only converts arguments.
PyTorch, when it sees a GPU, provides the device memory (a caller-owned
buffer sized by ``lbm_footprint_bytes``) and the current HIP stream.
Importing this module on a machine without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

# enums of include/lbm.h
LATTICE = {"D2Q9": 0, "D3Q19": 1}
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "f16_shifted": 2}
EQ = {"bgk": 0, "heluo": 1}
FACE = {"periodic": 0, "wall": 1, "inlet": 2, "outlet": 3, "outlet_velocity": 4, "zouhe_velocity": 5,
        "zouhe_pressure": 6}
PROFILE = {"uniform": 0, "parabolic": 1}
SHAPE = {"circle": 0, "sphere": 0, "ellipse": 1, "ellipsoid": 1, "outer_circle": 2}
BC = {"halfway": 0, "mls": 1}
ME = {"static": 0, "lattice": 1, "comoving": 2, "lattice_backward": 3}
MOTION = {"static": 0, "const_vel": 1, "rotate": 2, "oscillate": 3, "table": 4, "free": 5}
INTEGRATOR = {"euler": 0, "ab2": 1}
REFILL = {"mean": 0, "aidun": 1, "extrapolate": 2}
SETS = {"previous": 0, "predicted": 1}
KERNEL = {"stream_collide": 0, "body": 1, "near_box": 2}
STATUS = {0: "LBM_OK", -1: "LBM_E_INVAL", -2: "LBM_E_NOMEM", -3: "LBM_E_HIP", -4: "LBM_E_RANGE",
          -5: "LBM_E_UNSTABLE", -6: "LBM_E_STATE"}
REC_LEN = 20
FACE_REC_LEN = 18
WALLS = -1  # LBM_WALLS
MAX_BODIES = 64
MAX_STEADY_NOALLOC = 512  # LBM_STEADY_NOALLOC_MAX

EXPORTS = ["lbm_footprint_bytes", "lbm_body_footprint_bytes", "lbm_create_domain", "lbm_destroy_domain", "lbm_set_body", "lbm_step",
           "lbm_synchronize", "lbm_time", "lbm_force_torque", "lbm_records", "lbm_get_links",
           "lbm_get_fields", "lbm_get_types", "lbm_timing_enable", "lbm_timing_read", "lbm_last_error",
           "lbm_batch_create", "lbm_batch_destroy", "lbm_batch_add", "lbm_batch_remove", "lbm_batch_step",
           "lbm_batch_set_config", "lbm_batch_get_config", "lbm_batch_tune", "lbm_steady_state",
           "lbm_batch_steady_state", "lbm_copy", "lbm_get_sweep_config", "lbm_set_sweep_config",
           "lbm_batch_steady_state_noalloc", "lbm_get_moving_sets", "lbm_face_records", "lbm_body_trajectory",
           "lbm_get_populations", "lbm_lattice"]


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class DomainDesc(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("tau", C.c_double), ("rho0", C.c_double), ("storage", C.c_int32), ("eq_model", C.c_int32),
                ("face", C.c_int32 * 6), ("inlet_profile", C.c_int32), ("inlet_u", C.c_double),
                ("init_rho", C.POINTER(C.c_double)), ("init_u", C.POINTER(C.c_double)),
                ("stream", C.c_void_p), ("device_buffer", C.c_void_p), ("device_buffer_bytes", C.c_size_t),
                ("record_capacity", C.c_int64), ("split_schedule", C.c_int32), ("face_records", C.c_int32),
                ("debug_poison", C.c_int32), ("max_bodies", C.c_int32)]


class SweepConfig(C.Structure):
    _fields_ = [("block", C.c_int32), ("cells_per_thread", C.c_int32), ("memory", C.c_int32), ("remap", C.c_int32)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class BatchConfig(C.Structure):
    _fields_ = [("block", C.c_int32), ("cells_per_thread", C.c_int32), ("remap", C.c_int32), ("order", C.c_int32),
                ("overlap", C.c_int32), ("graph", C.c_int32), ("us_per_step", C.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class BodyDesc(C.Structure):
    _fields_ = [("shape", C.c_int32), ("axes", C.c_double * 3), ("bc", C.c_int32), ("me_mode", C.c_int32),
                ("motion", C.c_int32), ("c0", C.c_double * 3), ("theta0", C.c_double), ("vel", C.c_double * 3),
                ("omega", C.c_double), ("amp", C.c_double * 3), ("period", C.c_double),
                ("pose_table", C.POINTER(C.c_double)), ("pose_count", C.c_int64), ("mass", C.c_double),
                ("inertia", C.c_double), ("ext_force", C.c_double * 3), ("ext_torque", C.c_double),
                ("integrator", C.c_int32), ("refill", C.c_int32), ("sets", C.c_int32)]


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_1407_4524_amd.build)")
        # torch carries its own HIP runtime: loaded first, the library binds to
        # that one instead of starting a second runtime beside it
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        L.lbm_footprint_bytes.argtypes = [C.POINTER(DomainDesc), C.POINTER(C.c_size_t)]
        L.lbm_body_footprint_bytes.argtypes = [C.POINTER(DomainDesc), C.POINTER(BodyDesc), C.POINTER(C.c_size_t)]
        L.lbm_create_domain.argtypes = [C.POINTER(DomainDesc), C.POINTER(C.c_void_p)]
        L.lbm_destroy_domain.argtypes = [C.c_void_p]
        L.lbm_set_body.argtypes = [C.c_void_p, C.c_int32, C.POINTER(BodyDesc)]
        L.lbm_step.argtypes = [C.c_void_p, C.c_int64]
        L.lbm_synchronize.argtypes = [C.c_void_p]
        L.lbm_time.argtypes = [C.c_void_p]
        L.lbm_time.restype = C.c_int64
        L.lbm_force_torque.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_void_p]
        L.lbm_records.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_void_p]
        L.lbm_body_trajectory.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_void_p]
        L.lbm_get_populations.argtypes = [C.c_void_p, C.c_void_p]
        L.lbm_lattice.argtypes = [C.c_int32, C.c_void_p, C.c_void_p]
        L.lbm_lattice.restype = C.c_int32
        L.lbm_get_links.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(C.c_int64)]
        L.lbm_get_fields.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.lbm_get_types.argtypes = [C.c_void_p, C.c_void_p]
        L.lbm_timing_enable.argtypes = [C.c_void_p, C.c_int32]
        L.lbm_timing_read.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.lbm_batch_create.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
        L.lbm_batch_destroy.argtypes = [C.c_void_p]
        L.lbm_batch_add.argtypes = [C.c_void_p, C.c_void_p]
        L.lbm_batch_remove.argtypes = [C.c_void_p, C.c_void_p]
        L.lbm_batch_step.argtypes = [C.c_void_p, C.c_int64]
        L.lbm_batch_set_config.argtypes = [C.c_void_p, C.POINTER(BatchConfig)]
        L.lbm_batch_get_config.argtypes = [C.c_void_p, C.POINTER(BatchConfig)]
        L.lbm_batch_tune.argtypes = [C.c_void_p, C.c_int32, C.POINTER(BatchConfig), C.POINTER(BatchConfig),
                                     C.c_int32, C.POINTER(C.c_int32)]
        L.lbm_steady_state.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double)]
        L.lbm_batch_steady_state.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p]
        L.lbm_batch_steady_state_noalloc.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p]
        L.lbm_get_sweep_config.argtypes = [C.c_void_p, C.POINTER(SweepConfig)]
        L.lbm_set_sweep_config.argtypes = [C.c_void_p, C.POINTER(SweepConfig)]
        L.lbm_get_moving_sets.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_int64),
                                          C.POINTER(C.c_int64)]
        L.lbm_face_records.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]
        L.lbm_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p]
        L.lbm_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise LbmError(status, lib().lbm_last_error().decode())


def _torch_cuda():
    try:
        import torch
    except ImportError:
        return None
    return torch if torch.cuda.is_available() else None


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lattice_tables(lattice):
    """(c[Q,3], w[Q]) of the library's direction numbering"""
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    q = lib().lbm_lattice(_enum(LATTICE, lattice), c.ctypes.data, w.ctypes.data)
    return c[:q].copy(), w[:q].copy()


def _enum(table, v):
    return table[v] if isinstance(v, str) else int(v)


def domain_desc(lattice="D2Q9", nx=64, ny=64, nz=1, tau=0.8, rho0=1.0, storage="f32", eq="bgk",
                faces=("periodic",) * 6, inlet_profile="uniform", inlet_u=0.0, record_capacity=0,
                split_schedule=False, face_records=False, debug_poison=False, max_bodies=0):
    """lbm_domain_desc of these settings (no initial fields, stream or buffer)"""
    d = DomainDesc()
    d.lattice = _enum(LATTICE, lattice)
    d.nx, d.ny, d.nz = nx, ny, nz if d.lattice == 1 else 1
    d.tau, d.rho0 = tau, rho0
    d.storage = _enum(STORAGE, storage)
    d.eq_model = _enum(EQ, eq)
    for k in range(6):
        d.face[k] = _enum(FACE, faces[k])
    d.inlet_profile = _enum(PROFILE, inlet_profile)
    d.inlet_u = inlet_u
    d.record_capacity = record_capacity
    d.split_schedule = int(split_schedule)  # False/0: the default schedule, True/1: split, -1: plain
    d.face_records = 1 if face_records else 0
    d.debug_poison = 1 if debug_poison else 0
    d.max_bodies = max_bodies
    return d


def body_desc(shape="circle", axes=(1.0,), bc="halfway", me="static", motion="static", c0=(0, 0, 0), theta0=0.0,
              vel=(0, 0, 0), omega=0.0, amp=(0, 0, 0), period=1.0, table=None, mass=0.0, inertia=0.0,
              ext_force=(0, 0, 0), ext_torque=0.0, integrator="euler", refill="mean", sets="previous"):
    """(lbm_body_desc, arrays it points to) of these settings"""
    b = BodyDesc()
    b.mass, b.inertia, b.ext_torque = mass, inertia, ext_torque
    for a in range(3):
        b.ext_force[a] = ext_force[a] if a < len(ext_force) else 0.0
    b.integrator = _enum(INTEGRATOR, integrator)
    b.refill = _enum(REFILL, refill)
    b.sets = _enum(SETS, sets)
    b.shape = _enum(SHAPE, shape)
    ax = list(axes) + [0.0] * (3 - len(axes))
    if b.shape == 1 and len(axes) == 1:
        ax = [axes[0]] * 3
    for a in range(3):
        b.axes[a] = ax[a]
        b.c0[a] = c0[a] if a < len(c0) else 0.0
        b.vel[a] = vel[a] if a < len(vel) else 0.0
        b.amp[a] = amp[a] if a < len(amp) else 0.0
    b.bc = _enum(BC, bc)
    b.me_mode = _enum(ME, me)
    b.motion = _enum(MOTION, motion)
    b.theta0, b.omega, b.period = theta0, omega, period
    keep = None
    if table is not None:
        keep = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 8)
        b.pose_table = _dptr(keep)
        b.pose_count = keep.shape[0]
    return b, keep


_SPEC_KEYS = ("lattice", "nx", "ny", "nz", "tau", "rho0", "storage", "eq", "faces", "inlet_profile", "inlet_u")


def footprint_bytes(w, **kw):
    """Device bytes a domain built from workload dictionary w takes, its
    bodies included (lbm_footprint_bytes + lbm_body_footprint_bytes); no GPU
    needed."""
    nb = len(w.get("bodies", []))
    if nb > 4 and "max_bodies" not in kw:
        kw = dict(kw, max_bodies=nb)
    d = domain_desc(**{k: w[k] for k in _SPEC_KEYS if k in w}, **kw)
    n = C.c_size_t(0)
    _check(lib().lbm_footprint_bytes(C.byref(d), C.byref(n)))
    total = n.value
    for b in w.get("bodies", []):
        bd, _ = body_desc(**b)
        _check(lib().lbm_body_footprint_bytes(C.byref(d), C.byref(bd), C.byref(n)))
        total += n.value
    return total


class Domain:
    """One simulation domain on the current GPU (see include/lbm.h)."""

    def __init__(self, lattice="D2Q9", nx=64, ny=64, nz=1, tau=0.8, rho0=1.0, storage="f32", eq="bgk",
                 faces=("periodic",) * 6, inlet_profile="uniform", inlet_u=0.0, init_rho=None, init_u=None,
                 record_capacity=0, stream=None, torch_buffer=True, split_schedule=False, face_records=False,
                 debug_poison=False, max_bodies=0):
        d = domain_desc(lattice, nx, ny, nz, tau, rho0, storage, eq, faces, inlet_profile, inlet_u,
                        record_capacity, split_schedule, face_records, debug_poison, max_bodies)
        self.nx, self.ny, self.nz = nx, ny, (nz if d.lattice == 1 else 1)
        self.lattice = d.lattice
        self.N = self.nx * self.ny * self.nz
        keep = []
        if init_rho is not None:
            r = np.ascontiguousarray(init_rho, dtype=np.float64).reshape(-1)
            if r.size != self.N:
                raise ValueError("init_rho size")
            keep.append(r)
            d.init_rho = _dptr(r)
        if init_u is not None:
            u = np.ascontiguousarray(init_u, dtype=np.float64).reshape(-1)
            if u.size != 3 * self.N:
                raise ValueError("init_u size")
            keep.append(u)
            d.init_u = _dptr(u)
        torch = _torch_cuda()
        self._buffer = None
        if stream is not None:
            d.stream = stream
        elif torch is not None:
            d.stream = torch.cuda.current_stream().cuda_stream
        if torch is not None and torch_buffer:
            nbytes = C.c_size_t(0)
            _check(lib().lbm_footprint_bytes(C.byref(d), C.byref(nbytes)))
            self._buffer = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
            d.device_buffer = self._buffer.data_ptr()
            d.device_buffer_bytes = nbytes.value
        self._h = C.c_void_p()
        _check(lib().lbm_create_domain(C.byref(d), C.byref(self._h)))
        self._bodies = {}

    @classmethod
    def from_spec(cls, w, init_rho=None, init_u=None, **kw):
        """Build from a plain workload dictionary (lattice, nx, ny, nz, tau, rho0,
        storage, eq, faces, inlet_profile, inlet_u, bodies)."""
        faces = tuple(w["faces"])
        nb = len(w.get("bodies", []))
        if nb > 4 and "max_bodies" not in kw:
            kw = dict(kw, max_bodies=nb)
        dom = cls(lattice=w["lattice"], nx=w["nx"], ny=w["ny"], nz=w.get("nz", 1), tau=w["tau"],
                  rho0=w.get("rho0", 1.0), storage=w.get("storage", "f32"), eq=w.get("eq", "bgk"),
                  faces=faces, inlet_profile=w.get("inlet_profile", "uniform"), inlet_u=w.get("inlet_u", 0.0),
                  init_rho=init_rho, init_u=init_u, **kw)
        for k, b in enumerate(w.get("bodies", [])):
            dom.set_body(k, **b)
        return dom

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().lbm_destroy_domain(self._h))
            self._h = C.c_void_p()
        self._buffer = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self):
        return None if self._buffer is None else self._buffer.numel()

    def set_body(self, body_id, **body):
        """body settings as in body_desc()"""
        b, keep = body_desc(**body)
        _check(lib().lbm_set_body(self._h, body_id, C.byref(b)))
        self._bodies[body_id] = (b, keep)

    def step(self, n=1):
        _check(lib().lbm_step(self._h, n))

    def synchronize(self):
        _check(lib().lbm_synchronize(self._h))

    @property
    def t(self):
        return lib().lbm_time(self._h)

    def force_torque(self, body_id=0, first=0, count=None):
        if count is None:
            count = self.t - first
        out = np.zeros((count, 6))
        _check(lib().lbm_force_torque(self._h, body_id, first, count, out.ctypes.data))
        return out

    def populations(self):
        """f[node, i] (nx*ny*nz x Q, the numbering of lattice_tables()); NaN off the fluid"""
        q = 9 if self.lattice == 0 else 19
        f = np.zeros(self.N * q)
        _check(lib().lbm_get_populations(self._h, f.ctypes.data))
        return f.reshape(self.N, q)

    def trajectory(self, body_id=0, first=0, count=None):
        """poses X[3], theta, V[3], Omega_z of steps first .. first+count-1
        (default: up to the current step, inclusive)"""
        if count is None:
            count = self.t - first + 1
        out = np.zeros((count, 8))
        _check(lib().lbm_body_trajectory(self._h, body_id, first, count, out.ctypes.data))
        return out

    def records(self, body_id=0, first=0, count=None):
        if count is None:
            count = self.t - first
        out = np.zeros((count, REC_LEN))
        _check(lib().lbm_records(self._h, body_id, first, count, out.ctypes.data))
        return out

    def face_records(self, first=0, count=None):
        """per step: F, T of the wall layers, the inlet and the outlet (18
        values, T about the origin); the domain must record its faces"""
        if count is None:
            count = self.t - first
        out = np.zeros((count, FACE_REC_LEN))
        _check(lib().lbm_face_records(self._h, first, count, out.ctypes.data))
        return out

    def moving_sets(self, body_id, step):
        """(n_plus, n_minus): covered and uncovered node counts between step
        and step + 1"""
        a, b = C.c_int64(0), C.c_int64(0)
        _check(lib().lbm_get_moving_sets(self._h, body_id, step, C.byref(a), C.byref(b)))
        return a.value, b.value

    def links(self, body_id=0):
        n = C.c_int64(0)
        _check(lib().lbm_get_links(self._h, body_id, 0, None, None, None, C.byref(n)))
        node = np.zeros(n.value, np.int64)
        d = np.zeros(n.value, np.int32)
        delta = np.zeros(n.value)
        _check(lib().lbm_get_links(self._h, body_id, n.value, node.ctypes.data, d.ctypes.data,
                                   delta.ctypes.data, C.byref(n)))
        return node, d, delta

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        _check(lib().lbm_get_fields(self._h, rho.ctypes.data, u.ctypes.data))
        return rho, u.reshape(self.N, 3)

    @property
    def sweep_config(self):
        """launch shape of the stream-collide update (lbm_get_sweep_config)"""
        c = SweepConfig()
        _check(lib().lbm_get_sweep_config(self._h, C.byref(c)))
        return c.as_dict()

    @sweep_config.setter
    def sweep_config(self, d):
        c = SweepConfig(**d)
        _check(lib().lbm_set_sweep_config(self._h, C.byref(c)))

    def timing_enable(self, every=1):
        """time every n-th launch of each kernel (True = 1, False/0 = off)"""
        _check(lib().lbm_timing_enable(self._h, int(every)))

    def timing_read(self, kernel="stream_collide", issued=False):
        """(summed kernel time in ms, number of timed launches, node updates
        made by them) of the kernels "stream_collide", "body" or "near_box"
        since the last timing_enable; with issued=True a fourth entry, the
        number of launches of that kind issued (timed or not)"""
        ms = C.c_double(0)
        n = C.c_int64(0)
        nodes = C.c_int64(0)
        iss = C.c_int64(0)
        _check(lib().lbm_timing_read(self._h, _enum(KERNEL, kernel), C.byref(ms), C.byref(n), C.byref(nodes),
                                     C.byref(iss)))
        if issued:
            return ms.value, n.value, nodes.value, iss.value
        return ms.value, n.value, nodes.value

    def steady_state(self, window=500, tol=1e-6, body_id=0):
        """(steady, relative drag change over the last `window` steps), computed
        on the device in FP64"""
        st = C.c_int32(0)
        rel = C.c_double(0)
        _check(lib().lbm_steady_state(self._h, body_id, int(window), float(tol), C.byref(st), C.byref(rel)))
        return bool(st.value), rel.value

    def types(self):
        t = np.zeros(self.N, np.int32)
        _check(lib().lbm_get_types(self._h, t.ctypes.data))
        return t


def copy(src, dst, nbytes, variant=2, stream=None):
    """lbm_copy: the library's plain device copy (measurement only) of nbytes
    from device address src to dst, enqueued on `stream` (default: torch's
    current stream)."""
    if stream is None:
        torch = _torch_cuda()
        stream = torch.cuda.current_stream().cuda_stream if torch is not None else 0
    _check(lib().lbm_copy(C.c_void_p(src), C.c_void_p(dst), C.c_size_t(nbytes), int(variant), C.c_void_p(stream)))


class Batch:
    """Domains of one lattice, storage and equilibrium advanced by the same
    launches (see include/lbm.h, lbm_batch_*). Members keep their own
    handles; while they are members their work runs on the batch's stream."""

    def __init__(self, stream=None):
        torch = _torch_cuda()
        if stream is None and torch is not None:
            stream = torch.cuda.current_stream().cuda_stream
        self._h = C.c_void_p()
        _check(lib().lbm_batch_create(C.c_void_p(stream or 0), C.byref(self._h)))
        self.members = []

    def add(self, dom):
        _check(lib().lbm_batch_add(self._h, dom._h))
        self.members.append(dom)

    def remove(self, dom):
        _check(lib().lbm_batch_remove(self._h, dom._h))
        self.members.remove(dom)

    def step(self, n=1):
        _check(lib().lbm_batch_step(self._h, int(n)))

    @property
    def config(self):
        c = BatchConfig()
        _check(lib().lbm_batch_get_config(self._h, C.byref(c)))
        return c.as_dict()

    @config.setter
    def config(self, d):
        c = BatchConfig(**{k: v for k, v in d.items() if k != "us_per_step"})
        _check(lib().lbm_batch_set_config(self._h, C.byref(c)))

    def tune(self, trial_steps=10):
        """runs every candidate launch shape for trial_steps real steps, keeps
        the fastest; returns (chosen, [all trials]) as dictionaries"""
        chosen = BatchConfig()
        trials = (BatchConfig * 128)()
        n = C.c_int32(0)
        _check(lib().lbm_batch_tune(self._h, int(trial_steps), C.byref(chosen), trials, 128, C.byref(n)))
        return chosen.as_dict(), [trials[i].as_dict() for i in range(n.value)]

    def steady_state(self, window=500, tol=1e-6, noalloc=False):
        """per member (in the order added): steady flag (1, 0, or -1 when it
        cannot be evaluated yet) and relative drag change over `window` steps;
        noalloc=True calls lbm_batch_steady_state_noalloc (no device
        allocation, at most LBM_STEADY_NOALLOC_MAX members)"""
        n = len(self.members)
        st = np.zeros(n, np.int32)
        rel = np.zeros(n)
        fn = lib().lbm_batch_steady_state_noalloc if noalloc else lib().lbm_batch_steady_state
        if n:
            _check(fn(self._h, int(window), float(tol), st.ctypes.data, rel.ctypes.data))
        return st, rel

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().lbm_batch_destroy(self._h))
            self._h = C.c_void_p()
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

