"""Build oracle domains from the shared workload descriptions (test infrastructure)."""
import numpy as np

import lbm_workloads as W
import oracle as O

LATTICE = {"D2Q9": O.D2Q9, "D3Q19": O.D3Q19}
EQ = {"bgk": O.EQ_BGK, "heluo": O.EQ_HELUO}
PROFILE = {"uniform": O.PROFILE_UNIFORM, "parabolic": O.PROFILE_PARABOLIC}
SHAPE = {"circle": O.SHAPE_CIRCLE, "sphere": O.SHAPE_CIRCLE, "ellipse": O.SHAPE_ELLIPSE,
         "ellipsoid": O.SHAPE_ELLIPSE, "outer_circle": O.SHAPE_OUTER_CIRCLE}
BC = {"halfway": O.BC_HALFWAY, "mls": O.BC_MLS}
MOTION = {"static": O.MOTION_STATIC, "const_vel": O.MOTION_CONST_VEL, "rotate": O.MOTION_ROTATE,
          "oscillate": O.MOTION_OSCILLATE, "table": O.MOTION_TABLE, "free": O.MOTION_FREE}
DRIVE = {"static": O.DRIVE_STATIC, "lattice": O.DRIVE_LATTICE, "comoving": O.DRIVE_COMOVING,
         "lattice_backward": O.DRIVE_LATTICE}
INTEGRATOR = {"euler": O.INTEGRATOR_EULER, "ab2": O.INTEGRATOR_AB2}
REFILL = {"mean": O.REFILL_MEAN, "aidun": O.REFILL_AIDUN, "extrapolate": O.REFILL_EXTRAPOLATE}
SETS = {"previous": O.SETS_PREVIOUS, "predicted": O.SETS_PREDICTED}


def make_oracle(w, init_rho=None, init_u=None):
    if init_rho is None:
        init_rho = W.density_noise(w)
    d = O.OracleDomain(LATTICE[w["lattice"]], w["nx"], w["ny"], w["nz"], tau=w["tau"],
                       rho0=w["rho0"], eq_model=EQ[w["eq"]], faces=tuple(w["faces"]),
                       inlet_profile=PROFILE[w["inlet_profile"]], inlet_u=w["inlet_u"],
                       init_rho=init_rho, init_u=init_u)
    for k, b in enumerate(w.get("bodies", [])):
        d.set_body(k, SHAPE[b["shape"]], b["axes"], bc=BC[b["bc"]], motion=MOTION[b["motion"]],
                   c0=b.get("c0", (0, 0, 0)), theta0=b.get("theta0", 0.0), vel=b.get("vel", (0, 0, 0)),
                   omega=b.get("omega", 0.0), amp=b.get("amp", (0, 0, 0)),
                   period=b.get("period", 1.0), table=b.get("table"), mass=b.get("mass", 0.0),
                   inertia=b.get("inertia", 0.0), ext_force=b.get("ext_force", (0, 0, 0)),
                   ext_torque=b.get("ext_torque", 0.0), drive=DRIVE[b.get("me", "static")],
                   integrator=INTEGRATOR[b.get("integrator", "euler")], refill=REFILL[b.get("refill", "mean")],
                   sets=SETS[b.get("sets", "previous")])
    return d


def me_series(rec, mode):
    """(F[T,3], T[T,3]) of one ME variant from oracle records."""
    if mode == "static":
        return rec[:, 0:3], rec[:, 3:6]
    if mode == "lattice":
        return rec[:, 0:3] + rec[:, 6:9], rec[:, 3:6] + rec[:, 9:12]
    if mode == "comoving":
        return rec[:, 12:15], rec[:, 15:18]
    if mode == "lattice_backward":  # node terms of the step before
        prev = np.vstack([np.zeros((1, 6)), rec[:-1, 6:12]])
        return rec[:, 0:3] + prev[:, 0:3], rec[:, 3:6] + prev[:, 3:6]
    raise ValueError(mode)
