"""Shared pieces of the GPU parity tests: build the GPU domain and the oracle
from the same workload description and seeded inputs, and compare."""
import numpy as np

from oracle_helpers import make_oracle, me_series


def make_gpu(w, init_rho=None, init_u=None, **kw):
    """GPU domain of workload w; like make_oracle it applies the workload's
    seeded density noise when no initial density is given."""
    import lbm_workloads as W
    from paper_1407_4524_amd import Domain
    if init_rho is None:
        init_rho = W.density_noise(w)
    return Domain.from_spec(w, init_rho=init_rho, init_u=init_u, **kw)


def series_error(ft_gpu, F_ora, T_ora, R, scale=None):
    """Relative error of a force/torque series: max_t |F_gpu - F_ora| over
    max_t |drag| (x-force) for every force component, and over max|drag|*R
    for the torque (lift and torque pass near zero, so each is measured
    against the drag scale)."""
    drag = scale if scale is not None else max(np.abs(F_ora[:, 0]).max(), 1e-30)
    eF = np.abs(ft_gpu[:, 0:3] - F_ora).max() / drag
    eT = np.abs(ft_gpu[:, 3:6] - T_ora).max() / (drag * R)
    return eF, eT


def run_pair(w, steps, init_rho=None, init_u=None, **kw):
    g = make_gpu(w, init_rho=init_rho, init_u=init_u, **kw)
    o = make_oracle(w, init_rho=init_rho, init_u=init_u)
    g.step(steps)
    o.step(steps)
    return g, o


def velocity_error(g, o):
    """L-infinity velocity difference over nodes fluid on both sides, and
    the check that both sides agree on which nodes are fluid."""
    tg, to = g.types(), o.types()
    assert (tg == to).all(), "solid/fluid classification differs"
    _, ug = g.fields()
    _, uo = o.fields()
    m = to == 0
    return np.abs(ug[m] - uo[m]).max()


def ora_series(o, body, mode):
    return me_series(o.records(body), mode)
