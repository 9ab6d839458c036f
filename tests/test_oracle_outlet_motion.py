"""Pins of two oracle parts that the momentum budgets cannot see: the
zero-gradient outlet (its copy rule closes the channel budget whatever value
it supplies) and the oscillating prescribed motion (the budget closes for any
wall velocity). Each pin is checked on the oracle and, to show that it has
teeth, on copies of the oracle's source with one plausible mistake planted
(built here with gcc, on the CPU).

Readings pinned (the paper fixes neither; the workloads need both):
* zero-gradient outlet: a population entering the last column x = nx-1 from
  beyond the outlet is the same column's post-collision population of that
  direction, taken one link back along the transverse axes:
  f_i(nx-1, y, z, t+1) = fhat_i(nx-1, y - c_iy, z - c_iz, t) for c_ix = -1;
* oscillating motion: X(t) = c0 + A sin(2 pi t / T) at integer steps, and the
  body velocity V(t) = dX/dt = A (2 pi / T) cos(2 pi t / T).
"""
import hashlib
import math
import os

import numpy as np
import pytest

import lbm_workloads as W
import oracle as O

ORACLE_C = os.path.join(os.path.dirname(O.__file__), "lbm_oracle.c")


def mutant(tmp_path, old, new):
    """the oracle built from its source with `old` replaced by `new` (which
    must occur exactly once)"""
    src = open(ORACLE_C).read()
    assert src.count(old) == 1, old
    tag = hashlib.sha1(new.encode()).hexdigest()[:10]  # one file per variant: dlopen caches by path
    path = tmp_path / f"lbm_oracle_{tag}.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / f"liblbm_oracle_{tag}.so")
    O.compile_c([str(path)], so)
    return O.load(so)


OUTLET_NO_SHIFT = ("int o[3] = {d->nx - 1, q[1], q[2]};", "int o[3] = {d->nx - 1, p[1], p[2]};")
OUTLET_WRONG_DIR = ("fbc = d->fpost[mo * Q + i];", "fbc = d->fpost[mo * Q + L->opp[i]];")
OUTLET_WRONG_COLUMN = ("int o[3] = {d->nx - 1, q[1], q[2]};", "int o[3] = {d->nx - 2, q[1], q[2]};")
OSC_VELOCITY_PHASE = ("p.V[a] = d->amp[a] * ((2.0 * ORA_PI) / d->period) * c;",
                      "p.V[a] = d->amp[a] * ((2.0 * ORA_PI) / d->period) * s;")
OSC_POSITION_PHASE = ("p.X[a] = d->c0[a] + d->amp[a] * s;", "p.X[a] = d->c0[a] + d->amp[a] * c;")


def channel(lat, nx, ny, nz, u_in, library=None, init_rho=None, init_u=None, faces=None, tau=0.7):
    faces = faces or (O.FACE_INLET, O.FACE_OUTLET) + (O.FACE_PERIODIC,) * 4
    return O.OracleDomain(lat, nx, ny, nz, tau=tau, faces=faces, inlet_profile=O.PROFILE_UNIFORM,
                          inlet_u=u_in, init_rho=init_rho, init_u=init_u, library=library)


# ---------------------------------------------------------------------------
# the outlet


def plug_flow_defect(lat, library=None, steps=40):
    """largest deviation of any population from the uniform plug flow
    f^eq(rho0, u) after `steps` steps through a velocity inlet and the
    zero-gradient outlet, periodic across: every rule maps that state to itself
    (the inlet's bounce-back adds exactly the odd part 6 w_i rho c_i.u)"""
    nx, ny, nz = (20, 6, 1) if lat == O.D2Q9 else (14, 5, 4)
    u = 0.05
    n = nx * ny * nz
    U = np.tile([u, 0.0, 0.0], (n, 1))
    d = channel(lat, nx, ny, nz, u, library=library, init_rho=np.ones(n), init_u=U)
    f0 = d.populations().copy()
    d.step(steps)
    f = d.populations()
    d.close()
    return np.abs(f - f0).max()


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_outlet_keeps_a_plug_flow(lat):
    assert plug_flow_defect(lat) < 1e-14


def outlet_one_step_defect(lat, library=None):
    """From an equilibrium state varying along every axis (so that collision
    leaves it unchanged and fhat(t=0) is the initial f), one step: every
    population entering the last column from beyond the outlet must equal the
    initial population of the same direction at (nx-1, y - c_iy, z - c_iz)
    (periodic across). Returns the largest difference."""
    nx, ny, nz = (9, 7, 1) if lat == O.D2Q9 else (7, 5, 6)
    w = dict(nx=nx, ny=ny, nz=nz, rho0=1.0, seed=5, lattice="D2Q9" if lat == O.D2Q9 else "D3Q19")
    rho, u = W.random_state(w, rho_amp=0.05, u_amp=0.08, seed=5)
    d = channel(lat, nx, ny, nz, 0.03, library=library, init_rho=rho, init_u=u)
    f0 = d.populations().reshape(nz, ny, nx, -1).copy()
    d.step(1)
    f1 = d.populations().reshape(nz, ny, nx, -1)
    d.close()
    c, _, _ = O.lattice(lat)
    worst = 0.0
    for i in range(len(c)):
        if c[i, 0] != -1:
            continue
        for z in range(nz):
            for y in range(ny):
                ys, zs = (y - c[i, 1]) % ny, (z - c[i, 2]) % nz
                worst = max(worst, abs(f1[z, y, nx - 1, i] - f0[zs, ys, nx - 1, i]))
    return worst


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_outlet_copies_its_column_shifted_along_the_link(lat):
    assert outlet_one_step_defect(lat) < 1e-14


def x_independence_defect(lat, library=None, steps=5):
    """A state that varies across the channel but not along it stays
    independent of x near the outlet, bit for bit, until the inlet's influence
    (one column per step) arrives: the outlet column equals its upstream
    neighbours. Returns the number of populations that differ."""
    nx, ny, nz = (16, 9, 1) if lat == O.D2Q9 else (14, 7, 5)
    w = dict(nx=1, ny=ny, nz=nz, rho0=1.0, seed=9, lattice="D2Q9" if lat == O.D2Q9 else "D3Q19")
    rho1, u1 = W.random_state(w, rho_amp=0.05, u_amp=0.08, seed=9)  # one value per (y, z)
    rho = np.repeat(rho1.reshape(nz, ny, 1), nx, axis=2).reshape(-1)
    u = np.repeat(u1.reshape(nz, ny, 1, 3), nx, axis=2).reshape(-1, 3)
    d = channel(lat, nx, ny, nz, 0.02, library=library, init_rho=rho, init_u=u)
    d.step(steps)
    f = d.populations().reshape(nz, ny, nx, -1)
    d.close()
    ref = f[:, :, nx - 1, :]
    return sum(int((f[:, :, x, :] != ref).sum()) for x in range(steps + 1, nx - 1))


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_outlet_keeps_a_state_uniform_along_x(lat):
    assert x_independence_defect(lat) == 0


@pytest.mark.parametrize("mistake", [OUTLET_NO_SHIFT, OUTLET_WRONG_DIR, OUTLET_WRONG_COLUMN],
                         ids=["no_transverse_shift", "opposite_direction", "wrong_column"])
def test_outlet_pins_catch_planted_mistakes(tmp_path, mistake):
    L = mutant(tmp_path, *mistake)
    caught = []
    for lat in (O.D2Q9, O.D3Q19):
        caught.append(plug_flow_defect(lat, L) > 1e-6 or outlet_one_step_defect(lat, L) > 1e-6 or
                      x_independence_defect(lat, L) > 0)
    assert all(caught), caught


# ---------------------------------------------------------------------------
# the oscillating motion

AMP = (0.0, 2.0, 0.0)
PERIOD = 40.0
C0 = (12.3, 10.4, 0.0)
R = 3.7


def oscillating(library=None, nx=26, ny=22):
    d = O.OracleDomain(O.D2Q9, nx, ny, tau=0.8, library=library)
    d.set_body(0, O.SHAPE_CIRCLE, (R,), bc=O.BC_MLS, motion=O.MOTION_OSCILLATE, c0=C0, amp=AMP, period=PERIOD)
    return d


def oscillation_defects(library=None):
    """(position error against c0 + A sin(2 pi t/T); velocity error against
    the central difference of the positions, minus its truncation bound
    |A| w^3/6 with w = 2 pi/T) over two periods"""
    d = oscillating(library)
    w = 2.0 * math.pi / PERIOD
    steps = int(2 * PERIOD) + 2
    P = np.array([d.pose(0, t) for t in range(steps)])
    d.close()
    X = np.array([[C0[a] + AMP[a] * math.sin(w * t) for a in range(3)] for t in range(steps)])
    ex = np.abs(P[:, 0:3] - X).max()
    D = (P[2:, 0:3] - P[:-2, 0:3]) / 2.0
    bound = max(abs(a) for a in AMP) * w ** 3 / 6.0
    ev = np.abs(P[1:-1, 4:7] - D).max() - bound
    return ex, ev, np.abs(P[:, 4:7]).max()


def test_oscillating_pose_and_velocity():
    ex, ev, vmax = oscillation_defects()
    assert ex < 1e-13
    assert ev < 1e-12
    assert abs(vmax - AMP[1] * 2 * math.pi / PERIOD) < 1e-3 * vmax  # the bound is not met by V = 0


def solid_set_defect(library=None, steps=None):
    """number of (step, node) pairs where the oracle's solid set differs from
    the circle at X(t) = c0 + A sin(2 pi t/T) evaluated here, over a period;
    the nodes nearest the surface stay at least 1e-9 from it"""
    steps = steps or int(PERIOD)
    nx, ny = 26, 22
    d = oscillating(library, nx, ny)
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    bad = 0
    margin = np.inf
    for t in range(steps):
        X = [C0[a] + AMP[a] * math.sin(2.0 * math.pi * t / PERIOD) for a in range(3)]
        dx, dy = xx - X[0], yy - X[1]
        phi = (dx * dx + dy * dy) - R * R
        margin = min(margin, np.abs(phi).min())
        ty = d.types().reshape(ny, nx)
        bad += int(((phi <= 0.0) != (ty == 2)).sum())
        d.step(1)
    d.close()
    assert margin > 1e-9
    return bad


def test_oscillating_solid_sets_against_brute_force():
    assert solid_set_defect() == 0


def test_oscillation_pins_catch_planted_mistakes(tmp_path):
    L = mutant(tmp_path, *OSC_VELOCITY_PHASE)
    ex, ev, _ = oscillation_defects(L)
    assert ev > 1e-3
    L2 = mutant(tmp_path, *OSC_POSITION_PHASE)
    assert solid_set_defect(L2) > 0
