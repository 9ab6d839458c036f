"""Pins of the oracle's free bodies (Newton-Euler motion under the flow force,
the sedimentation set-up of the paper's Sec. IV) and of its refill rules
(Sec. III.B.3), against what holds independently of how the oracle writes
them:

* at rest: a free body in a fluid at rest, with no external force, stays
  where it is (to rounding);
* closed form: with a huge mass and inertia and a constant external force
  and torque, the flow's share of the acceleration vanishes and the motion
  is the discrete constant-acceleration one, X(T) = X0 + V0 T + a T(T+1)/2
  (the position takes the new velocity) and likewise theta; the cos/sin of
  the computed angle agree with libm to a few ulp;
* coupled momentum budget (P3 extended to the body): in a periodic box the
  fluid's momentum, measured from the populations, plus the body's M V,
  changes over T steps by exactly T F_ext minus the last step's covered/
  uncovered momentum (forward Euler, lattice-frame drive with the previous
  step's node terms), and by the Adams-Bashforth end terms for AB2;
* predicted sets (the paper's second approximation): for a body whose
  velocity cannot change (huge mass, no external force) the predicted pose
  is the next pose, so the predicted node terms that drive it equal the
  forward node terms the oracle records for the same step (separate code:
  the record comes from the actual advance); with a light body both
  approximations give close trajectories;
* refill rules: in uniform flow past a body translating with it every rule
  keeps the flow exactly uniform; AIDUN gives an uncovered node the wall
  velocity and the mean density of its fluid neighbours; EXTRAPOLATE matches
  a brute-force evaluation of its definition (direction, nodes, BGK
  post-collision states, quadratic extrapolation).
"""
import math

import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
from oracle_helpers import make_oracle, me_series


def _box(lattice="D2Q9", nx=48, ny=40, nz=1, tau=0.7, faces=W.PERIODIC_FACES, eq="bgk"):
    return dict(name="box", lattice=lattice, nx=nx, ny=ny, nz=nz if lattice == "D3Q19" else 1, tau=tau, rho0=1.0,
                eq=eq, faces=faces, inlet_profile="uniform", inlet_u=0.0, storage="f64", rho_noise=0.0, seed=0,
                bodies=[])


def _momentum(d):
    c, _, _ = O.lattice(d.lattice)
    f = d.populations()
    return (f[d.types() == 0] @ c.astype(float)).sum(axis=0)


def test_free_body_at_rest_stays():
    w = _box()
    R = 4.3
    M = math.pi * R * R
    w["bodies"] = [dict(shape="ellipse", axes=(5.0, 3.2), bc="mls", motion="free", me="lattice", c0=(20.3, 19.6, 0.0),
                        theta0=0.3, mass=M, inertia=0.5 * M * R * R)]
    d = make_oracle(w)
    d.step(40)
    p0, p1 = d.pose(0, 0), d.pose(0, 40)
    assert np.abs(p1 - p0).max() < 1e-12


@pytest.mark.parametrize("integrator", ["euler", "ab2"])
def test_free_body_constant_force_closed_form(integrator):
    w = _box()
    M = I = 1e14
    a = np.array([1.1e-3, -6e-4, 0.0])
    alpha = 3e-4
    V0, Om0, X0, th0 = np.array([0.01, 0.004, 0.0]), 0.002, np.array([18.3, 19.7, 0.0]), 0.4
    w["bodies"] = [dict(shape="ellipse", axes=(4.5, 2.5), bc="mls", motion="free", me="comoving", c0=tuple(X0),
                        theta0=th0, vel=tuple(V0), omega=Om0, mass=M, inertia=I, ext_force=tuple(M * a),
                        ext_torque=I * alpha, integrator=integrator)]
    d = make_oracle(w)
    T = 30
    d.step(T)
    p = d.pose(0, T)
    X = X0 + V0 * T + a * T * (T + 1) / 2
    th = th0 + Om0 * T + alpha * T * (T + 1) / 2
    assert np.abs(p[0:3] - X).max() < 1e-11
    assert abs(p[3] - th) < 1e-11
    assert np.abs(p[4:7] - (V0 + a * T)).max() < 1e-12 and abs(p[7] - (Om0 + alpha * T)) < 1e-12
    # the body's nodes are those of the shape at the reported pose (brute force)
    t = d.types().reshape(w["ny"], w["nx"])
    ys, xs = np.mgrid[0:w["ny"], 0:w["nx"]]
    dx, dy = xs - p[0], ys - p[1]
    ct, st = math.cos(p[3]), math.sin(p[3])
    xi, eta = ct * dx + st * dy, ct * dy - st * dx
    phi = xi * xi / 4.5 ** 2 + eta * eta / 2.5 ** 2 - 1.0
    near = np.abs(phi) < 1e-9
    assert ((t == 2) == (phi <= 0))[~near].all()


def test_free_trig_matches_libm():
    w = _box(tau=1.2)
    M = I = 1e18
    w["bodies"] = [dict(shape="ellipse", axes=(4.5, 2.5), bc="mls", motion="free", me="static", c0=(20.0, 20.0, 0.0),
                        theta0=-2.9, omega=0.11, mass=M, inertia=I)]
    d = make_oracle(w)
    d.step(60)  # theta sweeps more than a turn
    for t in range(61):
        th = d.pose(0, t)[3]
        assert abs(th - (-2.9 + 0.11 * t)) < 1e-12
    # the solid set at the last step is that of libm's cos/sin, away from ties
    p = d.pose(0, 60)
    ys, xs = np.mgrid[0:40, 0:48]
    ct, st = math.cos(p[3]), math.sin(p[3])
    dx, dy = xs - p[0], ys - p[1]
    phi = (ct * dx + st * dy) ** 2 / 4.5 ** 2 + (ct * dy - st * dx) ** 2 / 2.5 ** 2 - 1.0
    t = d.types().reshape(40, 48)
    assert ((t == 2) == (phi <= 0))[np.abs(phi) > 1e-12].all()


@pytest.mark.parametrize("integrator", ["euler", "ab2"])
def test_free_body_coupled_momentum_budget(integrator):
    w = _box(nx=50, ny=44, tau=0.7)
    R = 4.6
    M = 1.6 * math.pi * R * R
    F_ext = np.array([2.0e-3, -3.5e-3, 0.0])
    w["bodies"] = [dict(shape="circle", axes=(R,), bc="mls", motion="free", me="lattice", c0=(24.2, 21.7, 0.0),
                        vel=(0.01, -0.02, 0.0), mass=M, inertia=0.5 * M * R * R, ext_force=tuple(F_ext),
                        integrator=integrator)]
    rho, u = W.random_state(w, rho_amp=0.004, u_amp=0.015, seed=21)
    d = make_oracle(w, init_rho=rho, init_u=u)
    scale = d.populations()[d.types() == 0].sum()
    T = 80
    P = [_momentum(d)]
    for _ in range(T):
        d.step(1)
        P.append(_momentum(d))
    P = np.array(P)
    V = np.array([d.pose(0, t)[4:7] for t in range(T + 1)])
    rec = d.records(0)
    imp = rec[:, 6:9]
    assert rec[:, 18].sum() > 0 and rec[:, 19].sum() > 0  # the body moved across nodes
    total = (P[T] - P[0]) + M * (V[T] - V[0])
    if integrator == "euler":
        want = T * F_ext - imp[T - 1]
    else:
        # G(t) = F_static(t) + imp(t-1) + F_ext, with F_static(t) + imp(t) =
        # -(P(t+1) - P(t)) from the fluid; AB2 sums to sum G + (G(T-1) - G(0))/2
        dP = np.diff(P, axis=0)
        imp_prev = np.vstack([np.zeros(3), imp[:-1]])
        G = -dP - imp + imp_prev + F_ext
        want = G.sum(axis=0) + 0.5 * (G[T - 1] - G[0]) + dP.sum(axis=0)
        total = M * (V[T] - V[0]) + (P[T] - P[0])
    assert np.abs(total - want).max() < 1e-13 * scale


@pytest.mark.parametrize("refill", ["mean", "aidun", "extrapolate"])
def test_refill_keeps_uniform_flow(refill):
    V = np.array([0.05, -0.03, 0.0])
    w = _box(nx=40, ny=30, tau=0.75)
    w["bodies"] = [dict(shape="circle", axes=(5.1,), bc="mls", motion="const_vel", c0=(15.3, 14.8, 0.0),
                        vel=tuple(V), refill=refill)]
    n = w["nx"] * w["ny"]
    d = make_oracle(w, init_rho=np.ones(n), init_u=np.tile(V, (n, 1)))
    d.step(40)
    rho, u = d.fields()
    m = d.types() == 0
    assert np.abs(rho[m] - 1).max() < 1e-14 and np.abs(u[m] - V).max() < 1e-14
    assert d.records(0)[:, 19].sum() > 0


def _one_refill_step(refill, init_u, c0, vel=(0.0, 0.0, 0.0), omega=0.0, shape="circle", axes=(4.6,)):
    w = _box(nx=40, ny=36, tau=1.0)  # tau = 1: the populations after collision are the equilibrium
    n = w["nx"] * w["ny"]
    w["bodies"] = [dict(shape=shape, axes=axes, bc="mls", motion="table", c0=c0, refill=refill,
                        table=W.pose_table(3, c0, vel=vel, omega=omega))]
    d = make_oracle(w, init_rho=np.ones(n), init_u=init_u)
    t0 = d.types()
    d.step(1)
    t1 = d.types()
    unc = np.nonzero((t0 == 2) & (t1 == 0))[0]
    assert len(unc) > 0
    return w, d, unc


def test_refill_aidun_wall_velocity_and_mean_density():
    rng = np.random.default_rng(3)
    n = 40 * 36
    u0 = np.zeros((n, 3))
    u0[:, :2] = 0.01 * rng.uniform(-1, 1, (n, 2))
    c0, vel, om = (19.2, 17.6, 0.0), (0.6, -0.45, 0.0), 0.05
    w, d, unc = _one_refill_step("aidun", u0, c0, vel=vel, omega=om)
    rho, u = d.fields()
    f = d.populations()
    c, wq, _ = O.lattice(O.D2Q9)
    types0 = None
    X1 = np.array(c0) + np.array(vel)
    for k in unc:
        x, y = k % w["nx"], k // w["nx"]
        want_u = np.array([vel[0] - om * (y - X1[1]), vel[1] + om * (x - X1[0])])
        assert np.abs(u[k, :2] - want_u).max() < 1e-13
        # mean density of the neighbours fluid at t and t+1 (their densities
        # after the step, which the refill does not touch)
        t_now = d.types()
        dens = [f[(x + cx) + w["nx"] * (y + cy)].sum() for cx, cy in c[1:, :2]
                if t_now[(x + cx) + w["nx"] * (y + cy)] == 0 and ((x + cx) + w["nx"] * (y + cy)) not in set(unc)]
        assert abs(rho[k] - np.mean(dens)) < 1e-13
    del types0


def test_refill_extrapolate_brute_force():
    """EXTRAPOLATE, checked node by node against an independent evaluation:
    the direction by brute force over the eight lattice directions, the
    three nodes x + k c fluid at t and t+1 (node types), their BGK
    post-collision states computed here from their streamed populations,
    and the quadratic extrapolation of those, which the refilled node holds
    as its post-collision state (a moving circle in a sheared flow)."""
    nx, ny, tau = 40, 36, 0.8
    ys, xs = np.mgrid[0:ny, 0:nx]
    u0 = np.zeros((nx * ny, 3))
    u0[:, 0] = (0.01 + 0.0004 * (xs - 20) - 0.0003 * (ys - 18)).ravel()
    u0[:, 1] = (-0.005 + 0.0002 * (xs - 20) + 0.0005 * (ys - 18)).ravel()
    c0, vel = (17.4, 16.8, 0.0), (0.31, 0.17, 0.0)
    w = _box(nx=nx, ny=ny, tau=tau)
    w["bodies"] = [dict(shape="circle", axes=(4.6,), bc="mls", motion="table", c0=c0, refill="extrapolate",
                        table=W.pose_table(40, c0, vel=vel))]
    d = make_oracle(w, init_rho=np.ones(nx * ny), init_u=u0)
    c, wq, _ = O.lattice(O.D2Q9)
    checked = 0
    for t in range(12):
        t0 = d.types().copy()
        d.step(1)
        t1 = d.types()
        f = d.populations()
        X1 = np.array(c0[:2]) + (t + 1) * np.array(vel[:2])
        for k in np.nonzero((t0 == 2) & (t1 == 0))[0]:
            x, y = k % nx, k // nx
            n = np.array([x, y]) - X1
            score = [(n @ c[i, :2]) / math.hypot(*c[i, :2]) for i in range(1, 9)]
            e = c[1 + int(np.argmax(score)), :2]
            nodes = [(x + m * e[0]) + nx * (y + m * e[1]) for m in (1, 2, 3)]
            assert all(t0[q] == 0 and t1[q] == 0 for q in nodes)
            post = []
            for q in nodes:
                rho = f[q].sum()
                u = (f[q] @ c[:, :2].astype(float)) / rho
                cu = c[:, :2] @ u
                feq = wq * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))
                post.append(f[q] - (f[q] - feq) / tau)
            want = (3 * post[0] - 3 * post[1]) + post[2]
            assert np.abs(f[k] - want).max() < 1e-14
            checked += 1
    assert checked >= 5


@pytest.mark.parametrize("refill", ["mean", "aidun", "extrapolate"])
def test_predicted_sets_equal_forward_sets_at_constant_velocity(refill):
    w = _box(nx=48, ny=40, tau=0.7)
    M = I = 1e15
    w["bodies"] = [dict(shape="ellipse", axes=(5.2, 3.1), bc="mls", motion="free", me="lattice", sets="predicted",
                        c0=(15.3, 19.6, 0.0), theta0=0.3, vel=(0.21, 0.07, 0.0), omega=0.013, mass=M, inertia=I,
                        refill=refill)]
    rho, u = W.random_state(w, rho_amp=0.004, u_amp=0.015, seed=33)
    d = make_oracle(w, init_rho=rho, init_u=u)
    T = 40
    d.step(T)
    rec = d.records(0)
    assert rec[:, 18].sum() > 10 and rec[:, 19].sum() > 10
    scale = np.abs(rec[:, 6:9]).max()
    for t in range(T):
        drv = d.drive(0, t)
        # drive = static terms + predicted node terms; the record holds the
        # static terms and the forward node terms of the same step
        assert np.abs(drv[0:3] - rec[t, 0:3] - rec[t, 6:9]).max() < 1e-12 * scale, t
        assert abs(drv[3] - rec[t, 5] - rec[t, 11]) < 1e-12 * scale * 10, t


def test_two_approximations_agree_for_a_sinking_disc():
    """Sec. III.B.3 reports no appreciable difference between the two
    approximations: a disc sinking in a closed box moves the same way with
    either, to 1 % of its displacement."""
    traj = {}
    for sets in ("previous", "predicted"):
        R = 4.6
        area = math.pi * R * R
        w = dict(name="sink", lattice="D2Q9", nx=40, ny=120, nz=1, tau=0.7, rho0=1.0, eq="bgk",
                 faces=W.CLOSED_FACES, inlet_profile="uniform", inlet_u=0.0, storage="f64", rho_noise=0.0, seed=0,
                 bodies=[dict(shape="circle", axes=(R,), bc="mls", me="lattice", motion="free", sets=sets,
                              c0=(21.3, 90.6, 0.0), mass=1.1 * area, inertia=0.55 * area * R * R,
                              ext_force=(0.0, -0.1 * area * 4e-3, 0.0))])
        d = make_oracle(w)
        d.step(800)
        traj[sets] = np.array([d.pose(0, t) for t in range(801)])
    fall = traj["previous"][0, 1] - traj["previous"][-1, 1]
    assert fall > 2.0
    assert np.abs(traj["previous"][:, 0:2] - traj["predicted"][:, 0:2]).max() < 0.01 * fall
