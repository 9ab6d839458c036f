"""Free bodies (Newton-Euler motion under the flow force: the sedimentation
tests of the paper's Sec. IV, with both approximations of the covered and
uncovered sets of Sec. III.B.3), the refill rules of Sec. III.B.3 and the
backward-in-time lattice force, on the GPU through the C ABI against the CPU
oracle on the same inputs.

A free body's trajectory depends on its force history, so the GPU and the
oracle drift apart by the force differences integrated twice. Bars: FP64
storage, trajectory within 1e-9 nodes (positions) and 1e-11 (velocities)
after 600 steps (force differences ~1e-15 relative; measured values are
printed), link lists bit-exact at the end, force series within 1e-9; FP32
storage, velocity within 1e-4 of its largest value, positions within 1e-3
nodes. Prescribed motions with the AIDUN and EXTRAPOLATE refills keep the
bars of the other prescribed-motion tests (counts bit-exact, force within
1e-10 FP64 / 1e-4 FP32), on both advance kernels (the single-workgroup
list kernel and the many-workgroup one).
"""
import copy
import math

import numpy as np
import pytest

import lbm_workloads as W
from gpu_helpers import make_gpu, ora_series, run_pair, series_error
from oracle_helpers import make_oracle, me_series

pytestmark = pytest.mark.gpu


def _traj_oracle(o, steps):
    return np.array([o.pose(0, t) for t in range(steps + 1)])


def _small_sedimenting(shape="circle", storage="f64", me="lattice", integrator="euler", refill="mean", ratio=1.05,
                       sets="previous"):
    axes = (6.2,) if shape == "circle" else (7.0, 3.6)
    w = W.sedimenting(44, 150, shape, axes, (25.3, 112.6, 0.0), ratio, 1e-3, storage=storage, tau=0.7,
                      theta0=math.pi / 4 if shape == "ellipse" else 0.0, me=me, integrator=integrator, refill=refill)
    w["bodies"][0]["sets"] = sets
    return w


@pytest.mark.parametrize("shape,me,integrator,sets,refill", [
    ("circle", "lattice", "euler", "previous", "mean"), ("circle", "static", "euler", "previous", "mean"),
    ("circle", "comoving", "ab2", "previous", "mean"), ("ellipse", "lattice", "ab2", "previous", "mean"),
    ("ellipse", "comoving", "euler", "previous", "mean"), ("circle", "lattice", "euler", "predicted", "mean"),
    ("ellipse", "lattice", "ab2", "predicted", "extrapolate"), ("circle", "lattice", "euler", "predicted", "aidun")])
def test_free_body_trajectory_f64(shape, me, integrator, sets, refill):
    w = _small_sedimenting(shape, "f64", me, integrator, refill=refill, sets=sets)
    steps = 600
    print(f"free {shape}, {me} force, {integrator}, {sets} sets, {refill} refill, {steps} steps", flush=True)
    g, o = run_pair(w, steps)
    tg = g.trajectory(0, 0, steps + 1)
    to = _traj_oracle(o, steps)
    ex, ev = np.abs(tg[:, 0:2] - to[:, 0:2]).max(), np.abs(tg[:, 4:6] - to[:, 4:6]).max()
    eth, eom = np.abs(tg[:, 3] - to[:, 3]).max(), np.abs(tg[:, 7] - to[:, 7]).max()
    print(f"position {ex:.2e} velocity {ev:.2e} angle {eth:.2e} spin {eom:.2e}; fell {to[0, 1] - to[-1, 1]:.3f} nodes")
    assert to[0, 1] - to[-1, 1] > 0.5  # it sank
    assert ex < 1e-9 and eth < 1e-9 and ev < 1e-11 and eom < 1e-11
    ng, dg, lg = g.links(0)
    no, do, lo = o.links(0)
    assert np.array_equal(ng, no) and np.array_equal(dg, do) and np.abs(lg - lo).max() < 1e-9
    F, T = ora_series(o, 0, "lattice" if me == "lattice" else me)
    rg = g.records(0)
    G = {"static": rg[:, 0:6], "lattice": rg[:, 0:6] + rg[:, 6:12], "comoving": rg[:, 12:18]}[me]
    eF, eT = series_error(G, F, T, w["bodies"][0]["axes"][0], scale=np.abs(F).max())
    print(f"force {eF:.2e} torque {eT:.2e}")
    assert eF < 1e-9 and eT < 1e-9


def test_free_disc_full_size_f32():
    """The paper's sedimenting disc (135 x 1073, r = 1.03) in FP32 storage,
    1500 steps against the FP64 oracle."""
    w = W.sedimenting_disc(ratio=1.03, storage="f32")
    steps = 1500
    print(f"{w['name']}, {steps} steps", flush=True)
    g, o = run_pair(w, steps)
    tg = g.trajectory(0, 0, steps + 1)
    to = _traj_oracle(o, steps)
    vmax = np.abs(to[:, 4:6]).max()
    ev = np.abs(tg[:, 4:6] - to[:, 4:6]).max() / vmax
    ex = np.abs(tg[:, 0:2] - to[:, 0:2]).max()
    print(f"velocity {ev:.2e} of {vmax:.3e}, position {ex:.2e} nodes; fell {to[0, 1] - to[-1, 1]:.3f}")
    assert ev < 1e-4 and ex < 1e-3


def test_free_ellipse_full_size_f32():
    """The paper's sedimenting ellipse (135 x 1676, aspect ratio 2, density
    ratio 1.1, released at 45 degrees) in FP32 storage, 1000 steps against the
    FP64 oracle: velocity and spin within 1e-4 of their largest values,
    position within 1e-3 nodes, angle within 1e-4 of its largest change
    (the spin's bar integrated)."""
    w = W.sedimenting_ellipse(ratio=1.1, storage="f32")
    steps = 1000
    print(f"{w['name']}, {steps} steps", flush=True)
    g, o = run_pair(w, steps)
    tg = g.trajectory(0, 0, steps + 1)
    to = _traj_oracle(o, steps)
    vmax, wmax = np.abs(to[:, 4:6]).max(), np.abs(to[:, 7]).max()
    ev = np.abs(tg[:, 4:6] - to[:, 4:6]).max() / vmax
    ew = np.abs(tg[:, 7] - to[:, 7]).max() / wmax
    ex = np.abs(tg[:, 0:2] - to[:, 0:2]).max()
    dth = np.abs(to[:, 3] - to[0, 3]).max()
    eth = np.abs(tg[:, 3] - to[:, 3]).max()
    print(f"velocity {ev:.2e} of {vmax:.3e}, spin {ew:.2e} of {wmax:.3e}, position {ex:.2e} nodes, "
          f"angle {eth:.2e} of a {dth:.3e} turn; fell {to[0, 1] - to[-1, 1]:.3f}")
    assert ev < 1e-4 and ew < 1e-4 and ex < 1e-3 and eth < 1e-4 * dth
    assert to[0, 1] - to[-1, 1] > 0.1 and dth > 0


def test_free_sphere_d3q19_f64():
    """A free sphere sinking in a closed D3Q19 box, FP64, 300 steps."""
    R = 4.2
    area = 4.0 / 3.0 * math.pi * R ** 3
    M = 1.2 * area
    w = dict(name="free_sphere", lattice="D3Q19", nx=24, ny=48, nz=24, tau=0.7, rho0=1.0, eq="bgk",
             faces=W.CLOSED_FACES, inlet_profile="uniform", inlet_u=0.0, storage="f64", rho_noise=0.0, seed=0,
             bodies=[dict(shape="sphere", axes=(R, R, R), bc="mls", me="lattice", motion="free",
                          c0=(12.3, 33.6, 11.8), mass=M, inertia=0.4 * M * R * R,
                          ext_force=(0.0, -0.2 * area * 3e-4, 0.0))])
    steps = 300
    g, o = run_pair(w, steps)
    tg = g.trajectory(0, 0, steps + 1)
    to = _traj_oracle(o, steps)
    ex, ev = np.abs(tg[:, 0:3] - to[:, 0:3]).max(), np.abs(tg[:, 4:7] - to[:, 4:7]).max()
    print(f"position {ex:.2e} velocity {ev:.2e}; fell {to[0, 1] - to[-1, 1]:.3f}")
    assert ex < 1e-9 and ev < 1e-11 and to[0, 1] - to[-1, 1] > 0.1


def test_free_body_rejections():
    from paper_1407_4524_amd import Batch, LbmError
    w = _small_sedimenting()
    b = dict(w["bodies"][0])
    with pytest.raises(LbmError):
        make_gpu(dict(w, bodies=[dict(b, mass=0.0)]))
    d = make_gpu(dict(w, bodies=[]))
    B = Batch()
    B.add(d)
    with pytest.raises(LbmError):
        d.set_body(0, **b)
    B.close()


@pytest.mark.parametrize("refill", ["aidun", "extrapolate"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_refill_rules_list_kernel(refill, storage):
    """The oscillating cylinder at 1/10 scale (200x80, R=4) with the refill
    rule swapped: counts bit-exact, lattice and comoving forces."""
    w = W.channel_oscillating_f32(scale=10)
    w["storage"] = storage
    w["bodies"][0]["refill"] = refill
    steps = 800
    print(f"refill {refill}, {storage}, {steps} steps", flush=True)
    g, o = run_pair(w, steps)
    rg, ro = g.records(0), o.records(0)
    assert (rg[:, 18:20] == ro[:, 18:20]).all() and ro[:, 19].sum() > 0
    tol = 1e-10 if storage == "f64" else 1e-4
    for mode, G in (("lattice", rg[:, 0:6] + rg[:, 6:12]), ("comoving", rg[:, 12:18])):
        F, T = ora_series(o, 0, mode)
        eF, eT = series_error(G, F, T, 4.0)
        print(f"{mode}: F {eF:.2e} T {eT:.2e}")
        assert eF < tol and eT < tol


@pytest.mark.parametrize("refill", ["aidun", "extrapolate"])
def test_refill_rules_box_kernels(refill):
    """A translating sphere of radius 8 in D3Q19 (its surface list is too long
    for the list kernel: the many-workgroup advance runs) and a rotating 80x40
    ellipse, FP32: counts bit-exact, lattice force within 1e-4."""
    R = 8.0
    w3 = dict(name="sphere_move", lattice="D3Q19", nx=64, ny=40, nz=40, tau=0.7, rho0=1.0, eq="bgk",
              faces=W.PERIODIC_FACES, inlet_profile="uniform", inlet_u=0.0, storage="f32", rho_noise=0.0, seed=0,
              bodies=[dict(shape="sphere", axes=(R, R, R), bc="mls", me="lattice", motion="const_vel",
                           c0=(20.3, 19.7, 20.2), vel=(0.05, 0.01, -0.02), refill=refill)])
    w2 = copy.deepcopy(W.batched_domains(count=1, seed=0)[0])
    w2.update(nx=420, ny=300)
    w2["bodies"] = [dict(shape="ellipse", axes=(80.0, 40.0), bc="mls", me="lattice", motion="rotate",
                         c0=(150.0, 150.0, 0.0), theta0=0.2, omega=5e-4, refill=refill)]
    for w, steps, R_ in ((w3, 80, R), (w2, 40, 80.0)):
        print(f"refill {refill}: {w['name']}, {steps} steps", flush=True)
        g, o = run_pair(w, steps)
        rg, ro = g.records(0), o.records(0)
        assert (rg[:, 18:20] == ro[:, 18:20]).all() and ro[:, 19].sum() > 0
        F, T = ora_series(o, 0, "lattice")
        eF, eT = series_error(rg[:, 0:6] + rg[:, 6:12], F, T, R_, scale=max(np.abs(F).max(), np.abs(T).max() / R_))
        print(f"lattice: F {eF:.2e} T {eT:.2e}")
        assert eF < 1e-4 and eT < 1e-4
        g.close()


def test_backward_lattice_force():
    """LBM_ME_LATTICE_BACKWARD: the static terms of step t plus the node
    terms of step t-1, for any window of steps, equal to the oracle's."""
    w = W.channel_oscillating_f32(scale=10)
    w["storage"] = "f64"
    w["bodies"][0]["me"] = "lattice_backward"
    g, o = run_pair(w, 600)
    F, T = me_series(o.records(0), "lattice_backward")
    ft = g.force_torque(0)
    eF, eT = series_error(ft, F, T, 4.0)
    assert eF < 1e-10 and eT < 1e-10
    part = g.force_torque(0, 250, 100)  # a window that starts after step 0 takes step 249's node terms
    assert np.array_equal(part, ft[250:350])
