"""GPU (HIP, through the C ABI) against the CPU oracle on the same seeded inputs.

Bars:
* boundary-link lists (node, direction), fractional distances and the
  covered/uncovered node counts: bit-exact;
* FP64 storage: force/torque series within 1e-10 (relative, drag-scaled),
  velocity within 1e-12;
* FP32 storage: force/torque within 1e-4, FP16-shifted storage within 1e-3;
  velocity bounds are stated per case below with their derivation.
"""
import math

import numpy as np
import pytest

import lbm_workloads as W
from gpu_helpers import make_gpu, ora_series, run_pair, series_error, velocity_error
from oracle_helpers import make_oracle

pytestmark = pytest.mark.gpu


def box(lattice="D2Q9", nx=32, ny=24, nz=1, tau=0.8, eq="bgk", faces=W.PERIODIC_FACES, storage="f64",
        bodies=()):
    return dict(name="box", lattice=lattice, nx=nx, ny=ny, nz=nz if lattice == "D3Q19" else 1, tau=tau,
                rho0=1.0, eq=eq, faces=faces, inlet_profile="uniform", inlet_u=0.0, storage=storage,
                rho_noise=0.0, seed=0, bodies=list(bodies))


def same_links(g, o, body=0):
    ng, dg, lg = g.links(body)
    no, do, lo = o.links(body)
    assert len(ng) == len(no), (len(ng), len(no))
    assert (ng == no).all() and (dg == do).all()
    return lg, lo


# ---------------------------------------------------------------------------
# FP64: the algorithm itself


def test_channel_cylinder_f64():
    """100x50 channel, static cylinder R=5 with halfway bounce-back, FP64,
    2000 steps: identical 104-link list, force/torque every step and the
    final velocity field equal to the oracle's."""
    w = W.channel_cylinder_f64()
    rho = W.density_noise(w)
    g, o = run_pair(w, 0, init_rho=rho)
    lg, lo = same_links(g, o)
    assert len(lg) == 104 and (lg == 0.5).all()
    g.step(w["steps"])
    o.step(w["steps"])
    F, T = ora_series(o, 0, "static")
    eF, eT = series_error(g.force_torque(0), F, T, 5.0)
    du = velocity_error(g, o)
    print(f"F err {eF:.2e} T err {eT:.2e} u err {du:.2e}")
    assert eF < 1e-10 and eT < 1e-10 and du < 1e-12


def test_channel_cylinder_mls_f64_delta_bit_exact():
    """Interpolated rule on the same cylinder: Delta per link equal bit for bit,
    and the force/torque series within 1e-10."""
    w = W.channel_cylinder_f64()
    w["bodies"][0]["bc"] = "mls"
    w["bodies"][0]["c0"] = (25.3, 24.6, 0.0)
    g, o = run_pair(w, 0)
    lg, lo = same_links(g, o)
    assert (lg == lo).all(), np.abs(lg - lo).max()
    g.step(400)
    o.step(400)
    F, T = ora_series(o, 0, "static")
    eF, eT = series_error(g.force_torque(0), F, T, 5.0)
    print(f"F err {eF:.2e} T err {eT:.2e}")
    assert eF < 1e-10 and eT < 1e-10


@pytest.mark.parametrize("lat,eq,shape", [("D2Q9", "bgk", (37, 23, 1)), ("D2Q9", "heluo", (300, 5, 1)),
                                          ("D3Q19", "bgk", (19, 13, 11)), ("D2Q9", "bgk", (3, 3, 1)),
                                          ("D3Q19", "bgk", (3, 3, 3)), ("D2Q9", "bgk", (32000, 3, 1)),
                                          ("D3Q19", "bgk", (3, 3, 32000))])
def test_periodic_box_f64(lat, eq, shape):
    """Random density and velocity on a periodic box (ragged sizes, from the
    smallest box of 3 nodes per axis to an axis of 32000, the longest one
    allowed): fields after 150 steps equal the oracle's; mass is conserved."""
    w = box(lat, *shape, tau=0.7, eq=eq)
    rho, u = W.random_state(w, seed=21)
    g, o = run_pair(w, 150, init_rho=rho, init_u=u)
    rg, ug = g.fields()
    ro, uo = o.fields()
    assert np.abs(ug - uo).max() < 1e-12 and np.abs(rg - ro).max() < 1e-12
    assert abs(rg.sum() - rho.sum()) < 1e-11 * rho.sum()


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_body_at_rest_gpu(lat):
    """A body at rest in fluid at rest: zero force and torque, unchanged state."""
    w = box(lat, 30, 24, 20, faces=W.CHANNEL_FACES if lat == "D2Q9" else W.DUCT_FACES,
            bodies=[dict(shape="circle", axes=(4.5, 4.5, 4.5), bc="mls", me="static", motion="static",
                         c0=(12.3, 11.6, 9.8))])
    g = make_gpu(w)
    g.step(30)
    rec = g.records(0)
    assert np.abs(rec[:, 0:6]).max() < 1e-13
    rho, u = g.fields()
    m = g.types() == 0
    assert np.abs(rho[m] - 1).max() < 1e-15 and np.abs(u[m]).max() < 1e-15


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_uniform_flow_translating_body_gpu(lat):
    """Uniform flow past a body moving with it (FP64): the fluid stays uniform,
    the comoving force is zero, covered/uncovered counts and the lattice-frame
    force equal the oracle's every step."""
    V = np.array([0.06, -0.035, 0.0 if lat == "D2Q9" else 0.025])
    if lat == "D2Q9":
        w = box(lat, 40, 30, tau=0.75)
        c0, R = (15.3, 14.8, 0.0), 5.1
    else:
        w = box(lat, 24, 20, 19, tau=0.75)
        c0, R = (10.2, 10.7, 8.9), 3.6
    w["bodies"] = [dict(shape="circle", axes=(R, R, R), bc="mls", me="lattice", motion="const_vel", c0=c0,
                        vel=tuple(V))]
    n = w["nx"] * w["ny"] * w["nz"]
    g, o = run_pair(w, 50, init_rho=np.ones(n), init_u=np.tile(V, (n, 1)))
    rg, ug = g.fields()
    m = g.types() == 0
    assert np.abs(ug[m] - V).max() < 1e-14
    rec_g, rec_o = g.records(0), o.records(0)
    assert (rec_g[:, 18:20] == rec_o[:, 18:20]).all()
    assert np.abs(rec_g[:, 12:15]).max() < 1e-13
    assert np.abs(rec_g[:, 0:12] - rec_o[:, 0:12]).max() < 1e-12
    same_links(g, o)


def test_moving_ellipse_f64_links_and_counts():
    """Translating + rotating ellipse (pose table) in a channel, FP64:
    covered/uncovered counts every step and the final link list bit-exact;
    all three force/torque forms within 1e-10."""
    w = W.channel_cylinder_f64()
    steps = 300
    c0 = (30.2, 24.7, 0.0)
    tab = W.pose_table(steps + 2, c0, theta0=0.4, vel=(0.03, 0.01, 0.0), omega=0.01)
    w["bodies"] = [dict(shape="ellipse", axes=(6.0, 3.0), bc="mls", me="lattice", motion="table", c0=c0,
                        table=tab)]
    g, o = run_pair(w, steps)
    rg, ro = g.records(0), o.records(0)
    assert (rg[:, 18:20] == ro[:, 18:20]).all() and ro[:, 18].sum() > 0
    lg, lo = same_links(g, o)
    assert (lg == lo).all()
    for mode in ("static", "lattice", "comoving"):
        F, T = ora_series(o, 0, mode)
        G = {"static": rg[:, 0:6], "lattice": rg[:, 0:6] + rg[:, 6:12], "comoving": rg[:, 12:18]}[mode]
        eF, eT = series_error(G, F, T, 6.0)
        print(mode, f"F err {eF:.2e} T err {eT:.2e}")
        assert eF < 1e-10 and eT < 1e-10


# ---------------------------------------------------------------------------
# the configured workloads at the oracle's sizes


def test_oscillating_cylinder_f32_200x80():
    """The oscillating-cylinder channel at 1/10 scale (200x80, R=4, amplitude 2,
    period 400), FP32 storage, interpolated rule, lattice-frame ME, 2000 steps:
    covered/uncovered counts bit-exact every step, force/torque within 1e-4.
    Velocity bound 5e-6 (1.25e-4 of u_max): FP32 rounds each stored deviation
    (|h| < 0.02) to 2^-24 relative, i.e. < 1.2e-9 per value per step; the
    velocity error is a sum of such roundings damped by viscosity, far below
    the linear-growth bound 2000 * 9 * 1.2e-9 = 2.2e-5."""
    w = W.channel_oscillating_f32(scale=10)
    g, o = run_pair(w, w["steps"])
    rg, ro = g.records(0), o.records(0)
    assert (rg[:, 18:20] == ro[:, 18:20]).all() and ro[:, 18].sum() > 0
    same_links(g, o)
    F, T = ora_series(o, 0, "lattice")
    G = rg[:, 0:6] + rg[:, 6:12]
    eF, eT = series_error(G, F, T, 4.0)
    Fc, Tc = ora_series(o, 0, "comoving")
    eFc, eTc = series_error(rg[:, 12:18], Fc, Tc, 4.0)
    du = velocity_error(g, o)
    print(f"lattice F {eF:.2e} T {eT:.2e}; comoving F {eFc:.2e} T {eTc:.2e}; u {du:.2e}")
    assert eF < 1e-4 and eT < 1e-4 and eFc < 1e-4 and eTc < 1e-4
    assert du < 5e-6


@pytest.mark.parametrize("storage,tol_ft,tol_u", [("f32", 1e-4, 5e-6), ("f16", 1e-3, 3e-4)])
def test_duct_sphere_64x32x32(storage, tol_ft, tol_u):
    """D3Q19 duct at 1/4 scale (64x32x32, sphere R=4, plug inlet 0.03), 600
    steps, FP32 and FP16-shifted storage against the FP64 oracle. FP16 stores
    |h| < 0.02 with a half-ulp of 2^-11 relative (< 1e-5 per value per step)."""
    w = W.duct_sphere(scale=4, storage=storage)
    g, o = run_pair(w, 600)
    same_links(g, o)
    F, T = ora_series(o, 0, "static")
    eF, eT = series_error(g.force_torque(0), F, T, 4.0)
    du = velocity_error(g, o)
    print(f"{storage}: F {eF:.2e} T {eT:.2e} u {du:.2e}")
    assert eF < tol_ft and eT < tol_ft and du < tol_u


def test_duct_sphere_64x32x32_long_horizon():
    """The same quarter-scale duct over 3000 steps (five times the test
    above), FP32 and FP16 storage against one FP64 oracle run: the errors
    stay within the same bounds as the flow develops (measured: FP32 force
    1.2e-6, FP16 3.8e-4)."""
    steps = 3000
    w = W.duct_sphere(scale=4, storage="f32")
    print(f"quarter-scale duct, {steps} steps, FP32 and FP16", flush=True)
    o = make_oracle(w)
    o.step(steps)
    F, T = ora_series(o, 0, "static")
    for storage, tol_ft, tol_u in (("f32", 1e-4, 5e-6), ("f16", 1e-3, 3e-4)):
        g = make_gpu(W.duct_sphere(scale=4, storage=storage))
        g.step(steps)
        same_links(g, o)
        eF, eT = series_error(g.force_torque(0), F, T, 4.0)
        du = velocity_error(g, o)
        print(f"{storage}: F {eF:.2e} T {eT:.2e} u {du:.2e}", flush=True)
        assert eF < tol_ft and eT < tol_ft and du < tol_u
        g.close()


@pytest.mark.parametrize("storage,tol_ft,tol_u", [("f32", 1e-4, 5e-6), ("f16", 1e-3, 3e-4)])
def test_duct_sphere_full_size_first_steps(storage, tol_ft, tol_u):
    """The full 256x128x128 duct with the sphere of radius 16 (the benchmarked
    size and launch configuration: one sweep per step, the FP16 face rules in
    a launch of their own), 3 steps against the oracle at full size: links,
    force/torque and velocity. The fluid starts moving at the inlet speed
    everywhere, so the sphere's force is the impulsive start's from the first
    step rather than density noise."""
    w = W.duct_sphere(scale=1, storage=storage)
    n = w["nx"] * w["ny"] * w["nz"]
    u0 = np.zeros((n, 3))
    u0[:, 0] = w["inlet_u"]
    print(f"full-size duct {storage}: {w['nx']}x{w['ny']}x{w['nz']}, 3 steps", flush=True)
    g, o = run_pair(w, 3, init_u=u0)
    same_links(g, o)
    F, T = ora_series(o, 0, "static")
    eF, eT = series_error(g.force_torque(0), F, T, 16.0, scale=np.abs(F).max())
    du = velocity_error(g, o)
    print(f"{storage}: F {eF:.2e} T {eT:.2e} u {du:.2e} (|F| max {np.abs(F).max():.3e})")
    assert np.abs(F).max() > 1e-3
    assert eF < tol_ft and eT < tol_ft and du < tol_u


@pytest.mark.parametrize("lattice,storage,faces", [
    ("D2Q9", "f32", "ragged"), ("D2Q9", "f16", "ragged"), ("D3Q19", "f16", "ragged"), ("D2Q9", "f32", "wall_x"),
    ("D3Q19", "f32", "wall_x")])
def test_ragged_rows_and_odd_start(lattice, storage, faces):
    """Rows of odd length (a ragged last tile) and, with a wall face at x = 0,
    rows that start at x = 1, against the FP64 oracle, with a moving body so
    that the split schedule's hole cuts tiles too (with the wall in place of
    the inlet, the body's motion alone drives the flow, so those cases run
    FP32)."""
    import copy
    if lattice == "D2Q9":
        w = copy.deepcopy(W.channel_oscillating_f32(scale=10))
        w.update(nx=63, ny=33, storage=storage)
        w["bodies"][0].update(c0=(20.0, 16.0, 0.0), axes=(4.0,), amp=(0.0, 1.0, 0.0), period=100.0)
        R = 4.0
    else:
        w = copy.deepcopy(W.duct_sphere(scale=4, storage=storage))
        w.update(nx=33, ny=18, nz=17)
        w["bodies"][0].update(c0=(12.0, 9.0, 8.5), axes=(3.5,), motion="oscillate", amp=(0.0, 0.0, 1.0),
                              period=100.0, me="lattice")
        R = 3.5
    if faces == "wall_x":
        f = list(w["faces"])
        f[0] = W.WALL
        w["faces"] = tuple(f)
    steps = 150
    print(f"{lattice} {storage} {faces}: {w['nx']}x{w['ny']}x{w['nz']}", flush=True)
    g, o = run_pair(w, steps)
    rg, ro = g.records(0), o.records(0)
    assert (rg[:, 18:20] == ro[:, 18:20]).all()
    F, T = ora_series(o, 0, "lattice")
    eF, eT = series_error(rg[:, 0:6] + rg[:, 6:12], F, T, R)
    du = velocity_error(g, o)
    tol_ft, tol_u = (1e-4, 5e-6) if storage == "f32" else (1e-3, 3e-4)
    print(f"F {eF:.2e} T {eT:.2e} u {du:.2e}", flush=True)
    assert eF < tol_ft and eT < tol_ft and du < tol_u


def test_oscillating_cylinder_full_size_first_steps():
    """The full 2000x800 oscillating-cylinder channel (the benchmarked size and
    launch configuration), FP32, first 3 steps against the oracle at full
    size: links, counts, force/torque and velocity."""
    w = W.channel_oscillating_f32(scale=1)
    g, o = run_pair(w, 3)
    same_links(g, o)
    rg, ro = g.records(0), o.records(0)
    assert (rg[:, 18:20] == ro[:, 18:20]).all()
    F, T = ora_series(o, 0, "lattice")
    # in the first steps the drag is still ~0: measure against the largest force component
    eF, eT = series_error(rg[:, 0:6] + rg[:, 6:12], F, T, 40.0, scale=np.abs(F).max())
    du = velocity_error(g, o)
    print(f"F {eF:.2e} T {eT:.2e} u {du:.2e}")
    assert eF < 1e-4 and eT < 1e-4 and du < 5e-6


# ---------------------------------------------------------------------------
# the split schedule (the nodes away from a moving body updated on a second
# stream, overlapping the body's advance) against the plain one: bitwise the
# same


def _moving(case):
    import copy
    if case == "oscillating_f32":
        return W.channel_oscillating_f32(scale=10), 300
    if case == "ellipse_f64":
        w = copy.deepcopy(W.channel_cylinder_f64())
        w["bodies"] = [dict(shape="ellipse", axes=(6.0, 3.0), bc="mls", me="lattice", motion="rotate",
                            c0=(25.0, 25.0, 0.0), theta0=0.3, omega=0.01)]
        return w, 200
    w = copy.deepcopy(W.duct_sphere(scale=4, storage="f16"))
    w["bodies"][0].update(motion="oscillate", amp=(0.0, 0.0, 2.0), period=100.0, me="lattice")
    return w, 100


@pytest.mark.parametrize("case,own_stream", [("oscillating_f32", True), ("ellipse_f64", False),
                                             ("duct_f16", True)])
def test_split_schedule_bitwise_equals_plain(case, own_stream):
    """the split schedule against the default one (a moving body's domain
    steps as a one-member batch, whose overlapped step times the update of
    the nodes away from the body); on the default stream the second stream
    is a plain one, on a stream of the domain's own it is CU-masked"""
    import torch
    w, steps = _moving(case)
    print(f"split vs plain schedule: {w['name']} ({case}), {steps} steps, own stream {own_stream}", flush=True)
    if own_stream:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            a = make_gpu(w, split_schedule=True)
    else:
        a = make_gpu(w, split_schedule=True)
    b = make_gpu(w)
    a.timing_enable(1)
    b.timing_enable(1)
    for chunk in (1, steps // 2 - 1, steps - steps // 2):  # several calls: the hand-over between them
        a.step(chunk)
        b.step(chunk)
    _, na, nodes_a = a.timing_read("stream_collide")
    _, nn, nodes_n = a.timing_read("near_box")
    _, nb, nodes_b = b.timing_read("stream_collide")
    dims = 2 if w["lattice"] == "D2Q9" else 3
    active = 1
    for ax, n in enumerate((w["nx"], w["ny"], w.get("nz", 1) if dims == 3 else 1)):
        active *= n - ((w["faces"][2 * ax] == W.WALL) + (w["faces"][2 * ax + 1] == W.WALL) if ax < dims else 0)
    assert na == nn == nb == steps, "every split step is a far and a near launch"
    assert b.timing_read("near_box")[1] == 0
    assert nodes_a + nodes_n == steps * active
    assert 0 < nodes_b < steps * active
    assert a.timing_read("body")[1] == steps + 1  # the advances and the first step's link rule
    assert np.array_equal(a.records(0), b.records(0))
    rho_a, u_a = a.fields()
    rho_b, u_b = b.fields()
    assert np.array_equal(rho_a, rho_b, equal_nan=True) and np.array_equal(u_a, u_b, equal_nan=True)
    a.close()
    b.close()


@pytest.mark.parametrize("case", ["sphere_f32", "sphere_f16_face_records", "cylinder_f64"])
def test_split_schedule_fixed_body_bitwise_equals_plain(case):
    """a body with fixed links in the split schedule (its link rule and the
    near box's update on the domain's stream beside the far update on the
    second) against the plain schedule, bit for bit: records, fields and,
    with face records on, the faces' momentum exchange; the default is the
    plain schedule"""
    import torch
    if case == "cylinder_f64":
        w, steps, faces = W.channel_cylinder_f64(), 300, False
    else:
        w, steps, faces = W.duct_sphere(scale=4, storage=case[7:10]), 120, case.endswith("records")
    print(f"split vs plain schedule, fixed body: {w['name']} ({case}), {steps} steps", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = make_gpu(w, split_schedule=1, face_records=faces)
    b = make_gpu(w, split_schedule=-1, face_records=faces)
    c = make_gpu(w, face_records=faces)
    for d in (a, b, c):
        d.timing_enable(1)
    for chunk in (1, steps // 2 - 1, steps - steps // 2):
        for d in (a, b, c):
            d.step(chunk)
    _, na, nodes_a = a.timing_read("stream_collide")
    _, nn, nodes_n = a.timing_read("near_box")
    _, nb, nodes_b = b.timing_read("stream_collide")
    assert na == nn == nb == steps, "every split step is a far and a near launch"
    assert nodes_a + nodes_n == nodes_b and 0 < nodes_n < nodes_a
    assert a.timing_read("body")[1] == b.timing_read("body")[1] == steps  # the link rule once per step
    assert c.timing_read("near_box")[1] == 0, "a fixed body keeps the plain schedule by default"
    assert np.array_equal(a.records(0), b.records(0)) and np.array_equal(c.records(0), b.records(0))
    if faces:
        assert np.array_equal(a.face_records(0, steps), b.face_records(0, steps))
    rho_a, u_a = a.fields()
    rho_b, u_b = b.fields()
    assert np.array_equal(rho_a, rho_b, equal_nan=True) and np.array_equal(u_a, u_b, equal_nan=True)
    for d in (a, b, c):
        d.close()


def test_rotating_ellipsoid_with_a_large_surface():
    """a moving body whose region fits the one-workgroup kernel but whose
    near-surface node list would not is advanced by the box-scan kernel
    (the host bounds the list before choosing); against the oracle"""
    w = dict(name="duct_ellipsoid_f32", lattice="D3Q19", nx=44, ny=36, nz=36, tau=0.7, rho0=1.0, eq="bgk",
             faces=W.DUCT_FACES, inlet_profile="parabolic", inlet_u=0.04, storage="f32", rho_noise=0.0, seed=0,
             bodies=[dict(shape="ellipse", axes=(10.0, 7.0, 6.0), bc="mls", me="lattice", motion="rotate",
                          c0=(20.0, 18.0, 18.0), theta0=0.4, omega=0.02)])
    steps = 120
    g, o = run_pair(w, steps)
    lg, lo = same_links(g, o)
    F, T = ora_series(o, 0, "lattice")
    ft = g.force_torque(0, 0, steps)
    # the flow starts at rest and the body spins fast: its own motion, not the
    # drag, sets the force scale here, so each series is measured against its
    # own largest magnitude
    eF = np.abs(ft[:, 0:3] - F).max() / np.abs(F).max()
    eT = np.abs(ft[:, 3:6] - T).max() / np.abs(T).max()
    print(f"ellipsoid: eF {eF:.2e} eT {eT:.2e}", flush=True)
    assert eF < 1e-4 and eT < 1e-4
    g.close()
    o.close()


# ---------------------------------------------------------------------------
# error paths and calls that do nothing, on a live domain


def test_domain_error_paths_and_empty_calls():
    """step(0) changes nothing; a negative step count, a body id out of range
    or in use, a body that would leave the interior and steps outside the
    record ring each give their status, and the domain stays usable (the
    failed body id is free again)."""
    from paper_1407_4524_amd import LbmError
    w = W.channel_cylinder_f64()
    g = make_gpu(w, record_capacity=16)
    print("error paths: channel 100x50, record ring of 16 steps", flush=True)
    rho0, u0 = g.fields()
    g.step(0)
    assert g.t == 0
    rho1, u1 = g.fields()
    assert np.array_equal(rho0, rho1, equal_nan=True) and np.array_equal(u0, u1, equal_nan=True)

    def status(fn, *a, **kw):
        with pytest.raises(LbmError) as e:
            fn(*a, **kw)
        return e.value.status

    assert status(g.step, -1) == -1
    body = dict(w["bodies"][0])
    assert status(g.set_body, 0, **body) == -6                      # id in use
    assert status(g.set_body, 4, **body) == -1                      # id out of range
    outside = dict(body, c0=(97.0, 25.0, 0.0))
    assert status(g.set_body, 1, **outside) == -4                   # leaves the interior
    assert status(g.force_torque, 0, 0, 1) == -4                    # no step taken yet
    g.step(20)
    assert g.t == 20
    assert status(g.force_torque, 0, 0, 1) == -4                    # step 0 left the ring of 16
    assert np.isfinite(g.force_torque(0, 4, 16)).all()              # the last 16 steps are there
    g.set_body(1, **dict(body, c0=(70.2, 24.7, 0.0)))               # the failed id is free again
    g.step(5)
    assert np.isfinite(g.force_torque(1, 20, 5)).all()
    g.close()
