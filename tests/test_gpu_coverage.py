"""GPU (HIP, through the C ABI) against the CPU oracle on the paths the other
parity tests leave out: served requests, 3D batches, the global-memory
advance of a large moving body, the Couette pair with an outer circle, the
quasi-incompressible equilibrium with a body in FP32, halfway bounce-back on
a moving body, two bodies in one domain, all eight seeded members of a
batch, the face records (walls, inlet, outlet) and the wall force against the
pressure drop, the NaN-filled debug domain, the device instability flag and
the covered/uncovered counts.

Bars as in test_gpu_parity: link lists, Delta and covered/uncovered counts
bit-exact; FP64 force/torque within 1e-10 (relative to the largest drag),
FP32 within 1e-4, FP16-shifted within 1e-3; every measured error is printed
beside its bound.
"""
import copy
import math

import numpy as np
import pytest

import lbm_workloads as W
from gpu_helpers import make_gpu, ora_series, run_pair, series_error, velocity_error
from oracle_helpers import make_oracle, me_series

pytestmark = pytest.mark.gpu

TOL_FT = {"f64": 1e-10, "f32": 1e-4, "f16": 1e-3}


def same_links(g, o, body=0):
    ng, dg, lg = g.links(body)
    no, do, lo = o.links(body)
    assert len(ng) == len(no), (len(ng), len(no))
    assert (ng == no).all() and (dg == do).all() and (lg == lo).all()
    return len(ng)


def check_series(rec_g, o, body, mode, R, tol, label):
    """force/torque series error of one ME form: differences over the force
    scale (the largest oracle force, or the largest torque over R when the
    flow exerts almost no force, e.g. a body spun up in fluid at rest)"""
    F, T = ora_series(o, body, mode)
    G = {"static": rec_g[:, 0:6], "lattice": rec_g[:, 0:6] + rec_g[:, 6:12], "comoving": rec_g[:, 12:18]}[mode]
    eF, eT = series_error(G, F, T, R, scale=max(np.abs(F).max(), np.abs(T).max() / R, 1e-30))
    print(f"{label}: F err {eF:.2e} T err {eT:.2e} (bound {tol:.0e})", flush=True)
    assert eF < tol and eT < tol


def box(lattice="D2Q9", nx=32, ny=24, nz=1, tau=0.8, eq="bgk", faces=W.PERIODIC_FACES, storage="f64", bodies=()):
    return dict(name="box", lattice=lattice, nx=nx, ny=ny, nz=nz if lattice == "D3Q19" else 1, tau=tau, rho0=1.0,
                eq=eq, faces=faces, inlet_profile="uniform", inlet_u=0.0, storage=storage, rho_noise=0.0, seed=0,
                bodies=list(bodies))


# ---------------------------------------------------------------------------
# served results against the oracle


def test_served_requests_against_the_oracle():
    """a mixed stream (2D and 3D, FP32 and FP16-shifted, static and rotating
    bodies) served with continuous batching; every result's last force and
    torque against an oracle run of the same request for the same steps"""
    from paper_1407_4524_amd.serve import GpuEngine, Server
    reqs = W.serving_requests(count=6, seed=12, rate=500.0, max_steps=600, scale=8, d3_fraction=0.5)
    kinds = {(r["spec"]["lattice"], r["spec"]["storage"]) for r in reqs}
    print("requests:", [(r["spec"]["name"], r["spec"]["bodies"][0]["shape"], r["spec"]["bodies"][0]["motion"])
                        for r in reqs], flush=True)
    assert len(kinds) >= 3
    eng = GpuEngine(record_capacity=2048)
    srv = Server(eng, 64 * 2 ** 30, epoch=500, window=500, tol=1e-14)
    served = {r.id: r for r in srv.run(reqs)}
    eng.close()
    for r in reqs:
        res = served[r["id"]]
        assert not res.failed, res.error
        o = make_oracle(r["spec"])
        o.step(res.steps)
        F, T = me_series(o.records(0), "lattice")
        R = r["spec"]["bodies"][0]["axes"][0]
        scale = max(np.abs(F[:, 0]).max(), 1e-30)
        eF = np.abs(np.array(res.force_torque[0:3]) - F[-1]).max() / scale
        eT = np.abs(np.array(res.force_torque[3:6]) - T[-1]).max() / (scale * R)
        tol = TOL_FT[r["spec"]["storage"]]
        print(f"request {r['id']} {r['spec']['name']} ({res.steps} steps): F err {eF:.2e} T err {eT:.2e} "
              f"(bound {tol:.0e})", flush=True)
        assert eF < tol and eT < tol
        o.close()


# ---------------------------------------------------------------------------
# batches against the oracle


def ducts_3d():
    """three small D3Q19 FP32 ducts: a sphere, a rotating ellipsoid, a sphere
    off-centre (bounding boxes plus two nodes inside the walls, checked)"""
    base = dict(lattice="D3Q19", tau=0.7, rho0=1.0, eq="bgk", faces=W.DUCT_FACES, inlet_profile="uniform",
                inlet_u=0.03, storage="f32", rho_noise=0.0, seed=0)
    ws = [dict(base, name="duct_a", nx=36, ny=24, nz=24,
               bodies=[dict(shape="circle", axes=(4.0,), bc="mls", me="lattice", motion="static",
                            c0=(12.2, 11.7, 12.4))]),
          dict(base, name="duct_b", nx=40, ny=26, nz=24,
               bodies=[dict(shape="ellipse", axes=(5.0, 3.5, 3.0), bc="mls", me="lattice", motion="rotate",
                            c0=(14.0, 12.3, 11.2), theta0=0.3, omega=0.01)]),
          dict(base, name="duct_c", nx=33, ny=22, nz=25, tau=0.9,
               bodies=[dict(shape="circle", axes=(3.2,), bc="halfway", me="lattice", motion="static",
                            c0=(10.5, 9.4, 13.1))])]
    for w in ws:
        b = w["bodies"][0]
        r = max(b["axes"])
        for a, n in zip(range(3), (w["nx"], w["ny"], w["nz"])):
            lo = 0 if a == 0 else 1
            hi = n - 1 if a == 0 else n - 2
            assert math.floor(b["c0"][a] - r) - 2 >= lo and math.ceil(b["c0"][a] + r) + 2 <= hi
    return ws


def test_3d_batch_against_the_oracle():
    from paper_1407_4524_amd import Batch
    ws = ducts_3d()
    steps = 150
    batch = Batch()
    members = [make_gpu(w) for w in ws]
    for d in members:
        batch.add(d)
    batch.step(steps)
    for w, d in zip(ws, members):
        o = make_oracle(w)
        o.step(steps)
        rg, ro = d.records(0), o.records(0)
        assert (rg[:, 18:20] == ro[:, 18:20]).all()
        n = same_links(d, o)
        check_series(rg, o, 0, "lattice", w["bodies"][0]["axes"][0], TOL_FT["f32"], f"3D batch {w['name']} ({n} links)")
        du = velocity_error(d, o)
        print(f"  u err {du:.2e} (bound 5e-6)", flush=True)
        assert du < 5e-6
        o.close()
    batch.close()


def seeded_batch(count=8, seed=3, max_side=120):
    out = []
    for w in W.batched_domains(count=count, seed=seed):
        w = copy.deepcopy(w)
        s = max(w["nx"], w["ny"]) / max_side
        if s > 1:
            w["nx"], w["ny"] = int(w["nx"] / s), int(w["ny"] / s)
            b = w["bodies"][0]
            b["axes"] = tuple(max(4.0, a / s) for a in b["axes"])
            b["c0"] = (max(b["c0"][0] / s, b["axes"][0] + 4), min(max(b["c0"][1] / s, b["axes"][0] + 4),
                                                                   w["ny"] - b["axes"][0] - 5), 0.0)
        out.append(w)
    return out


def test_all_eight_seeded_batch_members_against_the_oracle():
    """the eight members of the seeded batch (downscaled), stepped together:
    covered/uncovered counts every step and the final link lists bit-exact,
    force/torque within the FP32 bound"""
    from paper_1407_4524_amd import Batch
    ws = seeded_batch()
    steps = 300
    batch = Batch()
    members = [make_gpu(w) for w in ws]
    for d in members:
        batch.add(d)
    batch.step(steps)
    for w, d in zip(ws, members):
        o = make_oracle(w)
        o.step(steps)
        rg, ro = d.records(0), o.records(0)
        assert (rg[:, 18:20] == ro[:, 18:20]).all()
        n = same_links(d, o)
        check_series(rg, o, 0, "lattice", w["bodies"][0]["axes"][0], TOL_FT["f32"],
                     f"{w['name']} {w['nx']}x{w['ny']} {w['bodies'][0]['motion']} ({n} links)")
        o.close()
    batch.close()


# ---------------------------------------------------------------------------
# single domains


def test_large_region_advance_against_the_oracle():
    """a rotating 80x40 ellipse in a 420x300 channel: its region is too large
    for the single-workgroup list kernel, so the many-workgroup advance runs;
    counts every step and links bit-exact, force/torque within 1e-4"""
    w = copy.deepcopy(W.batched_domains(count=1, seed=0)[0])
    w.update(nx=420, ny=300)
    w["bodies"] = [dict(shape="ellipse", axes=(80.0, 40.0), bc="mls", me="lattice", motion="rotate",
                        c0=(150.0, 150.0, 0.0), theta0=0.2, omega=5e-4)]
    steps = 40
    g, o = run_pair(w, steps)
    rg, ro = g.records(0), o.records(0)
    assert (rg[:, 18:20] == ro[:, 18:20]).all() and ro[:, 18].sum() > 0
    n = same_links(g, o)
    check_series(rg, o, 0, "lattice", 80.0, TOL_FT["f32"], f"many-workgroup advance ({n} links)")
    check_series(rg, o, 0, "comoving", 80.0, TOL_FT["f32"], "  comoving form")


def test_couette_pair_against_the_oracle_and_the_closed_form():
    """rotating inner circle R1=10 inside a static outer circle R2=25 (solid
    outside), interpolated rule, FP64, from the analytic profile: both
    bodies' force/torque equal to the oracle's within 1e-10 over 400 steps;
    after 3000 steps the inner torque within 1% of -4 pi mu Omega R1^2 R2^2 /
    (R2^2 - R1^2) and the outer torque opposite (check e, on the GPU)"""
    R1, R2, tau = 10.0, 25.0, 0.8
    L = int(2 * R2 + 6)
    X = (L / 2 - 0.37, L / 2 + 0.21, 0.0)
    Om = 0.01 / R1
    w = box("D2Q9", L, L, tau=tau, bodies=[
        dict(shape="circle", axes=(R1,), bc="mls", me="static", motion="rotate", c0=X, omega=Om),
        dict(shape="outer_circle", axes=(R2,), bc="mls", me="static", motion="static", c0=X)])
    n = L * L
    idx = np.arange(n)
    x = idx % L - X[0]
    y = idx // L - X[1]
    r = np.maximum(np.hypot(x, y), 1e-9)
    A = -Om * R1 ** 2 / (R2 ** 2 - R1 ** 2)
    B = Om * R1 ** 2 * R2 ** 2 / (R2 ** 2 - R1 ** 2)
    ut = np.where(r < R2, A * r + B / r, 0.0)
    u = np.zeros((n, 3))
    u[:, 0] = -ut * y / r
    u[:, 1] = ut * x / r
    g, o = run_pair(w, 400, init_rho=np.ones(n), init_u=u)
    for b in (0, 1):
        same_links(g, o, b)
        check_series(g.records(b), o, b, "static", R1, TOL_FT["f64"], f"Couette body {b}")
    g.step(2600)
    nu = (tau - 0.5) / 3
    exact = -4 * math.pi * nu * Om * R1 ** 2 * R2 ** 2 / (R2 ** 2 - R1 ** 2)
    t_in = g.records(0, g.t - 1, 1)[0, 5]
    t_out = g.records(1, g.t - 1, 1)[0, 5]
    print(f"Couette torque: inner {t_in:.6e} outer {t_out:.6e} exact {exact:.6e} "
          f"(inner err {t_in / exact - 1:.2e}, bound 1e-2)", flush=True)
    assert abs(t_in / exact - 1) < 1e-2 and abs(-t_out / exact - 1) < 1e-2


def test_quasi_incompressible_equilibrium_with_a_body_fp32():
    """the channel cylinder with the He-Luo equilibrium and the interpolated
    rule in FP32 storage, 600 steps"""
    w = W.channel_cylinder_f64()
    w.update(eq="heluo", storage="f32")
    w["bodies"][0].update(bc="mls", c0=(25.3, 24.6, 0.0))
    g, o = run_pair(w, 600)
    same_links(g, o)
    check_series(g.records(0), o, 0, "static", 5.0, TOL_FT["f32"], "He-Luo FP32")
    du = velocity_error(g, o)
    print(f"  u err {du:.2e} (bound 5e-6)", flush=True)
    assert du < 5e-6


def test_halfway_bounce_back_on_a_moving_body():
    """the oscillating cylinder at 1/10 scale with halfway bounce-back, FP64,
    400 steps: counts every step bit-exact, lattice and comoving forms
    within 1e-10"""
    w = copy.deepcopy(W.channel_oscillating_f32(scale=10))
    w["storage"] = "f64"
    w["bodies"][0]["bc"] = "halfway"
    g, o = run_pair(w, 400)
    rg, ro = g.records(0), o.records(0)
    assert (rg[:, 18:20] == ro[:, 18:20]).all() and ro[:, 18].sum() > 0
    same_links(g, o)
    check_series(rg, o, 0, "lattice", 4.0, TOL_FT["f64"], "halfway moving, lattice")
    check_series(rg, o, 0, "comoving", 4.0, TOL_FT["f64"], "halfway moving, comoving")
    for t in (0, 57, 399):
        assert g.moving_sets(0, t) == (int(ro[t, 18]), int(ro[t, 19]))


def test_two_bodies_in_one_domain():
    """a static cylinder (halfway) and an oscillating ellipse (interpolated)
    in one FP64 channel, 300 steps: both link lists bit-exact, both bodies'
    force/torque within 1e-10, counts of the moving one every step"""
    w = W.channel_cylinder_f64()
    w.update(nx=120, ny=60, rho_noise=0.0)
    w["bodies"] = [dict(shape="circle", axes=(5.0,), bc="halfway", me="static", motion="static",
                        c0=(30.0, 30.0, 0.0)),
                   dict(shape="ellipse", axes=(6.0, 3.5), bc="mls", me="lattice", motion="oscillate",
                        c0=(72.3, 29.6, 0.0), theta0=0.5, amp=(0.0, 3.0, 0.0), period=150.0)]
    g, o = run_pair(w, 300)
    for b, mode, R in ((0, "static", 5.0), (1, "lattice", 6.0)):
        same_links(g, o, b)
        check_series(g.records(b), o, b, mode, R, TOL_FT["f64"], f"two bodies: body {b}")
    assert (g.records(1)[:, 18:20] == o.records(1)[:, 18:20]).all()


# ---------------------------------------------------------------------------
# faces, debug fill, instability


@pytest.mark.parametrize("case", ["channel_f64", "duct_f32"])
def test_face_records_against_the_oracle(case):
    """the momentum exchange of walls, inlet and outlet every step (the
    domain's face records) against the oracle's, 300 steps"""
    if case == "channel_f64":
        w, tol, steps = W.channel_cylinder_f64(), TOL_FT["f64"], 300
    else:
        w, tol, steps = W.duct_sphere(scale=4, storage="f32"), TOL_FT["f32"], 200
    g, o = run_pair(w, steps, face_records=True)
    fg, fo = g.face_records(), o.face_records()
    scale = np.abs(fo[:, 0:3]).max()
    tscale = np.abs(fo[:, 3:6]).max()
    for k, name in ((0, "walls"), (6, "inlet"), (12, "outlet")):
        eF = np.abs(fg[:, k:k + 3] - fo[:, k:k + 3]).max() / scale
        eT = np.abs(fg[:, k + 3:k + 6] - fo[:, k + 3:k + 6]).max() / tscale
        print(f"{case} {name}: F err {eF:.2e} T err {eT:.2e} (bound {tol:.0e})", flush=True)
        assert eF < tol and eT < tol
    assert np.array_equal(g.force_torque(-1), fg[:, 0:6])


def test_wall_force_balances_the_pressure_drop():
    """check (d) on the GPU: the empty 100x50 channel with velocity
    bounce-back at both ends, 12000 steps (near steady state): the x-force on
    the walls equals the pressure drop times the channel width, dp H with dp
    from the cross-section mean densities at the two ends (c_s^2 = 1/3) and
    H = ny - 2, within 2 % (the residual is the ends' own non-ideality); and
    the wall, inlet and outlet records of the last step equal the oracle's
    within 1e-10"""
    w = W.channel_cylinder_f64()
    w.update(bodies=[], rho_noise=0.0, faces=W.CHANNEL_VELOCITY_FACES)
    nx, ny = w["nx"], w["ny"]
    steps = 12000
    g = make_gpu(w, face_records=True, record_capacity=64)
    g.step(steps)
    f = g.face_records(g.t - 1, 1)[0]
    rho, _ = g.fields()
    r = rho.reshape(ny, nx)
    dp = (r[1:-1, 0].mean() - r[1:-1, nx - 1].mean()) / 3.0
    H = ny - 2
    print(f"wall force {f[0]:.6e} dp*H {dp * H:.6e} ratio {f[0] / (dp * H):.4f} (bound 2e-2)", flush=True)
    assert abs(f[0] / (dp * H) - 1) < 2e-2
    o = make_oracle(w)
    o.step(steps)
    fo = o.face_records(steps - 1, 1)[0]
    err = np.abs(f - fo).max() / np.abs(fo).max()
    print(f"face records at step {steps - 1} against the oracle: {err:.2e} (bound 1e-10)", flush=True)
    assert err < 1e-10


@pytest.mark.parametrize("case", ["channel_f64", "duct_f16", "oscillating_f32"])
def test_nan_filled_solid_slots_change_nothing(case):
    """with every non-fluid slot NaN at the start (and a static body's solid
    nodes NaN after placement), the run gives bitwise the same records and
    fluid fields as with zeros: no pull reads a slot that no rule wrote"""
    if case == "channel_f64":
        w, steps = W.channel_cylinder_f64(), 200
    elif case == "duct_f16":
        w, steps = W.duct_sphere(scale=4, storage="f16"), 150
    else:
        w, steps = W.channel_oscillating_f32(scale=10), 200
    a = make_gpu(w, debug_poison=True)
    b = make_gpu(w)
    a.step(steps)
    b.step(steps)
    ra, rb = a.records(0), b.records(0)
    assert np.isfinite(ra).all() and np.array_equal(ra, rb)
    fa, ua = a.fields()
    fb, ub = b.fields()
    assert np.array_equal(fa, fb, equal_nan=True) and np.array_equal(ua, ub, equal_nan=True)
    print(f"{case}: {steps} steps, records and fields identical with NaN-filled solid slots", flush=True)


def test_instability_is_flagged_on_the_device():
    """a fluid whose speed exceeds 0.4 somewhere (set from the host through
    the initial field) is reported as LBM_E_UNSTABLE at the next
    synchronisation; a stable run is not"""
    from paper_1407_4524_amd import LbmError
    w = box("D2Q9", 48, 40, tau=0.8, storage="f32")
    n = 48 * 40
    u = np.zeros((n, 3))
    for yy in range(10, 17):  # a 7x7 patch: its inner nodes keep their speed through the first steps
        u[yy * 48 + 20:yy * 48 + 27, 0] = 0.45
    g = make_gpu(w, init_u=u)
    g.step(3)
    with pytest.raises(LbmError) as e:
        g.synchronize()
    assert e.value.status == -5
    print("flagged:", e.value, flush=True)
    ok = make_gpu(w, init_u=u * 0.5)
    ok.step(3)
    ok.synchronize()
