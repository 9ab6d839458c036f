"""The many-workgroup advance (moving bodies whose region or near-surface
list does not fit the single-workgroup list kernel: the rows of the region
cut into slabs of 16, a workgroup per slab, two launches per step) on the GPU
through the C ABI, against the CPU oracle on the same inputs: the link list
of the last pose and every step's covered/uncovered counts bit-exact, the
force/torque series within the storage's bar (FP64 1e-10, FP32 1e-4 of the
drag scale), the velocity field within 1e-12 / 5e-6. The same bodies stepped
alone and in a batch give the same bits, also for a body that changes
kernels during the run.
"""
import copy

import numpy as np
import pytest

import lbm_workloads as W
from gpu_helpers import make_gpu, ora_series, run_pair, series_error, velocity_error

pytestmark = pytest.mark.gpu


def _oscillating(storage, refill="mean", me="lattice", bc="mls"):
    """a cylinder of radius 75.5 (a region of about 160 x 160 nodes, beyond the
    list kernel's 20480) oscillating across a 400 x 240 channel"""
    return dict(name=f"wide_cylinder_{storage}", lattice="D2Q9", nx=400, ny=240, nz=1, tau=0.7, rho0=1.0, eq="bgk",
                faces=W.CHANNEL_FACES, inlet_profile="parabolic", inlet_u=0.04, storage=storage, rho_noise=0.0,
                seed=0, bodies=[dict(shape="circle", axes=(75.5,), bc=bc, me=me, motion="oscillate",
                                     c0=(130.3, 120.2, 0.0), amp=(0.0, 6.0, 0.0), period=600.0, refill=refill)])


def _ellipsoid(storage):
    """an ellipsoid (9, 6, 5) rotating about z at 0.01 rad/step in a 48 x 40 x 40
    duct (its near-surface list, about 4000 nodes, is beyond the list
    kernel's 2048)"""
    return dict(name=f"wide_ellipsoid_{storage}", lattice="D3Q19", nx=48, ny=40, nz=40, tau=0.7, rho0=1.0,
                eq="bgk", faces=W.DUCT_FACES, inlet_profile="uniform", inlet_u=0.02, storage=storage, rho_noise=0.0,
                seed=0, bodies=[dict(shape="ellipse", axes=(9.0, 6.0, 5.0), bc="mls", me="lattice", motion="rotate",
                                     c0=(20.3, 19.8, 20.1), theta0=0.3, omega=0.01)])


def _check(g, o, w, tol, tol_u):
    ng, dg, lg = g.links(0)
    no, do, lo = o.links(0)
    assert len(ng) == len(no) and np.array_equal(ng, no) and np.array_equal(dg, do), "links"
    assert np.abs(lg - lo).max() == 0.0, "delta"
    rg, ro = g.records(0), o.records(0)
    assert np.array_equal(rg[:, 18:20], ro[:, 18:20]), "covered/uncovered counts"
    assert ro[:, 18].sum() > 0 and ro[:, 19].sum() > 0
    R = w["bodies"][0]["axes"][0]
    worst = 0.0
    for mode, G in (("lattice", rg[:, 0:6] + rg[:, 6:12]), ("comoving", rg[:, 12:18])):
        F, T = ora_series(o, 0, mode)
        eF, eT = series_error(G, F, T, R)
        print(f"{mode}: F {eF:.2e} T {eT:.2e}")
        worst = max(worst, eF, eT)
    du = velocity_error(g, o)
    print(f"u {du:.2e}")
    assert worst < tol and du < tol_u


@pytest.mark.parametrize("storage,tol,tol_u", [("f64", 1e-10, 1e-12), ("f32", 1e-4, 5e-6)])
@pytest.mark.parametrize("refill", ["mean", "extrapolate"])
def test_oscillating_cylinder(storage, tol, tol_u, refill):
    w = _oscillating(storage, refill)
    print(f"{w['name']}, {refill} refill, 600 steps", flush=True)
    g, o = run_pair(w, 600)
    _check(g, o, w, tol, tol_u)


def test_oscillating_cylinder_halfway_aidun_f32():
    w = _oscillating("f32", "aidun", me="comoving", bc="halfway")
    print(f"{w['name']}, halfway, aidun refill, 600 steps", flush=True)
    g, o = run_pair(w, 600)
    _check(g, o, w, 1e-4, 5e-6)


@pytest.mark.parametrize("storage,tol,tol_u", [("f64", 1e-10, 1e-12), ("f32", 1e-4, 5e-6)])
def test_rotating_ellipsoid(storage, tol, tol_u):
    w = _ellipsoid(storage)
    print(f"{w['name']}, 150 steps", flush=True)
    g, o = run_pair(w, 150)
    _check(g, o, w, tol, tol_u)


def test_alone_equals_batch():
    """the cylinder and the ellipsoid, each alone and each as a batch member
    beside a domain with a small moving body (advanced by the list kernel in
    the same batch step), bit for bit"""
    from paper_1407_4524_amd import Batch
    small = W.channel_oscillating_f32(scale=10)  # R = 4: the single-workgroup kernel
    small.update(nx=400, ny=240)
    for w, steps in ((_oscillating("f32"), 300), (_ellipsoid("f32"), 100)):
        print(f"{w['name']} alone and in a batch, {steps} steps", flush=True)
        alone = make_gpu(w)
        alone.step(steps)
        alone.synchronize()
        a = make_gpu(w)
        s = make_gpu(small) if w["lattice"] == "D2Q9" else None
        b = Batch()
        b.add(a)
        if s is not None:
            b.add(s)
        b.step(steps)
        a.synchronize()
        assert np.array_equal(a.records(0), alone.records(0))
        assert np.array_equal(a.links(0)[0], alone.links(0)[0])
        assert np.array_equal(a.fields()[1], alone.fields()[1], equal_nan=True)
        b.close()


def test_many_slabs_large_ellipse_f32():
    """a 150 x 30 ellipse rotating at 5e-4 rad/step (tip speed 0.075; its
    region spans up to 308 rows: 20 slabs) in a 420 x 330 box, 60 steps"""
    w = copy.deepcopy(_oscillating("f32"))
    w.update(name="wide_long_ellipse_f32", nx=420, ny=330, faces=W.PERIODIC_FACES, inlet_u=0.0)
    w["bodies"] = [dict(shape="ellipse", axes=(150.0, 30.0), bc="mls", me="lattice", motion="rotate",
                        c0=(210.2, 165.1, 0.0), theta0=1.1, omega=5e-4)]
    print(f"{w['name']}, 60 steps", flush=True)
    g, o = run_pair(w, 60)
    ng, dg, _ = g.links(0)
    no, do, _ = o.links(0)
    assert np.array_equal(ng, no) and np.array_equal(dg, do)
    rg, ro = g.records(0), o.records(0)
    assert np.array_equal(rg[:, 18:20], ro[:, 18:20]) and ro[:, 19].sum() > 0
    F, T = ora_series(o, 0, "lattice")
    eF, eT = series_error(rg[:, 0:6] + rg[:, 6:12], F, T, 150.0,
                          scale=max(np.abs(F).max(), np.abs(T).max() / 150.0))
    print(f"lattice: F {eF:.2e} T {eT:.2e}")
    assert eF < 1e-4 and eT < 1e-4


def _switching():
    """a 100 x 40 ellipse rotating at 1e-3 rad/step from 0.25 rad: its region
    grows from about 19300 to 22700 nodes during 200 steps, so its advance
    moves from the list kernel to the many-workgroup kernels"""
    w = copy.deepcopy(_oscillating("f32"))
    w.update(name="switching_ellipse_f32", nx=300, ny=260, faces=W.PERIODIC_FACES, inlet_u=0.0)
    w["bodies"] = [dict(shape="ellipse", axes=(100.0, 40.0), bc="mls", me="lattice", motion="rotate",
                        c0=(150.2, 130.1, 0.0), theta0=0.25, omega=1e-3)]
    return w


def test_kernel_switch_against_oracle_and_batch():
    from paper_1407_4524_amd import Batch
    w = _switching()
    print(f"{w['name']}, 200 steps", flush=True)
    g, o = run_pair(w, 200)
    ng, dg, _ = g.links(0)
    no, do, _ = o.links(0)
    assert np.array_equal(ng, no) and np.array_equal(dg, do)
    rg, ro = g.records(0), o.records(0)
    assert np.array_equal(rg[:, 18:20], ro[:, 18:20]) and ro[:, 19].sum() > 0
    F, T = ora_series(o, 0, "lattice")
    eF, eT = series_error(rg[:, 0:6] + rg[:, 6:12], F, T, 100.0,
                          scale=max(np.abs(F).max(), np.abs(T).max() / 100.0))
    print(f"lattice: F {eF:.2e} T {eT:.2e}")
    assert eF < 1e-4 and eT < 1e-4
    # the same run in a batch, in calls of uneven length
    a = make_gpu(w)
    b = Batch()
    b.add(a)
    for n in (37, 90, 73):
        b.step(n)
    a.synchronize()
    assert np.array_equal(a.records(0), rg)
    assert np.array_equal(a.fields()[1], g.fields()[1], equal_nan=True)
    b.close()


def test_flat_ellipsoid_many_links_per_slab_f32():
    """a flat ellipsoid (48, 46, 3) rotating about z at 1e-3 rad/step in a
    120 x 112 x 24 duct (73 thousand links): the slabs of rows just above and
    below its flat faces hold up to about 5000 links, more than a workgroup
    keeps in LDS (4096), so the rest go through global memory; links, counts
    and force against the oracle"""
    w = dict(name="flat_ellipsoid_f32", lattice="D3Q19", nx=120, ny=112, nz=24, tau=0.7, rho0=1.0, eq="bgk",
             faces=W.DUCT_FACES, inlet_profile="uniform", inlet_u=0.01, storage="f32", rho_noise=0.0, seed=0,
             bodies=[dict(shape="ellipse", axes=(48.0, 46.0, 3.0), bc="mls", me="lattice", motion="rotate",
                          c0=(60.2, 56.1, 11.8), theta0=0.4, omega=1e-3)])
    print(f"{w['name']}, 30 steps", flush=True)
    g, o = run_pair(w, 30)
    ng, dg, lg = g.links(0)
    no, do, lo = o.links(0)
    print(f"{len(no)} links")
    assert len(no) > 60000
    assert np.array_equal(ng, no) and np.array_equal(dg, do) and np.abs(lg - lo).max() == 0.0
    rg, ro = g.records(0), o.records(0)
    assert np.array_equal(rg[:, 18:20], ro[:, 18:20]) and ro[:, 19].sum() > 0
    F, T = ora_series(o, 0, "lattice")
    eF, eT = series_error(rg[:, 0:6] + rg[:, 6:12], F, T, 48.0,
                          scale=max(np.abs(F).max(), np.abs(T).max() / 48.0))
    print(f"lattice: F {eF:.2e} T {eT:.2e}")
    assert eF < 1e-4 and eT < 1e-4
