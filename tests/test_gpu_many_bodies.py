"""Many bodies in one domain (a fixed suspension) on the GPU, through the C
ABI, against the CPU oracle: every body's link list and covered/uncovered
counts bit-exact, every body's force/torque series within the storage's bar
(FP64 1e-10, FP32 1e-4; drag-scaled per body), the velocity field within
1e-12 / 5e-6. Bodies are placed, stepped and recorded independently: the
record ring holds one record per body slot (max_bodies) and step.

The bodies keep far apart (at least 8 nodes; the library requires more than
the two-node reach of the interpolated rule and the refill's one-node
neighbourhood, see include/lbm.h), so the order in which their advances run
does not matter and the oracle's simultaneous update is the reference.
"""
import numpy as np
import pytest

import lbm_workloads as W
from gpu_helpers import make_gpu, run_pair, series_error, velocity_error
from oracle_helpers import make_oracle, me_series

pytestmark = pytest.mark.gpu


def _mode(b):
    return {"static": "static", "lattice": "lattice", "comoving": "comoving"}[b["me"]]


def _check_bodies(g, o, w, tol):
    worst = 0.0
    for k, b in enumerate(w["bodies"]):
        ng, dg, lg = g.links(k)
        no, do, lo = o.links(k)
        assert len(ng) == len(no) and (ng == no).all() and (dg == do).all(), f"body {k} links"
        assert (lg == lo).all(), f"body {k} delta"
        rg, ro = g.records(k), o.records(k)
        assert (rg[:, 18:20] == ro[:, 18:20]).all(), f"body {k} covered/uncovered counts"
        F, T = me_series(ro, _mode(b))
        G = me_series(rg, _mode(b))
        eF, eT = series_error(np.hstack(G), F, T, b["axes"][0])
        worst = max(worst, eF, eT)
        assert eF < tol and eT < tol, (k, b["motion"], eF, eT)
    return worst


@pytest.mark.parametrize("storage,tol,tol_u", [("f64", 1e-10, 1e-12), ("f32", 1e-4, 5e-6)])
def test_suspension8_d2q9(storage, tol, tol_u):
    """8 bodies (static MLS and halfway circles, rotating ellipses,
    oscillating circles) in a 320x160 channel, 400 steps."""
    w = W.suspension(storage, nx=320, ny=160, rows=2, cols=4, radius=(5.0, 9.0))
    print(f"{w['name']}, 400 steps", flush=True)
    g, o = run_pair(w, 400)
    worst = _check_bodies(g, o, w, tol)
    du = velocity_error(g, o)
    print(f"worst body F/T error {worst:.2e}, u {du:.2e}")
    assert du < tol_u


def test_suspension64_slots_f32():
    """All 64 body slots: 64 bodies (16 of them rotating, 16 oscillating) in a
    640x320 channel, FP32, 200 steps."""
    w = W.suspension("f32", nx=640, ny=320, rows=8, cols=8, radius=(4.0, 8.0), seed=3)
    assert len(w["bodies"]) == 64
    print(f"{w['name']}, 200 steps", flush=True)
    g, o = run_pair(w, 200)
    worst = _check_bodies(g, o, w, 1e-4)
    du = velocity_error(g, o)
    print(f"worst body F/T error {worst:.2e}, u {du:.2e}")
    assert du < 5e-6


def test_suspension_d3q19_f32():
    """6 spheres/ellipsoids (static, rotating, oscillating) in a 96x64x32
    duct, FP32, 200 steps."""
    w = W.suspension("f32", nx=96, ny=64, rows=2, cols=3, radius=(4.0, 6.0), lattice="D3Q19", nz=32)
    print(f"{w['name']}, 200 steps", flush=True)
    g, o = run_pair(w, 200)
    worst = _check_bodies(g, o, w, 1e-4)
    du = velocity_error(g, o)
    print(f"worst body F/T error {worst:.2e}, u {du:.2e}")
    assert du < 5e-6


def test_suspension_batch_equals_alone():
    """The 8-body channel stepped as a one-member batch (every body's advance
    in one launch) equals the same domain stepped alone, bit for bit."""
    from paper_1407_4524_amd import Batch
    w = W.suspension("f32", nx=320, ny=160, rows=2, cols=4, radius=(5.0, 9.0))
    alone = make_gpu(w)
    alone.step(300)
    a = make_gpu(w)
    b = Batch()
    b.add(a)
    b.step(300)
    a.synchronize()
    for k in range(len(w["bodies"])):
        assert np.array_equal(a.records(k), alone.records(k)), k
    assert np.array_equal(a.fields()[1], alone.fields()[1], equal_nan=True)
    b.close()


def test_body_slots_validated():
    from paper_1407_4524_amd import Domain, LbmError
    w = W.channel_cylinder_f64()
    with pytest.raises(LbmError):
        make_gpu(w, max_bodies=65)
    d = make_gpu(w, max_bodies=2)
    with pytest.raises(LbmError):
        d.set_body(2, shape="circle", axes=(3.0,), c0=(60.0, 25.0, 0.0))
    d.set_body(1, shape="circle", axes=(3.0,), c0=(60.0, 25.0, 0.0))
    d.step(10)
    assert d.records(1).shape == (10, 20)
    assert isinstance(d, Domain)
