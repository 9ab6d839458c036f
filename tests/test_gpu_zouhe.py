"""Zou-He velocity/pressure faces (the face method of the paper's Sec. IV
set-up) and the quasi-incompressible equilibrium on the GPU, through the C
ABI, against the CPU oracle on the same inputs: a static body in a channel
driven through a Zou-He velocity face against a Zou-He pressure face.

Bars as for the other faces: FP64 storage force/torque within 1e-10 and
velocity within 1e-12; FP32 within 1e-4 / 5e-6; FP16-shifted force/torque
within 1e-3, velocity as derived in its test (the face rule adds a handful
of operations per face node). The face nodes themselves
carry the prescribed moments on the GPU too (within the storage's rounding).
"""
import numpy as np
import pytest

import lbm_workloads as W
from gpu_helpers import make_gpu, ora_series, run_pair, series_error, velocity_error
from oracle_helpers import make_oracle

pytestmark = pytest.mark.gpu


def _profile(y, ny, u):
    H = ny - 2.0
    return 4.0 * u * (y - 0.5) * (ny - 1.5 - y) / (H * H)


@pytest.mark.parametrize("eq", ["bgk", "heluo"])
def test_zouhe_channel_f64(eq):
    """D2Q9 100x40 channel, circle R=4 (interpolated rule), FP64, 800 steps."""
    w = W.channel_zouhe("D2Q9", "f64", eq, scale=4)
    print(f"{w['name']}, 800 steps", flush=True)
    g, o = run_pair(w, 800)
    F, T = ora_series(o, 0, "static")
    eF, eT = series_error(g.force_torque(0), F, T, 4.0)
    du = velocity_error(g, o)
    print(f"F {eF:.2e} T {eT:.2e} u {du:.2e}")
    assert eF < 1e-10 and eT < 1e-10 and du < 1e-12
    # the inlet face nodes carry the profile, no transverse velocity
    rho, u = g.fields()
    ny, nx = w["ny"], w["nx"]
    ux = u[:, 0].reshape(ny, nx)
    uy = u[:, 1].reshape(ny, nx)
    ys = np.arange(1, ny - 1)
    want = np.array([_profile(y, ny, w["inlet_u"]) for y in ys])
    assert np.abs(ux[1:ny - 1, 0] - want).max() < 1e-14
    assert np.abs(uy[1:ny - 1, 0]).max() < 1e-14 and np.abs(uy[1:ny - 1, nx - 1]).max() < 1e-14
    assert np.abs(rho.reshape(ny, nx)[1:ny - 1, nx - 1] - 1.0).max() < 1e-14


@pytest.mark.parametrize("storage,tol_ft,tol_u", [("f32", 1e-4, 5e-6), ("f16", 1e-3, 1.5e-3)])
def test_zouhe_channel_heluo_reduced_precision(storage, tol_ft, tol_u):
    """The quasi-incompressible equilibrium with a body and FP32 / FP16-shifted
    storage: D2Q9 200x80 channel, circle R=8, 1000 steps against the FP64
    oracle. FP16 velocity bound: each stored deviation (|h| <= 0.015 here)
    is rounded to a half-ulp of 2^-11 relative, <= 7.3e-6 per value and
    step; as a random walk of 9 values over 1000 weakly damped steps
    (tau = 0.6) that is of order 9 * 7.3e-6 * sqrt(1000) = 2e-3 (measured
    5.9e-4)."""
    w = W.channel_zouhe("D2Q9", storage, "heluo", scale=2)
    print(f"{w['name']}, 1000 steps", flush=True)
    g, o = run_pair(w, 1000)
    F, T = ora_series(o, 0, "static")
    eF, eT = series_error(g.force_torque(0), F, T, 8.0)
    du = velocity_error(g, o)
    print(f"{storage}: F {eF:.2e} T {eT:.2e} u {du:.2e}")
    assert eF < tol_ft and eT < tol_ft and du < tol_u


@pytest.mark.parametrize("eq", ["bgk", "heluo"])
def test_zouhe_duct_d3q19_f32(eq):
    """D3Q19 64x24x24 duct, Zou-He faces on x with halfway walls on the four
    other faces (the face nodes on the edges included), sphere R=4, FP32,
    400 steps."""
    w = W.channel_zouhe("D3Q19", "f32", eq, scale=2)
    print(f"{w['name']}, 400 steps", flush=True)
    g, o = run_pair(w, 400)
    F, T = ora_series(o, 0, "static")
    eF, eT = series_error(g.force_torque(0), F, T, 4.0)
    du = velocity_error(g, o)
    print(f"F {eF:.2e} T {eT:.2e} u {du:.2e}")
    assert eF < 1e-4 and eT < 1e-4 and du < 5e-6


def test_zouhe_channel_full_size_f32():
    """The full 400x160 channel with the circle of radius 16, FP32,
    quasi-incompressible, 1500 steps against the oracle at full size."""
    w = W.channel_zouhe("D2Q9", "f32", "heluo")
    print(f"{w['name']}, 1500 steps", flush=True)
    g, o = run_pair(w, 1500)
    F, T = ora_series(o, 0, "static")
    eF, eT = series_error(g.force_torque(0), F, T, 16.0)
    du = velocity_error(g, o)
    print(f"F {eF:.2e} T {eT:.2e} u {du:.2e}")
    assert eF < 1e-4 and eT < 1e-4 and du < 5e-6


def test_zouhe_batch_member_equals_alone():
    """A Zou-He channel stepped in a batch beside an ordinary channel equals
    the same domain stepped alone, bit for bit."""
    from paper_1407_4524_amd import Batch
    wz = W.channel_zouhe("D2Q9", "f32", "heluo", scale=4)
    wc = W.with_changes(W.channel_oscillating_f32(scale=10), eq="heluo")
    alone = make_gpu(wz)
    alone.step(300)
    a, c = make_gpu(wz), make_gpu(wc)
    b = Batch()
    b.add(a)
    b.add(c)
    b.step(300)
    a.synchronize()
    assert np.array_equal(a.force_torque(0), alone.force_torque(0))
    assert np.array_equal(a.fields()[1], alone.fields()[1], equal_nan=True)
    b.close()


def test_zouhe_rejected_off_x_and_with_face_records():
    from paper_1407_4524_amd import LbmError
    w = W.channel_zouhe("D2Q9", "f64", "heluo", scale=4, body=False)
    with pytest.raises(LbmError):
        make_gpu(dict(w, faces=(W.WALL, W.WALL, W.ZOUHE_VELOCITY, W.ZOUHE_PRESSURE, W.PERIODIC, W.PERIODIC)))
    with pytest.raises(LbmError):
        make_gpu(w, face_records=True)
