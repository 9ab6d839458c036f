"""Steady-flow pins of the CPU oracle against closed forms.

* Poiseuille: the parabolic profile between two resting walls, and the wall
  force equal to the pressure drop times the channel height (global momentum
  balance).
* Circular Couette: torque on a rotating inner cylinder inside a resting outer
  one, T = -4 pi mu Omega R1^2 R2^2 / (R2^2 - R1^2) per unit length; the
  outer cylinder takes the opposite torque. This exercises the interpolated
  boundary rule, its moving-wall term and the ME torque of
  Eq. flow_torque_2; the interpolated rule converges at second order as both
  radii double, halfway bounce-back at first order.

The Poiseuille case uses velocity bounce-back at both ends: with a
zero-gradient outlet the velocity inlet sets no pressure level and the mass
drifts (the flux then falls linearly along the channel), so no steady
parabola exists to compare with.
"""
import math

import numpy as np
import pytest

import lbm_workloads as W
from oracle_helpers import make_oracle


def poiseuille_channel(eq, tau):
    w = W.channel_cylinder_f64()
    w.update(bodies=[], eq=eq, tau=tau, rho_noise=0.0, faces=W.CHANNEL_VELOCITY_FACES)
    return w


@pytest.mark.parametrize("eq,tau,tol", [("heluo", 0.5 + math.sqrt(3) / 4, 2e-3), ("bgk", 0.8, 2e-2)])
def test_poiseuille_profile_and_wall_force(eq, tau, tol):
    """P4/P5: at steady state u_x(y) at mid-channel matches
    4 u_max (y-1/2)(ny-3/2-y)/H^2 (no-slip planes half way to the wall
    layers, H = ny-2) within ``tol`` of u_max (at tau = 1/2 + sqrt(3)/4 halfway
    bounce-back puts the wall exactly mid-link), and the x-force on the walls
    equals (p_in - p_out) H with p = rho/3 within 2%."""
    w = poiseuille_channel(eq, tau)
    d = make_oracle(w)
    d.step(12000)
    nx, ny = w["nx"], w["ny"]
    rho, u = d.fields()
    y = np.arange(ny)
    H = ny - 2
    exact = 4 * w["inlet_u"] * (y - 0.5) * (ny - 1.5 - y) / H ** 2
    ux = u[:, 0].reshape(ny, nx)[:, nx // 2]
    assert np.abs(ux[1:-1] - exact[1:-1]).max() <= tol * w["inlet_u"]
    r = rho.reshape(ny, nx)
    dp = (r[1:-1, 0].mean() - r[1:-1, nx - 1].mean()) / 3.0
    Fw = d.face_records(d.t - 1, 1)[0, 0]
    assert abs(Fw / (dp * H) - 1) < 0.02


def couette_torque(R1, R2, bc, steps, tau=0.8):
    """Run the rotating-inner-cylinder problem from the analytic profile and
    return (inner torque, outer torque, exact inner torque)."""
    L = int(2 * R2 + 6)
    X = (L / 2 - 0.37, L / 2 + 0.21, 0.0)
    Om = 0.01 / R1
    w = dict(name="couette", lattice="D2Q9", nx=L, ny=L, nz=1, tau=tau, rho0=1.0, eq="bgk",
             faces=W.PERIODIC_FACES, inlet_profile="uniform", inlet_u=0.0, storage="f64",
             rho_noise=0.0, seed=0,
             bodies=[dict(shape="circle", axes=(R1,), bc=bc, motion="rotate", c0=X, omega=Om),
                     dict(shape="outer_circle", axes=(R2,), bc=bc, motion="static", c0=X)])
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
    d = make_oracle(w, init_rho=np.ones(n), init_u=u)
    d.step(steps)
    nu = (tau - 0.5) / 3
    exact = -4 * math.pi * nu * Om * R1 ** 2 * R2 ** 2 / (R2 ** 2 - R1 ** 2)
    return d.records(0, d.t - 1, 1)[0, 5], d.records(1, d.t - 1, 1)[0, 5], exact


def test_couette_torque_interpolated_second_order():
    """P6 with the interpolated (Mei-Luo-Shyy) rule: inner torque within 0.1%
    at R1=20, R2=50; outer torque opposite; error shrinks by >= 3 when both
    radii double. A wrong sign of the moving-wall term flips the torque."""
    t_in, t_out, exact = couette_torque(20, 50, "mls", 3000)
    e1 = t_in / exact - 1
    assert exact < 0 and abs(e1) < 1e-3
    assert abs(-t_out / exact - 1) < 1e-3
    t_in2, _, exact2 = couette_torque(40, 100, "mls", 3000)
    e2 = t_in2 / exact2 - 1
    assert abs(e1 / e2) >= 3


def test_couette_torque_halfway_first_order():
    """P6 with halfway bounce-back (stair-step wall): within 2%, and the error
    of the stair-step body does not vanish like the interpolated rule's."""
    t_in, t_out, exact = couette_torque(20, 50, "halfway", 3000)
    e = t_in / exact - 1
    assert abs(e) < 0.02 and abs(e) > 2e-3
