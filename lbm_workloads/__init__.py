"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds workload descriptions (plain dictionaries of sizes,
parameters and body placements) and seeded random generators. It contains
none of the lattice-Boltzmann or momentum-exchange arithmetic: both the GPU
library and the CPU oracle receive these values as inputs.

Workloads (lattice units; see the channel and duct set-ups of the paper's
Sec. IV for the shape of the problems these stand in for):

* ``channel_cylinder_f64``: D2Q9, 100x50 channel, walls on the rows y=0 and
  y=49, parabolic inlet u_max=0.05, zero-gradient outlet, tau=0.8, static
  cylinder R=5 at (25,25) with halfway bounce-back, density noise 1e-6.
* ``channel_oscillating_f32``: D2Q9 FP32 channel 2000x800, tau=0.55,
  u_max=0.04, cylinder R=40 at (400,400) with interpolated bounce-back,
  oscillating y(t)=400+20 sin(2 pi t/4000), covered/uncovered-node ME.
  ``scale=10`` gives the 200x80 case (R=4, amplitude 2, period 400) the
  oracle runs in seconds.
* ``duct_sphere``: D3Q19 duct 256x128x128, tau=0.6, plug inlet u=0.03,
  sphere R=16 at (64,64,64), interpolated bounce-back; ``scale=4`` gives
  64x32x32.
"""
from __future__ import annotations

import copy
import math

import numpy as np

PERIODIC, WALL, INLET, OUTLET, OUTLET_VELOCITY = 0, 1, 2, 3, 4

CHANNEL_FACES = (INLET, OUTLET, WALL, WALL, PERIODIC, PERIODIC)
DUCT_FACES = (INLET, OUTLET, WALL, WALL, WALL, WALL)
PERIODIC_FACES = (PERIODIC,) * 6
CLOSED_FACES = (WALL,) * 6
CHANNEL_VELOCITY_FACES = (INLET, OUTLET_VELOCITY, WALL, WALL, PERIODIC, PERIODIC)


def channel_cylinder_f64():
    return dict(
        name="channel_cylinder_f64_100x50", lattice="D2Q9", nx=100, ny=50, nz=1, tau=0.8,
        rho0=1.0, eq="bgk", faces=CHANNEL_FACES, inlet_profile="parabolic", inlet_u=0.05,
        storage="f64", rho_noise=1e-6, seed=0, steps=2000,
        bodies=[dict(shape="circle", axes=(5.0,), bc="halfway", me="static", motion="static",
                     c0=(25.0, 25.0, 0.0))])


def channel_oscillating_f32(scale: int = 1):
    s = scale
    nx, ny = 2000 // s, 800 // s
    return dict(
        name=f"channel_oscillating_f32_{nx}x{ny}", lattice="D2Q9", nx=nx, ny=ny, nz=1, tau=0.55,
        rho0=1.0, eq="bgk", faces=CHANNEL_FACES, inlet_profile="parabolic", inlet_u=0.04,
        storage="f32", rho_noise=0.0, seed=0, steps=20000 // s,
        bodies=[dict(shape="circle", axes=(40.0 / s,), bc="mls", me="lattice", motion="oscillate",
                     c0=(400.0 / s, 400.0 / s, 0.0), amp=(0.0, 20.0 / s, 0.0),
                     period=4000.0 / s)])


def duct_sphere(scale: int = 1, storage: str = "f32"):
    s = scale
    nx, ny, nz = 256 // s, 128 // s, 128 // s
    return dict(
        name=f"duct_sphere_{storage}_{nx}x{ny}x{nz}", lattice="D3Q19", nx=nx, ny=ny, nz=nz,
        tau=0.6, rho0=1.0, eq="bgk", faces=DUCT_FACES, inlet_profile="uniform", inlet_u=0.03,
        storage=storage, rho_noise=0.0, seed=0, steps=10000 // s,
        bodies=[dict(shape="circle", axes=(16.0 / s,), bc="mls", me="static", motion="static",
                     c0=(64.0 / s, 64.0 / s, 64.0 / s))])


def channel_large(storage: str = "f32", n: int = 8192):
    """D2Q9 channel n x n (8192 x 8192: 4.8 GB of FP32 populations, well past
    the 256 MB last-level cache), static cylinder R=40 at (n/5, n/2) with the
    interpolated rule and static momentum exchange; a footprint point for the
    stream-collide kernel beyond 1 GB."""
    return dict(
        name=f"channel_large_{storage}_{n}x{n}", lattice="D2Q9", nx=n, ny=n, nz=1, tau=0.6, rho0=1.0, eq="bgk",
        faces=CHANNEL_FACES, inlet_profile="parabolic", inlet_u=0.04, storage=storage, rho_noise=0.0, seed=0,
        steps=200,
        bodies=[dict(shape="circle", axes=(40.0,), bc="mls", me="static", motion="static",
                     c0=(n / 5.0, n / 2.0 + 0.3, 0.0))])


def with_changes(w, **kw):
    w = copy.deepcopy(w)
    w.update(kw)
    return w


# ---------------------------------------------------------------------------
# seeded generators


def density_noise(w):
    """rho0 * (1 + eps * U[-1,1)) per node, x fastest, numpy default_rng(seed)."""
    n = w["nx"] * w["ny"] * w["nz"]
    eps = w.get("rho_noise", 0.0)
    if not eps:
        return None
    rng = np.random.default_rng(w.get("seed", 0))
    return w["rho0"] * (1.0 + eps * rng.uniform(-1.0, 1.0, n))


def random_state(w, rho_amp=0.01, u_amp=0.05, seed=None):
    """Random density and velocity fields (periodic-box tests)."""
    rng = np.random.default_rng(w.get("seed", 0) if seed is None else seed)
    n = w["nx"] * w["ny"] * w["nz"]
    rho = w["rho0"] * (1.0 + rho_amp * rng.uniform(-1.0, 1.0, n))
    u = u_amp * rng.uniform(-1.0, 1.0, (n, 3))
    if w["lattice"] == "D2Q9":
        u[:, 2] = 0.0
    return rho, u


def pose_table(steps, c0, theta0=0.0, vel=(0, 0, 0), omega=0.0, amp=(0, 0, 0), period=None):
    """Per-step pose rows (X[3], theta, V[3], Omega_z) of a prescribed motion:
    translation at constant velocity plus a sinusoidal displacement plus a
    constant rotation. The test inputs of moving-body cases."""
    rows = np.zeros((steps, 8))
    for t in range(steps):
        ph = 0.0 if period is None else (2.0 * math.pi) * t / period
        for a in range(3):
            rows[t, a] = c0[a] + vel[a] * t + (amp[a] * math.sin(ph) if period else 0.0)
            rows[t, 4 + a] = vel[a] + (amp[a] * (2.0 * math.pi / period) * math.cos(ph) if period else 0.0)
        rows[t, 3] = theta0 + omega * t
        rows[t, 7] = omega
    return rows


def batched_domains(count=64, seed=0):
    """Seeded draw of uneven D2Q9 channel domains with one circle or ellipse each
    (sizes 64..512, semi-axes 4..nx/8 in the first third, half of them rotating
    at Omega in [0, 1e-3] rad/step, tau in [0.52, 1.0])."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nx = int(rng.integers(64, 513))
        ny = int(rng.integers(64, 513))
        while True:
            ellipse = bool(rng.integers(0, 2))
            a = float(rng.uniform(4.0, max(4.0, nx / 8)))
            b = float(rng.uniform(4.0, a)) if ellipse else a
            cx = float(rng.uniform(0.0, nx / 3))
            cy = float(rng.uniform(0.0, ny))
            if cx - a - 3 > 0 and cy - a - 3 > 1 and cy + a + 3 < ny - 2 and cx + a + 3 < nx - 1:
                break
        theta0 = float(rng.uniform(0.0, math.pi))
        rotating = k % 2 == 1
        omega = float(rng.uniform(0.0, 1e-3)) if rotating else 0.0
        tau = float(rng.uniform(0.52, 1.0))
        out.append(dict(
            name=f"batch{k}", lattice="D2Q9", nx=nx, ny=ny, nz=1, tau=tau, rho0=1.0, eq="bgk",
            faces=CHANNEL_FACES, inlet_profile="parabolic", inlet_u=0.04, storage="f32",
            rho_noise=0.0, seed=seed, steps=5000,
            bodies=[dict(shape="ellipse" if ellipse else "circle", axes=(a, b), bc="mls",
                         me="lattice", motion="rotate" if rotating else "static",
                         c0=(cx, cy, 0.0), theta0=theta0, omega=omega)]))
    return out


def serving_requests(count=256, seed=0, rate=200.0, max_steps=50000, scale=1, d3_fraction=0.2):
    """Seeded stream of drag/torque solve requests: Poisson arrivals at `rate`
    per second; 80 % D2Q9 channels with sides U{128..1024}, 20 % D3Q19 ducts
    with sides U{48..160} (sides divided by `scale`); one circle/sphere or
    ellipse/ellipsoid each, static or rotating at Omega in [0, 1e-3]
    rad/step; storage FP32 or FP16-shifted at 50/50; Re ~ U[10, 100] on the
    body diameter with parabolic inflow u_max = 0.04, tau = 1/2 + 3 u_max D /
    Re, at least 0.52. Each request runs until its drag changes by less than
    the tolerance over the steady window, or to max_steps."""
    rng = np.random.default_rng(seed)
    u_max = 0.04
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        is3d = bool(rng.random() < d3_fraction)
        storage = "f16" if rng.random() < 0.5 else "f32"
        re = float(rng.uniform(10.0, 100.0))
        ellipse = bool(rng.integers(0, 2))
        rotating = bool(rng.integers(0, 2))
        omega = float(rng.uniform(0.0, 1e-3)) if rotating else 0.0
        theta0 = float(rng.uniform(0.0, math.pi))
        if not is3d:
            nx = max(64, int(rng.integers(128, 1025)) // scale)
            ny = max(32, int(rng.integers(128, 1025)) // scale)
            a = float(rng.uniform(4.0, max(4.0, min(nx, ny) / 8)))
            b = float(rng.uniform(4.0, a)) if ellipse else a
            cx = float(rng.uniform(a + 4, max(a + 4.5, nx / 3)))
            cy = float(rng.uniform(a + 5, ny - a - 6))
            w = dict(name=f"req{k}_d2q9_{storage}_{nx}x{ny}", lattice="D2Q9", nx=nx, ny=ny, nz=1,
                     faces=CHANNEL_FACES, c0=(cx, cy, 0.0), axes=(a, b))
        else:
            nx, ny, nz = (max(32, int(rng.integers(48, 161)) // scale) for _ in range(3))
            a = float(rng.uniform(4.0, max(4.0, min(nx, ny, nz) / 6)))
            b = float(rng.uniform(4.0, a)) if ellipse else a
            c = float(rng.uniform(4.0, a)) if ellipse else a
            cx = float(rng.uniform(a + 4, max(a + 4.5, nx / 3)))
            cy = float(rng.uniform(a + 5, ny - a - 6))
            cz = float(rng.uniform(a + 5, nz - a - 6))
            w = dict(name=f"req{k}_d3q19_{storage}_{nx}x{ny}x{nz}", lattice="D3Q19", nx=nx, ny=ny, nz=nz,
                     faces=DUCT_FACES, c0=(cx, cy, cz), axes=(a, b, c))
        tau = max(0.52, 0.5 + 3.0 * u_max * 2.0 * a / re)
        body = dict(shape="ellipse" if ellipse else "circle", axes=w.pop("axes") if ellipse else (a,), bc="mls",
                    me="lattice", motion="rotate" if rotating else "static", c0=w.pop("c0"), theta0=theta0,
                    omega=omega)
        w.pop("axes", None)
        w.pop("c0", None)
        w.update(tau=tau, rho0=1.0, eq="bgk", inlet_profile="parabolic", inlet_u=u_max, storage=storage,
                 rho_noise=0.0, seed=seed, bodies=[body], reynolds=re)
        out.append(dict(id=k, arrival=t, spec=w, max_steps=max_steps))
    return out
