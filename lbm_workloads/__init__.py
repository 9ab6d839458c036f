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
ZOUHE_VELOCITY, ZOUHE_PRESSURE = 5, 6

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


def channel_zouhe(lattice: str = "D2Q9", storage: str = "f64", eq: str = "heluo", scale: int = 1, body: bool = True):
    """Channel (D2Q9 400x160, or D3Q19 duct 128x48x48) with the face method
    of the paper's Sec. IV set-up: Zou-He velocity inlet (parabolic, u_max
    0.04) and Zou-He pressure outlet (rho0), halfway walls, the
    quasi-incompressible equilibrium by default, tau 0.6, and a static
    circle/sphere (R 16, interpolated rule) a quarter of the way in.
    ``scale`` divides the sizes."""
    s = scale
    if lattice == "D2Q9":
        nx, ny, nz, r = 400 // s, 160 // s, 1, 16.0 / s
        faces, c0 = (ZOUHE_VELOCITY, ZOUHE_PRESSURE, WALL, WALL, PERIODIC, PERIODIC), (nx / 4, ny / 2 + 0.3, 0.0)
    else:
        nx, ny, nz, r = 128 // s, 48 // s, 48 // s, 8.0 / s
        faces, c0 = (ZOUHE_VELOCITY, ZOUHE_PRESSURE, WALL, WALL, WALL, WALL), (nx / 4, ny / 2 + 0.3, nz / 2 - 0.2)
    return dict(
        name=f"channel_zouhe_{lattice.lower()}_{eq}_{storage}_{nx}x{ny}" + (f"x{nz}" if nz > 1 else ""),
        lattice=lattice, nx=nx, ny=ny, nz=nz, tau=0.6, rho0=1.0, eq=eq, faces=faces, inlet_profile="parabolic",
        inlet_u=0.04, storage=storage, rho_noise=0.0, seed=0, steps=4000 // s,
        bodies=[dict(shape="circle", axes=(r,), bc="mls", me="static", motion="static", c0=c0)] if body else [])


def suspension(storage: str = "f32", nx: int = 2048, ny: int = 1024, rows: int = 4, cols: int = 8, seed: int = 0,
               radius=(12.0, 24.0), lattice: str = "D2Q9", nz: int = 1):
    """Many bodies in one channel (a fixed suspension): rows x cols cells,
    one body per cell at a seeded jittered position, radius (or semi-axes)
    drawn from `radius`. Cell k takes, by k % 4: a static circle (interpolated
    rule, static ME), a static circle with halfway bounce-back, an ellipse
    rotating in place at Omega in [2e-4, 1e-3] rad/step (lattice-frame ME),
    a circle oscillating across the channel with amplitude 2 and period
    U[300, 600] (lattice-frame ME). Parabolic inflow u_max = 0.04, tau = 0.6,
    zero-gradient outlet; every body stays at least 8 nodes from its cell's
    edges, so bodies keep far apart. D3Q19 gives spheres/ellipsoids in a
    duct (rows along y, cols along x, one layer in z)."""
    rng = np.random.default_rng(seed)
    cw, ch = nx / (cols + 1), ny / rows
    bodies = []
    for r in range(rows):
        for c in range(cols):
            k = r * cols + c
            a = float(rng.uniform(*radius))
            kind = k % 4
            b = float(rng.uniform(0.5 * a, a)) if kind == 2 else a
            slack = max(0.0, min(cw, ch) / 2 - a - 8.0 - (2.0 if kind == 3 else 0.0))
            cx = cw * (c + 0.5) + float(rng.uniform(-slack, slack))
            cy = ch * (r + 0.5) + float(rng.uniform(-slack, slack))
            cz = nz / 2 + float(rng.uniform(-0.5, 0.5)) if lattice == "D3Q19" else 0.0
            theta0 = float(rng.uniform(0.0, math.pi))
            if kind == 0:
                bd = dict(shape="circle", axes=(a,), bc="mls", me="static", motion="static", c0=(cx, cy, cz))
            elif kind == 1:
                bd = dict(shape="circle", axes=(a,), bc="halfway", me="static", motion="static", c0=(cx, cy, cz))
            elif kind == 2:
                bd = dict(shape="ellipse", axes=(a, b, b), bc="mls", me="lattice", motion="rotate", c0=(cx, cy, cz),
                          theta0=theta0, omega=float(rng.uniform(2e-4, 1e-3)))
            else:
                bd = dict(shape="circle", axes=(a,), bc="mls", me="lattice", motion="oscillate", c0=(cx, cy, cz),
                          amp=(0.0, 2.0, 0.0), period=float(rng.uniform(300.0, 600.0)))
            bodies.append(bd)
    faces = CHANNEL_FACES if lattice == "D2Q9" else DUCT_FACES
    name = f"suspension{len(bodies)}_{lattice.lower()}_{storage}_{nx}x{ny}" + (f"x{nz}" if lattice == "D3Q19" else "")
    return dict(name=name, lattice=lattice, nx=nx, ny=ny, nz=nz if lattice == "D3Q19" else 1, tau=0.6, rho0=1.0,
                eq="bgk", faces=faces, inlet_profile="parabolic", inlet_u=0.04, storage=storage, rho_noise=0.0,
                seed=seed, steps=2000, bodies=bodies)


def sedimenting(nx, ny, shape, axes, c0, ratio, g, storage="f64", tau=0.6, theta0=0.0, me="lattice",
                integrator="euler", refill="mean", eq="bgk", bc="mls"):
    """A free body released from rest in a closed vertical channel of fluid at
    rest (the set-up of the paper's Sec. IV sedimentation tests): halfway
    walls on every face, gravity g along -y; mass ratio*rho0*area (per unit
    depth), inertia of a uniform disc/ellipse, external force weight minus
    buoyancy, (ratio - 1) rho0 area g."""
    a = axes[0]
    b = axes[1] if shape == "ellipse" else a
    area = math.pi * a * b
    M = ratio * area
    inertia = M * (a * a + b * b) / 4.0
    return dict(name=f"sedimenting_{shape}_{storage}_{nx}x{ny}", lattice="D2Q9", nx=nx, ny=ny, nz=1, tau=tau, rho0=1.0,
                eq=eq, faces=CLOSED_FACES, inlet_profile="uniform", inlet_u=0.0, storage=storage, rho_noise=0.0,
                seed=0, steps=20000,
                bodies=[dict(shape=shape, axes=tuple(axes), bc=bc, me=me, motion="free", c0=tuple(c0), theta0=theta0,
                             mass=M, inertia=inertia, ext_force=(0.0, -(ratio - 1.0) * area * g, 0.0),
                             integrator=integrator, refill=refill)])


def _paper_units(width_m, nx, tau=0.6, nu=1e-6, gravity=9.81):
    """lattice spacing, time step and gravity of a channel of width_m metres
    resolved by nx nodes (walls half way out of the first and last), at the
    given tau and kinematic viscosity"""
    dx = width_m / (nx - 1)
    dt = ((tau - 0.5) / 3.0) * dx * dx / nu
    return dx, dt, gravity * dt * dt / dx


def sedimenting_disc(ratio=1.01, storage="f32", me="lattice", integrator="euler", refill="mean"):
    """The paper's sedimenting disc: d = 1e-3 m, W = 4d, H = 8W on 135 x 1073
    nodes (dx = W/134), tau = 0.6, water (nu = 1e-6 m^2/s), released from rest
    at x = 7.6e-4 m from the left wall (reading of the printed position),
    2.5e-2 m above the bottom; density ratio 1.01 or 1.03."""
    dx, dt, g = _paper_units(4e-3, 135)
    R = 0.5e-3 / dx
    w = sedimenting(135, 1073, "circle", (R,), (7.6e-4 / dx, 2.5e-2 / dx, 0.0), ratio, g, storage=storage, me=me,
                    integrator=integrator, refill=refill)
    w["name"] = f"sedimenting_disc_r{ratio}_{storage}_135x1073"
    w["dt_s"], w["dx_m"] = dt, dx
    return w


def sedimenting_ellipse(ratio=1.1, storage="f32", me="lattice", integrator="euler", refill="mean"):
    """The paper's sedimenting ellipse: major axis a = 1e-3 m, aspect ratio 2,
    W = 4a, H = 50a on 135 x 1676 nodes, tau = 0.6, water, released from rest
    at the channel centre 4.8e-2 m above the bottom at theta0 = pi/4, density
    ratio 1.1 (semi-axes a/2 and a/4)."""
    dx, dt, g = _paper_units(4e-3, 135)
    A = 0.5e-3 / dx
    w = sedimenting(135, 1676, "ellipse", (A, A / 2.0), (2e-3 / dx, 4.8e-2 / dx, 0.0), ratio, g, storage=storage,
                    theta0=math.pi / 4, me=me, integrator=integrator, refill=refill)
    w["name"] = f"sedimenting_ellipse_r{ratio}_{storage}_135x1676"
    w["dt_s"], w["dx_m"] = dt, dx
    return w


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
