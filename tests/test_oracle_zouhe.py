"""Pins of the oracle's Zou-He faces (the boundary method of the paper's
Sec. IV set-up for its faces), against what the method fixes independently of
how the oracle writes it:

* the defining property: after each step every fluid node of a velocity face
  carries exactly the prescribed velocity (the inlet profile along x, no
  transverse velocity) and every node of a pressure face exactly rho0 and no
  transverse velocity, with the node's moments summed here from the raw
  populations (standard and quasi-incompressible equilibria, D2Q9 and D3Q19,
  edge nodes next to the walls included);
* the closure of the normal population: its non-equilibrium part equals that
  of the opposite direction (Zou & He's bounce-back of the non-equilibrium
  part), with the equilibrium evaluated here from those moments;
* plane Poiseuille flow: driven by a parabolic velocity face against a
  pressure face between halfway walls, the steady flow reaches the parabola
  in the interior, keeps the mass flux constant along the channel, and its
  density gradient gives the viscous pressure drop 8 nu rho0 u_max / H^2
  (c_s^2 = 1/3).
"""
import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
from oracle_helpers import make_oracle

ZV, ZP = W.ZOUHE_VELOCITY, W.ZOUHE_PRESSURE


def _profile(y, ny, u):
    H = ny - 2.0
    return 4.0 * u * (y - 0.5) * (ny - 1.5 - y) / (H * H)


def _moments(f, c):
    rho = f.sum(axis=1)
    j = f @ c.astype(float)
    return rho, j


def _feq(rho, u, c, w, rho0, heluo):
    cu = u @ c.T.astype(float)
    uu = (u * u).sum(axis=1)[:, None]
    poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu
    if heluo:
        return w[None, :] * (rho[:, None] + rho0 * poly)
    return w[None, :] * rho[:, None] * (1.0 + poly)


def _face_nodes(d, x):
    t = d.types().reshape(d.nz, d.ny, d.nx)
    zz, yy = np.nonzero(t[:, :, x] == 0)
    return x + d.nx * (yy + d.ny * zz), yy, zz


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("eq", ["bgk", "heluo"])
def test_zouhe_faces_carry_prescribed_moments(lattice, eq):
    w = W.channel_zouhe(lattice, "f64", eq, scale=4 if lattice == "D2Q9" else 2, body=False)
    d = make_oracle(w)
    c, wt, opp = O.lattice(O.D2Q9 if lattice == "D2Q9" else O.D3Q19)
    heluo = eq == "heluo"
    rho0 = w["rho0"]
    for _ in range(3):
        d.step(7)
        f = d.populations()
        # velocity face at x = 0
        n, yy, zz = _face_nodes(d, 0)
        rho, j = _moments(f[n], c)
        rho_u = rho0 if heluo else rho
        ux = j[:, 0] / rho_u
        want = np.array([_profile(y, w["ny"], w["inlet_u"]) for y in yy])
        if lattice == "D3Q19":
            want = want * np.array([_profile(z, w["nz"], 1.0) for z in zz])
        assert np.max(np.abs(ux - want)) < 1e-14
        assert np.max(np.abs(j[:, 1:])) < 1e-14
        # normal population: bounce-back of its non-equilibrium part
        u = j / rho_u[:, None] if not heluo else j / rho0
        fe = _feq(rho, u, c, wt, rho0, heluo)
        i_n = int(np.nonzero((c[:, 0] == 1) & (c[:, 1] == 0) & (c[:, 2] == 0))[0][0])
        neq = f[n] - fe
        assert np.max(np.abs(neq[:, i_n] - neq[:, opp[i_n]])) < 1e-14
        # pressure face at x = nx - 1
        n, yy, zz = _face_nodes(d, w["nx"] - 1)
        rho, j = _moments(f[n], c)
        assert np.max(np.abs(rho - rho0)) < 1e-14
        assert np.max(np.abs(j[:, 1:])) < 1e-14
        i_m = int(opp[i_n])
        rho_u = rho0 if heluo else rho
        u = j / (rho_u[:, None] if not heluo else rho0)
        neq = f[n] - _feq(rho, u, c, wt, rho0, heluo)
        assert np.max(np.abs(neq[:, i_m] - neq[:, opp[i_m]])) < 1e-14
        assert np.all(np.isfinite(f[d.types() == 0]))


@pytest.mark.parametrize("eq", ["bgk", "heluo"])
def test_zouhe_poiseuille(eq):
    # tau = 1/2 + sqrt(3/16): halfway bounce-back places the no-slip planes
    # of a BGK Poiseuille flow exactly half way (He, Zou, Luo & Dembo 1997),
    # so the steady interior profile is the parabola the inlet prescribes
    nx, ny, umax = 48, 19, 0.02
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    w = dict(lattice="D2Q9", nx=nx, ny=ny, nz=1, tau=tau, rho0=1.0, eq=eq,
             faces=(ZV, ZP, W.WALL, W.WALL, W.PERIODIC, W.PERIODIC), inlet_profile="parabolic",
             inlet_u=umax, storage="f64", rho_noise=0.0, seed=0, bodies=[])
    d = make_oracle(w)
    d.step(16000)
    # the start from rest excites a slowly decaying mode that alternates in
    # sign every step (and between neighbouring columns): average two steps
    rho, u = d.fields()
    d.step(1)
    rho1, u1 = d.fields()
    rho, u = 0.5 * (rho + rho1), 0.5 * (u + u1)
    rho = rho.reshape(ny, nx)
    ux = u[:, 0].reshape(ny, nx)
    uy = u[:, 1].reshape(ny, nx)
    ys = np.arange(1, ny - 1)
    want = np.array([_profile(y, ny, umax) for y in ys])
    mid = ux[1:ny - 1, nx // 2]
    if eq == "heluo":
        assert np.max(np.abs(mid - want)) < 1e-4 * umax
    else:
        # the standard equilibrium is weakly compressible: rho u is what the
        # channel conserves, and the density falls along it, so only the
        # shape is the parabola's
        assert np.max(np.abs(mid / mid.sum() - want / want.sum())) < 1e-4 * np.max(want / want.sum())
    assert np.max(np.abs(uy[1:ny - 1, 2:nx - 2])) < 1e-4 * umax
    flux = ux[1:ny - 1, :].sum(axis=0) if eq == "heluo" else (rho * ux)[1:ny - 1, :].sum(axis=0)
    assert np.max(np.abs(flux - flux[nx // 2])) < (1e-6 if eq == "heluo" else 1e-4) * abs(flux[nx // 2])
    # pressure drop: d rho / dx = -3 * 8 nu rho0 u_max / H^2 with nu = (tau - 1/2) / 3
    nu = (tau - 0.5) / 3.0
    H = ny - 2.0
    grad = np.polyfit(np.arange(8, nx - 8), rho[ny // 2, 8:nx - 8], 1)[0]
    want_grad = -3.0 * 8.0 * nu * 1.0 * umax / (H * H)
    assert abs(grad - want_grad) < (0.01 if eq == "heluo" else 0.02) * abs(want_grad)


def test_zouhe_rejected_off_x():
    with pytest.raises(ValueError):
        O.OracleDomain(O.D2Q9, 20, 20, faces=(W.WALL, W.WALL, ZV, ZP, W.PERIODIC, W.PERIODIC))
