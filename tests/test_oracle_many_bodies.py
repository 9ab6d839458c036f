"""Pins of the oracle with many bodies in one domain.

* P3 for a suspension: in a periodic box holding five bodies (two static,
  three moving in different ways) the fluid's momentum changes every step by
  exactly minus the sum of the five lattice-frame forces of
  Eq. ForceInMovement; a body missed, counted twice or given another body's
  links breaks the budget.
* Locality: two bodies side by side in one box have, over the first steps,
  the records each has alone in its half.
"""
import numpy as np

import lbm_workloads as W
import oracle as O
from oracle_helpers import make_oracle, me_series


def _box(nx, ny, tau=0.7, faces=W.PERIODIC_FACES):
    return dict(name="box", lattice="D2Q9", nx=nx, ny=ny, nz=1, tau=tau, rho0=1.0, eq="bgk", faces=faces,
                inlet_profile="uniform", inlet_u=0.0, storage="f64", rho_noise=0.0, seed=0, bodies=[])


def _momentum(d):
    c, _, _ = O.lattice(d.lattice)
    f = d.populations()
    return (f[d.types() == 0] @ c.astype(float)).sum(axis=0)


def test_momentum_budget_five_bodies():
    w = _box(96, 64)
    steps = 50
    w["bodies"] = [
        dict(shape="circle", axes=(4.2,), bc="mls", motion="static", c0=(16.3, 15.2, 0.0)),
        dict(shape="circle", axes=(3.7,), bc="halfway", motion="static", c0=(70.1, 47.6, 0.0)),
        dict(shape="ellipse", axes=(5.5, 2.8), bc="mls", motion="rotate", c0=(45.2, 16.7, 0.0), theta0=0.4,
             omega=0.03),
        dict(shape="circle", axes=(4.3,), bc="halfway", motion="oscillate", c0=(20.4, 46.1, 0.0),
             amp=(2.5, 1.5, 0.0), period=40.0),
        dict(shape="ellipse", axes=(4.6, 3.1), bc="mls", motion="table", c0=(72.5, 17.3, 0.0),
             table=W.pose_table(steps + 2, (72.5, 17.3, 0.0), theta0=0.2, vel=(0.06, 0.03, 0), omega=-0.02)),
    ]
    rho, u = W.random_state(w, rho_amp=0.005, u_amp=0.02, seed=9)
    d = make_oracle(w, init_rho=rho, init_u=u)
    scale = d.populations()[d.types() == 0].sum()
    P = [_momentum(d)]
    for _ in range(steps):
        d.step(1)
        P.append(_momentum(d))
    dP = np.diff(np.array(P), axis=0)
    F = sum(me_series(d.records(k), "lattice")[0] for k in range(5))
    assert np.abs(dP + F).max() < 1e-14 * scale
    moved = [d.records(k)[:, 18].sum() + d.records(k)[:, 19].sum() for k in range(5)]
    assert moved[0] == 0 and moved[1] == 0 and min(moved[2:]) > 0
    # every body has links, and each link's fluid node is fluid
    t = d.types()
    for k in range(5):
        node, _, _ = d.links(k)
        assert len(node) > 0 and (t[node] == 0).all()


def test_bodies_in_separated_halves_match_alone():
    """Locality: a signal moves at most one node per step, so over the first
    steps a body's records depend only on the nodes near it. Two bodies, each
    alone in a 40x40 wall-bounded box, and the same two placed side by side
    in one 80x40 box with the same initial fields, have the same records
    (bit for bit for the body that keeps its coordinates) while no signal
    from the joined middle can have reached either body: body ids, links and
    sums stay apart."""
    nx, ny, steps = 80, 40, 8
    walls = (W.WALL,) * 4 + (W.PERIODIC,) * 2
    a = dict(shape="ellipse", axes=(5.0, 3.0), bc="mls", motion="rotate", c0=(19.6, 20.3, 0.0), theta0=0.1,
             omega=0.02)
    b = dict(shape="circle", axes=(4.0,), bc="mls", motion="oscillate", c0=(20.2, 19.7, 0.0), amp=(0.0, 2.0, 0.0),
             period=50.0)
    half = _box(nx // 2, ny, faces=walls)
    ra, ua = W.random_state(half, rho_amp=0.003, u_amp=0.01, seed=11)
    rb, ub = W.random_state(half, rho_amp=0.003, u_amp=0.01, seed=12)
    da = make_oracle(dict(half, bodies=[a]), init_rho=ra, init_u=ua)
    db = make_oracle(dict(half, bodies=[b]), init_rho=rb, init_u=ub)
    rho = np.concatenate([ra.reshape(ny, nx // 2), rb.reshape(ny, nx // 2)], axis=1).reshape(-1)
    u = np.concatenate([ua.reshape(ny, nx // 2, 3), ub.reshape(ny, nx // 2, 3)], axis=1).reshape(-1, 3)
    bb = dict(b, c0=(b["c0"][0] + nx // 2, b["c0"][1], 0.0))
    dfull = make_oracle(dict(_box(nx, ny, faces=walls), bodies=[a, bb]), init_rho=rho, init_u=u)
    # both bodies (and the two-node reach of their rules) stay more than
    # `steps` nodes from the columns 39 and 40 where the boxes differ
    da.step(steps)
    db.step(steps)
    dfull.step(steps)
    assert np.array_equal(da.records(0), dfull.records(0))
    # body b sits 40 nodes further along x, where x - X and so Delta and the
    # torque arms round differently: equal counts, sums equal to rounding
    r1, r2 = db.records(0), dfull.records(1)
    assert np.array_equal(r1[:, 18:20], r2[:, 18:20])
    assert np.abs(r1 - r2).max() < 1e-13 * np.abs(r1).max()
    assert da.records(0)[:, 18:20].sum() + db.records(0)[:, 18:20].sum() > 0
