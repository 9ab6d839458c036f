"""Batches of domains (lbm_batch_*): the batched launches against each
member advanced alone by lbm_step, and against the CPU oracle.

Bars: bitwise equality of records and fields with the member stepped alone
(the batched kernels do every node's and every link's arithmetic in the
same order); FP32 storage against the FP64 oracle within 1e-4 (force and
torque series, drag-scaled), as for a single domain.
"""
import copy

import numpy as np
import pytest

import lbm_workloads as W
from gpu_helpers import make_gpu, ora_series, series_error
from oracle_helpers import make_oracle

pytestmark = pytest.mark.gpu


def small_batch(count=8, seed=3, max_side=200):
    """Seeded uneven channel domains like the 64-domain workload, with the
    sides capped so that the tests stay short."""
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


def assert_same(a, b):
    assert a.t == b.t
    assert np.array_equal(a.records(0), b.records(0))
    ra, ua = a.fields()
    rb, ub = b.fields()
    assert np.array_equal(ra, rb, equal_nan=True) and np.array_equal(ua, ub, equal_nan=True)


@pytest.mark.parametrize("overlap,own_stream,graph,order", [(1, True, 0, 0), (1, False, 0, 0), (0, False, 0, 0),
                                                            (0, True, 1, 0), (1, True, 1, 0), (0, True, 0, 3),
                                                            (1, True, 1, 3)])
def test_batch_equals_each_domain_alone(overlap, own_stream, graph, order):
    """overlap on a stream of the batch's own uses the CU-masked second
    stream, on the default stream a plain one; graph mode replays a captured
    32-step sequence in the 100-step call (3 replays and 4 ordinary steps);
    order 3 sweeps spans of consecutive nodes across rows"""
    import torch
    from paper_1407_4524_amd import Batch
    ws = small_batch()
    kinds = {(w["bodies"][0]["shape"], w["bodies"][0]["motion"]) for w in ws}
    assert ("ellipse", "rotate") in kinds and any(m == "static" for _, m in kinds)
    print("batch of", [(w["nx"], w["ny"], w["bodies"][0]["shape"], w["bodies"][0]["motion"]) for w in ws],
          f"overlap {overlap} own stream {own_stream}", flush=True)
    alone = [make_gpu(w) for w in ws]
    for d in alone:
        d.step(150)
    s = torch.cuda.Stream() if own_stream else torch.cuda.current_stream()
    batch = Batch(stream=s.cuda_stream)
    batch.config = dict(batch.config, overlap=overlap, graph=graph, order=order, cells_per_thread=1)
    with torch.cuda.stream(s):
        members = [make_gpu(w) for w in ws]
    for d in members:
        batch.add(d)
    for n in (1, 49, 100):  # several calls: the tables are rebuilt at each
        batch.step(n)
    for a, b in zip(members, alone):
        assert_same(a, b)
    batch.close()


def test_batch_large_moving_body():
    """a rotating ellipse whose region exceeds the single-workgroup list
    kernel is advanced by the many-workgroup kernels inside the batched step"""
    from paper_1407_4524_amd import Batch
    w = copy.deepcopy(W.batched_domains(count=1, seed=0)[0])
    w.update(nx=420, ny=300)
    w["bodies"] = [dict(shape="ellipse", axes=(80.0, 40.0), bc="mls", me="lattice", motion="rotate",
                        c0=(150.0, 150.0, 0.0), theta0=0.2, omega=5e-4)]
    small = small_batch(count=2)
    alone = [make_gpu(x) for x in [w] + small]
    for d in alone:
        d.step(40)
    batch = Batch()
    members = [make_gpu(x) for x in [w] + small]
    for d in members:
        batch.add(d)
    batch.step(40)
    for a, b in zip(members, alone):
        assert_same(a, b)
    batch.close()


@pytest.mark.parametrize("graph", [0, 1])
def test_batch_3d_many_links(graph):
    """D3Q19 FP32 members: a static sphere of radius 18 (more than 16384
    links, so its link rule spans more than 256 wavefronts), a rotating
    ellipsoid (many-workgroup advance) and a small translating sphere (list
    kernel), batched in calls of 70 and 30 steps, against each alone"""
    from paper_1407_4524_amd import Batch
    base = dict(lattice="D3Q19", tau=0.7, rho0=1.0, eq="bgk", faces=W.DUCT_FACES, inlet_profile="uniform",
                inlet_u=0.02, storage="f32", rho_noise=0.0, seed=0)
    ws = [dict(base, name="sphere18", nx=96, ny=48, nz=48,
               bodies=[dict(shape="circle", axes=(18.0,), bc="mls", me="static", motion="static",
                            c0=(40.3, 24.1, 23.8))]),
          dict(base, name="ellipsoid", nx=48, ny=40, nz=40,
               bodies=[dict(shape="ellipse", axes=(9.0, 6.0, 5.0), bc="mls", me="lattice", motion="rotate",
                            c0=(20.3, 19.8, 20.1), theta0=0.3, omega=0.01)]),
          dict(base, name="small_sphere", nx=40, ny=32, nz=32,
               bodies=[dict(shape="circle", axes=(3.0,), bc="mls", me="lattice", motion="const_vel",
                            c0=(12.2, 15.7, 16.1), vel=(0.02, 0.0, 0.0))])]
    alone = [make_gpu(w) for w in ws]
    for d in alone:
        d.step(100)
    assert len(alone[0].links(0)[0]) > 16384
    batch = Batch()
    batch.config = dict(batch.config, graph=graph, order=3 if graph else 0, block=64, cells_per_thread=1)
    members = [make_gpu(w) for w in ws]
    for d in members:
        batch.add(d)
    for n in (70, 30):
        batch.step(n)
    for a, b in zip(members, alone):
        assert_same(a, b)
    batch.close()


def test_batch_members_at_different_steps_and_tuning():
    from paper_1407_4524_amd import Batch
    ws = small_batch(count=4, seed=5)
    alone = [make_gpu(w) for w in ws]
    members = [make_gpu(w) for w in ws]
    for k, (a, m) in enumerate(zip(alone, members)):  # members start at steps 0, 7, 14, 21
        a.step(7 * k)
        m.step(7 * k)
    batch = Batch()
    for d in members:
        batch.add(d)
    chosen, trials = batch.tune(trial_steps=3)
    # 72 shapes of 3 steps (60 with row tiles, 12 with spans across rows), then
    # the best shape in ordinary and graph mode over 64 steps each
    assert len(trials) == 75 and chosen["us_per_step"] == min(t["us_per_step"] for t in trials[72:])
    assert {t["graph"] for t in trials[72:]} == {0, 1}
    assert sum(t["order"] == 3 for t in trials[:72]) == 12
    batch.step(20)
    for a in alone:
        a.step(72 * 3 + 3 * 64 + 20)
    for a, m in zip(alone, members):
        assert_same(m, a)
    # a member can still be stepped on its own while it belongs to the batch
    members[0].step(5)
    alone[0].step(5)
    assert_same(members[0], alone[0])
    batch.remove(members[1])
    batch.step(3)
    for a in (alone[0], alone[2], alone[3]):
        a.step(3)
    for a, m in zip(alone, members):
        assert_same(m, a)
    batch.close()


def test_batch_against_oracle():
    from paper_1407_4524_amd import Batch
    ws = small_batch(count=8, seed=3, max_side=120)[:3]
    steps = 300
    batch = Batch()
    members = [make_gpu(w) for w in ws]
    for d in members:
        batch.add(d)
    batch.step(steps)
    for w, d in zip(ws, members):
        o = make_oracle(w)
        o.step(steps)
        F, T = ora_series(o, 0, "lattice")
        ft = d.force_torque(0, 0, steps)
        eF, eT = series_error(ft, F, T, w["bodies"][0]["axes"][0])
        print(f"{w['name']} {w['nx']}x{w['ny']} {w['bodies'][0]['motion']}: eF {eF:.2e} eT {eT:.2e}", flush=True)
        assert eF < 1e-4 and eT < 1e-4
        o.close()
    batch.close()


def test_batch_rejects_a_different_storage():
    from paper_1407_4524_amd import Batch, LbmError
    ws = small_batch(count=2)
    w64 = copy.deepcopy(ws[1])
    w64["storage"] = "f64"
    batch = Batch()
    a = make_gpu(ws[0])
    b = make_gpu(w64)
    batch.add(a)
    with pytest.raises(LbmError):
        batch.add(b)
    with pytest.raises(LbmError):
        batch.add(a)
    batch.close()
