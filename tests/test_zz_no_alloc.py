"""lbm_batch_steady_state_noalloc (the entry point for callers that cannot
allocate device memory) against lbm_batch_steady_state on the same batch,
through the C ABI: bitwise the same flags and relative changes, on two calls
in a row, the second with fewer members; beyond its maximum it refuses."""
import copy

import numpy as np
import pytest

import lbm_workloads as W
from gpu_helpers import make_gpu

pytestmark = pytest.mark.gpu


def small_members(count, seed=3, side=120):
    out = []
    for w in W.batched_domains(count=count, seed=seed):
        w = copy.deepcopy(w)
        s = max(w["nx"], w["ny"]) / side
        if s > 1:
            w["nx"], w["ny"] = int(w["nx"] / s), int(w["ny"] / s)
            b = w["bodies"][0]
            b["axes"] = tuple(max(4.0, a / s) for a in b["axes"])
            b["c0"] = (max(b["c0"][0] / s, b["axes"][0] + 4), min(max(b["c0"][1] / s, b["axes"][0] + 4),
                                                                   w["ny"] - b["axes"][0] - 5), 0.0)
        out.append(w)
    return out


def both(batch, window, tol):
    st_a, rel_a = batch.steady_state(window, tol)
    st_b, rel_b = batch.steady_state(window, tol, noalloc=True)
    return st_a, rel_a, st_b, rel_b


def test_noalloc_steady_state_equals_the_allocating_one():
    from paper_1407_4524_amd import Batch
    ws = small_members(6)
    print("no-alloc steady state: members", [(w["nx"], w["ny"]) for w in ws], flush=True)
    batch = Batch()
    members = [make_gpu(w, record_capacity=512) for w in ws]
    for d in members:
        batch.add(d)
    batch.step(160)
    late = make_gpu(ws[0], record_capacity=512)  # too few steps for the window: -1 / NaN
    batch.add(late)
    st_a, rel_a, st_b, rel_b = both(batch, 100, 1e-2)
    print("first call:", st_a, rel_a, flush=True)
    assert np.array_equal(st_a, st_b) and np.array_equal(rel_a, rel_b, equal_nan=True)
    assert st_a[-1] == -1 and np.isnan(rel_a[-1]) and (st_a[:-1] >= 0).all()
    assert np.isfinite(rel_a[:-1]).all() and (rel_a[:-1] > 0).any()
    # second call, smaller input: three members fewer, more steps
    for d in members[:3]:
        batch.remove(d)
    batch.step(40)
    st_a, rel_a, st_b, rel_b = both(batch, 150, 1e-3)
    print("second call:", st_a, rel_a, flush=True)
    assert len(st_a) == 4
    assert np.array_equal(st_a, st_b) and np.array_equal(rel_a, rel_b, equal_nan=True)
    assert st_a[-1] == -1 and (st_a[:-1] >= 0).all()
    batch.close()
    for d in members + [late]:
        d.close()


def test_noalloc_steady_state_refuses_more_members_than_its_table():
    from paper_1407_4524_amd import Batch, LbmError, lbm
    n = 513  # LBM_STEADY_NOALLOC_MAX + 1
    w = dict(name="tiny", lattice="D2Q9", nx=3, ny=3, nz=1, tau=0.8, rho0=1.0, eq="bgk", faces=W.PERIODIC_FACES,
             inlet_profile="uniform", inlet_u=0.0, storage="f64", rho_noise=0.0, seed=0, bodies=[])
    print(f"no-alloc steady state: {n} tiny members", flush=True)
    batch = Batch()
    doms = [make_gpu(w, record_capacity=16) for _ in range(n)]
    for d in doms:
        batch.add(d)
    with pytest.raises(LbmError) as e:
        batch.steady_state(10, 1e-3, noalloc=True)
    assert e.value.status == -1 and str(lbm.MAX_STEADY_NOALLOC) in str(e.value)
    st, rel = batch.steady_state(10, 1e-3)  # the allocating one takes any size
    assert (st == -1).all()
    batch.close()
    for d in doms:
        d.close()
