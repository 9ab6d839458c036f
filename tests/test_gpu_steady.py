"""Steady-state check on the device (FP64, from the record rings) against
the same relative drag change taken from the oracle's records, and the
batched check against the single-domain one."""
import numpy as np
import pytest

import lbm_workloads as W
from gpu_helpers import make_gpu, ora_series
from oracle_helpers import make_oracle

pytestmark = pytest.mark.gpu


def test_steady_check_matches_oracle_records():
    w = W.channel_cylinder_f64()
    g = make_gpu(w)
    o = make_oracle(w)
    for steps in (1500, 3000):
        g.step(steps - g.t)
        o.step(steps - o.t)
        F, _ = ora_series(o, 0, "static")
        for window in (100, 500):
            ref = abs(F[steps - 1, 0] - F[steps - 1 - window, 0]) / abs(F[steps - 1, 0])
            for tol in (ref * 10, ref / 10):
                steady, rel = g.steady_state(window, tol)
                print(f"t={steps} window={window} oracle {ref:.6e} gpu {rel:.6e}", flush=True)
                assert abs(rel - ref) <= 1e-9
                assert steady == (ref < tol)
    with pytest.raises(Exception):
        g.steady_state(window=steps + 5)  # the ring does not reach back that far
    g.close()
    o.close()


def test_batched_check_equals_single_checks():
    from paper_1407_4524_amd import Batch
    ws = W.batched_domains(count=4, seed=11)
    doms = [make_gpu(w) for w in ws]
    batch = Batch()
    for d in doms:
        batch.add(d)
    st0, rel0 = batch.steady_state(500, 1e-3)
    assert (st0 == -1).all() and np.isnan(rel0).all()  # not enough steps yet
    batch.step(700)
    st, rel = batch.steady_state(500, 1e-3)
    for k, d in enumerate(doms):
        s1, r1 = d.steady_state(500, 1e-3)
        assert r1 == rel[k] and s1 == bool(st[k])
    batch.close()
