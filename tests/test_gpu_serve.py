"""The serving loop on the GPU: a mixed stream (D2Q9 and D3Q19, FP32 and
FP16-shifted storage, static and rotating bodies) served with continuous
batching under a memory budget that forces queueing, against the same
requests served one at a time; each result must be the same bit for bit."""
import numpy as np
import pytest

import lbm_workloads as W

pytestmark = pytest.mark.gpu


def test_served_results_equal_requests_served_alone():
    from paper_1407_4524_amd import lbm
    from paper_1407_4524_amd.serve import GpuEngine, Server, serve_plain, summary
    reqs = W.serving_requests(count=8, seed=7, rate=500.0, max_steps=1500, scale=8, d3_fraction=0.4)
    kinds = {(r["spec"]["lattice"], r["spec"]["storage"]) for r in reqs}
    print("requests:", [(r["spec"]["name"], r["spec"]["bodies"][0]["motion"]) for r in reqs], flush=True)
    assert len(kinds) >= 3
    fps = [lbm.footprint_bytes(r["spec"], record_capacity=2048) for r in reqs]
    budget = sum(sorted(fps)[-3:])  # room for about three at once: requests queue
    eng = GpuEngine(record_capacity=2048)
    srv = Server(eng, budget, epoch=500, window=500, tol=1e-3)
    served = {r.id: r for r in srv.run(reqs)}
    eng.close()
    alone = {r.id: r for r in serve_plain(reqs, epoch=500, window=500, tol=1e-3)}
    assert sorted(served) == sorted(alone) == [r["id"] for r in reqs]
    assert srv.peak_memory <= budget and 1 < srv.peak_active < len(reqs)
    for k in served:
        a, b = served[k], alone[k]
        print(k, a.steps, a.converged, a.force_torque[:2], flush=True)
        assert a.steps == b.steps and a.converged == b.converged
        assert a.force_torque == b.force_torque
        assert np.isfinite(a.force_torque).all()
    s = summary(list(served.values()))
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
