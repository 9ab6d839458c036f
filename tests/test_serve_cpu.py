"""The serving scheduler on a simulated engine and clock (no GPU): admission
by memory budget and slots, arrival-order admission, continuous batching,
rejection of requests that can never fit, and results independent of the
mix."""
import pytest

from paper_1407_4524_amd.serve import Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeEngine:
    """A request converges once it has run spec['conv'] steps; an epoch of
    n steps costs dt seconds of simulated time whatever the mix."""

    def __init__(self, clock, dt=0.01):
        self.clock, self.dt = clock, dt
        self.active = {}
        self.used = 0
        self.peak_used = 0
        self.budget_seen = []
        self._n = 0

    def footprint(self, spec):
        return spec["fp"]

    def start(self, spec):
        h = self._n
        self._n += 1
        self.active[h] = [spec, 0]
        self.used += spec["fp"]
        self.peak_used = max(self.peak_used, self.used)
        return h

    def step(self, n):
        for v in self.active.values():
            v[1] += n
        self.clock.t += self.dt

    def poll(self, window, tol):
        out = {}
        for h, (spec, t) in self.active.items():
            ok = t - 1 - window >= 0
            out[h] = ((1 if t >= spec["conv"] else 0) if ok else -1, 0.0, t)
        return out

    def finish(self, h):
        spec, t = self.active.pop(h)
        self.used -= spec["fp"]
        return (float(spec["id"]), float(t), 0.0, 0.0, 0.0, 0.0)


def requests(n=20, seed=1):
    import numpy as np
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += float(rng.exponential(0.005))
        out.append(dict(id=k, arrival=t, max_steps=5000,
                        spec=dict(id=k, fp=int(rng.integers(1, 10)) * 100, conv=int(rng.integers(1, 8)) * 500)))
    return out


def serve(reqs, budget, max_active=256):
    clock = FakeClock()
    eng = FakeEngine(clock)
    srv = Server(eng, budget, max_active=max_active, epoch=500, window=500, clock=clock, sleep=clock.sleep)
    res = srv.run(reqs)
    return srv, eng, {r.id: r for r in res}


@pytest.mark.parametrize("budget,max_active", [(10 ** 9, 256), (1500, 256), (10 ** 9, 3), (900, 2)])
def test_every_request_completes_within_budget_and_slots(budget, max_active):
    reqs = requests()
    srv, eng, res = serve(reqs, budget, max_active)
    assert sorted(res) == [r["id"] for r in reqs]
    assert eng.peak_used <= budget and srv.peak_active <= max_active
    for r in reqs:
        x = res[r["id"]]
        # converged at the first epoch boundary with a full window at or after its convergence step
        want = max(r["spec"]["conv"], 1000)
        assert x.converged and x.steps == want
        assert x.admitted >= x.arrival and x.finished >= x.admitted


def test_admission_in_arrival_order():
    reqs = requests(30, seed=2)
    _, _, res = serve(reqs, 1200)
    adm = [res[r["id"]].admitted for r in sorted(reqs, key=lambda r: r["arrival"])]
    assert adm == sorted(adm)


def test_continuous_batching_admits_while_others_run():
    """with room for everything, a request that arrives while others are on
    the device starts at the next epoch boundary, not after they finish"""
    reqs = [dict(id=0, arrival=0.0, max_steps=5000, spec=dict(id=0, fp=1, conv=4000)),
            dict(id=1, arrival=0.015, max_steps=5000, spec=dict(id=1, fp=1, conv=1000))]
    _, _, res = serve(reqs, 10)
    assert res[1].admitted < res[0].finished
    assert res[1].finished < res[0].finished


def test_request_too_large_is_rejected_not_blocking():
    reqs = requests(6)
    reqs[2]["spec"]["fp"] = 10 ** 6
    srv, _, res = serve(reqs, 1000)
    assert srv.rejected == [2] and 2 not in res and len(res) == 5


def test_result_is_the_same_alone_and_in_the_mix():
    reqs = requests(12, seed=3)
    _, _, mix = serve(reqs, 10 ** 9)
    for r in reqs:
        _, _, alone = serve([dict(r, arrival=0.0)], 10 ** 9)
        assert alone[r["id"]].steps == mix[r["id"]].steps
        assert alone[r["id"]].force_torque == mix[r["id"]].force_torque


class FailingEngine(FakeEngine):
    """start refuses a spec marked 'refuse'; a spec with 'breaks' reports an
    error (flag -2) once it has run that many steps"""

    def start(self, spec):
        if spec.get("refuse"):
            raise RuntimeError("LBM_E_RANGE: body leaves the interior")
        return super().start(spec)

    def poll(self, window, tol):
        out = {}
        for h, (spec, t) in self.active.items():
            if spec.get("breaks") and t >= spec["breaks"]:
                out[h] = (-2, float("nan"), t, "LBM_E_UNSTABLE: speed out of range")
                continue
            ok = t - 1 - window >= 0
            out[h] = ((1 if t >= spec["conv"] else 0) if ok else -1, 0.0, t, "")
        return out

    def drop(self, h):
        spec, t = self.active.pop(h)
        self.used -= spec["fp"]


def test_failed_requests_finish_as_failed_and_release_memory():
    """a request the library refuses and one whose domain turns unstable end
    as failed results with the error's text; their memory goes back to the
    budget and every other request is served as usual"""
    reqs = requests(10, seed=4)
    reqs[1]["spec"]["refuse"] = True
    reqs[4]["spec"]["breaks"] = 1000
    clock = FakeClock()
    eng = FailingEngine(clock)
    budget = 2000
    srv = Server(eng, budget, epoch=500, window=500, clock=clock, sleep=clock.sleep)
    res = {r.id: r for r in srv.run(reqs)}
    assert sorted(res) == [r["id"] for r in reqs]
    assert res[1].failed and "LBM_E_RANGE" in res[1].error and res[1].steps == 0
    assert res[4].failed and "UNSTABLE" in res[4].error and res[4].steps == 1000
    for k, r in res.items():
        if k not in (1, 4):
            assert not r.failed and r.converged
    assert eng.used == 0 and not eng.active and eng.peak_used <= budget


def test_one_at_a_time_failures_do_not_stop_the_stream(monkeypatch):
    """the one-request-at-a-time reference also ends a refused request and one
    whose domain turns unstable as failed results, and serves the rest"""
    from paper_1407_4524_amd import lbm
    from paper_1407_4524_amd.serve import serve_plain

    class FakeDomain:
        closed = 0

        def __init__(self, spec):
            if spec.get("refuse"):
                raise lbm.LbmError(-4, "refused")
            self.spec, self.t = spec, 0

        @classmethod
        def from_spec(cls, spec, record_capacity=0):
            return cls(spec)

        def step(self, n):
            self.t += n
            if self.t >= self.spec.get("breaks", 1 << 30):
                raise lbm.LbmError(-5, "speed")

        def steady_state(self, window, tol):
            return self.t >= self.spec["conv"], 0.0

        def force_torque(self, body, t0, n):
            return [(float(self.spec["id"]),) + (0.0,) * 5]

        def close(self):
            FakeDomain.closed += 1

    monkeypatch.setattr(lbm, "Domain", FakeDomain)
    reqs = requests(8, seed=5)
    reqs[2]["spec"]["refuse"] = True
    reqs[5]["spec"]["breaks"] = 1000
    clock = FakeClock()
    res = {r.id: r for r in serve_plain(reqs, clock=clock, sleep=clock.sleep)}
    assert sorted(res) == list(range(8))
    assert res[2].failed and "LBM_E_RANGE" in res[2].error and res[2].steps == 0
    assert res[5].failed and "UNSTABLE" in res[5].error and res[5].steps == 1000
    for k, r in res.items():
        if k not in (2, 5):
            assert not r.failed and r.converged and r.force_torque[0] == float(k)
    assert FakeDomain.closed == 7
