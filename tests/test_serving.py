"""Scheduler logic of the continuous-batching server (CPU, fake backends)."""
import numpy as np
import pytest

import oracle
from paper_2304_06437_amd.serving import JobSpec, Server, ServeReport, JobResult, poisson_mix


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-3)


class CountingBackend:
    """No physics: counts concurrency, advances a simulated clock by the work."""

    def __init__(self, clock, bytes_per_node=100, fail_create=(), fail_read=(), ns_per_lu=1.0):
        self.clock = clock
        self.bpn = bytes_per_node
        self.fail_create = set(fail_create)
        self.fail_read = set(fail_read)
        self.ns = ns_per_lu
        self.live = 0
        self.max_live = 0
        self.admit_order = []

    def required_bytes(self, spec):
        return spec.nodes * self.bpn

    def create(self, spec):
        if spec.job_id in self.fail_create:
            raise RuntimeError("create failed")
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        self.admit_order.append(spec.job_id)
        return spec

    def step(self, handles, nsteps):
        self.clock.t += sum(h.nodes * k for h, k in zip(handles, nsteps)) * self.ns * 1e-9

    def read(self, h, spec):
        if spec.job_id in self.fail_read:
            raise FloatingPointError("non-finite state")
        return {}

    def destroy(self, h):
        self.live -= 1


def _specs(n, nodes_edge=32, steps=100, gap=0.0):
    return [JobSpec(job_id=i, lattice=19, shape=(nodes_edge,) * 3, steps=steps, arrival=i * gap)
            for i in range(n)]


def test_admission_respects_hbm_budget():
    clk = FakeClock()
    be = CountingBackend(clk)
    specs = _specs(6)
    need = specs[0].nodes * 100
    rep = Server(be, hbm_budget=int(2.5 * need), chunk_steps=30, clock=clk, sleep=clk.sleep).run(specs)
    assert be.max_live == 2 and rep.max_active == 2
    assert all(r.status == "done" for r in rep.results)
    assert rep.peak_bytes <= 2.5 * need
    assert be.live == 0


def test_admission_is_in_arrival_order():
    clk = FakeClock()
    be = CountingBackend(clk)
    specs = _specs(8, gap=1e-4)[::-1]  # submitted out of order
    Server(be, hbm_budget=10 ** 12, chunk_steps=50, clock=clk, sleep=clk.sleep).run(specs)
    assert be.admit_order == list(range(8))


def test_oversized_and_invalid_requests_rejected():
    clk = FakeClock()
    be = CountingBackend(clk)
    specs = _specs(3)
    specs.append(JobSpec(job_id=3, lattice=19, shape=(200, 200, 200), steps=10))
    rep = Server(be, hbm_budget=specs[0].nodes * 100 * 3, clock=clk, sleep=clk.sleep).run(specs)
    st = {r.job_id: r.status for r in rep.results}
    assert st == {0: "done", 1: "done", 2: "done", 3: "rejected"}


def test_failures_are_isolated():
    clk = FakeClock()
    be = CountingBackend(clk, fail_create={1}, fail_read={3})
    rep = Server(be, hbm_budget=10 ** 12, chunk_steps=40, clock=clk, sleep=clk.sleep).run(_specs(5))
    st = [r.status for r in rep.results]
    assert st == ["done", "failed", "done", "failed", "done"]
    assert be.live == 0
    assert rep.summary()["failed"] == 2


def test_late_short_request_joins_and_finishes_first():
    """Continuous batching: a short request arriving while a long one runs is
    admitted at the next chunk boundary and completes before it."""
    clk = FakeClock()
    be = CountingBackend(clk)
    long = JobSpec(job_id=0, lattice=19, shape=(64, 64, 64), steps=2000, arrival=0.0)
    t_long = long.nodes * long.steps * 1e-9
    short = JobSpec(job_id=1, lattice=19, shape=(16, 16, 16), steps=200, arrival=0.3 * t_long)
    rep = Server(be, hbm_budget=10 ** 12, chunk_steps=100, clock=clk, sleep=clk.sleep).run([long, short])
    r0, r1 = rep.results
    assert r1.admitted < r0.finished
    assert r1.finished < r0.finished
    assert r1.admitted - short.arrival <= long.nodes * 100 * 1e-9 + 1e-12  # within one chunk
    assert rep.max_active == 2


class ThreadedBackend:
    """Real-time fake for the overlapped server: set-up and read-back run on
    the worker thread while steps run on the main thread; tracks the live
    bytes under a lock and records when set-ups ran during a step."""

    def __init__(self, bytes_per_node=100, fail_create=(), fail_read=(), t_create=0.004,
                 t_read=0.002, s_per_lu=2e-9):
        import threading

        self.lock = threading.Lock()
        self.bpn = bytes_per_node
        self.fail_create, self.fail_read = set(fail_create), set(fail_read)
        self.t_create, self.t_read, self.s_per_lu = t_create, t_read, s_per_lu
        self.live = self.max_live = self.live_bytes = self.max_live_bytes = 0
        self.admit_order = []
        self.stepping = False
        self.overlapped = 0

    def required_bytes(self, spec):
        return spec.nodes * self.bpn

    def create(self, spec):
        import time as _t

        with self.lock:
            self.admit_order.append(spec.job_id)
            self.overlapped += self.stepping
        _t.sleep(self.t_create)
        if spec.job_id in self.fail_create:
            raise RuntimeError("create failed")
        with self.lock:
            self.live += 1
            self.max_live = max(self.max_live, self.live)
            self.live_bytes += self.required_bytes(spec)
            self.max_live_bytes = max(self.max_live_bytes, self.live_bytes)
        return spec

    def step(self, handles, nsteps):
        import time as _t

        self.stepping = True
        _t.sleep(sum(h.nodes * k for h, k in zip(handles, nsteps)) * self.s_per_lu)
        self.stepping = False

    def read(self, h, spec):
        import time as _t

        _t.sleep(self.t_read)
        if spec.job_id in self.fail_read:
            raise FloatingPointError("non-finite state")
        return {"job": spec.job_id}

    def destroy(self, h):
        with self.lock:
            self.live -= 1
            self.live_bytes -= self.required_bytes(h)


def test_overlapped_server_respects_budget_order_and_failures():
    be = ThreadedBackend(fail_create={2}, fail_read={5})
    specs = _specs(10, gap=2e-3)
    need = specs[0].nodes * 100
    rep = Server(be, hbm_budget=int(3.5 * need), chunk_steps=40, keep_moments=True,
                 overlap=True).run(specs)
    st = [r.status for r in rep.results]
    assert st == ["done", "done", "failed", "done", "done", "failed", "done", "done", "done", "done"]
    assert be.admit_order == list(range(10))
    assert be.max_live_bytes <= 3.5 * need and rep.peak_bytes <= 3.5 * need
    assert be.live == 0 and be.live_bytes == 0
    assert all(r.moments == {"job": r.job_id} for r in rep.results if r.status == "done")
    assert all(r.admitted >= r.arrival and r.finished >= r.admitted for r in rep.results)
    # set-ups ran on the worker while the main thread was stepping
    assert be.overlapped > 0
    assert set(rep.phase_s) >= {"create", "step", "read", "wait", "idle"}


def test_overlapped_server_matches_serial_statuses_and_work():
    specs = poisson_mix(30, rate=400.0, seed=3, edge_min=8, edge_max=24, steps=(20, 120))
    clk = FakeClock()
    serial = Server(CountingBackend(clk), hbm_budget=60 * 24 ** 3 * 100, chunk_steps=25,
                    clock=clk, sleep=clk.sleep).run(specs)
    over = Server(ThreadedBackend(s_per_lu=1e-10), hbm_budget=60 * 24 ** 3 * 100, chunk_steps=25,
                  overlap=True).run(specs)
    assert [r.status for r in over.results] == [r.status for r in serial.results]
    assert over.lattice_updates == serial.lattice_updates


def test_percentiles_and_throughput():
    res = [JobResult(i, "done", 0.0, 0.0, float(i + 1), lattice_updates=10 ** 6) for i in range(100)]
    res.append(JobResult(100, "failed", 0.0, 0.0, 1e9))
    rep = ServeReport(res, makespan=100.0, max_active=4, peak_bytes=0)
    tts = np.arange(1, 101, dtype=float)
    assert rep.p50 == pytest.approx(np.percentile(tts, 50))
    assert rep.p99 == pytest.approx(np.percentile(tts, 99))
    assert rep.mlups == pytest.approx(1.0)


def test_poisson_mix_is_seeded_and_in_range():
    a = poisson_mix(200, rate=50.0, seed=5)
    b = poisson_mix(200, rate=50.0, seed=5)
    assert [(s.shape, s.steps, s.arrival) for s in a] == [(s.shape, s.steps, s.arrival) for s in b]
    gaps = np.diff([0.0] + [s.arrival for s in a])
    assert 0.012 < gaps.mean() < 0.03
    for s in a:
        n = s.shape[0]
        assert 64 <= n <= 256 and 200 <= s.steps <= 2000
        assert s.shape == ((n, n, 1) if s.lattice == 9 else (n, n, n))
        assert s.storage in ("f32", "f16s") and s.flow in ("tg", "channel")


class OracleBackend:
    """Tiny grids through the FP64 oracle: results must not depend on the mix."""

    def __init__(self):
        self.state = {}

    def _params(self, spec):
        return oracle.Params(lattice=spec.lattice, nx=spec.shape[0], ny=spec.shape[1],
                             nz=spec.shape[2], tau=spec.tau, force=spec.force(), bb=spec.bc())

    def required_bytes(self, spec):
        return spec.nodes * 8 * spec.lattice

    def create(self, spec):
        rho, u = spec.fields()
        p = self._params(spec)
        return (p, oracle.init(p, rho, u))

    def step(self, handles, nsteps):
        for (p, f), k in zip(handles, nsteps):
            oracle.run(p, f, k)

    def read(self, h, spec):
        return oracle.moments(h[0], h[1])

    def destroy(self, h):
        pass


def test_result_in_a_mix_equals_result_alone():
    specs = [JobSpec(0, 19, (8, 6, 5), 37, flow="tg"),
             JobSpec(1, 9, (12, 10, 1), 55, flow="channel", arrival=0.0),
             JobSpec(2, 19, (6, 6, 9), 20, flow="channel"),
             JobSpec(3, 9, (9, 7, 1), 80, flow="tg")]
    mix = Server(OracleBackend(), hbm_budget=10 ** 9, chunk_steps=16, keep_moments=True).run(specs)
    for s, r in zip(specs, mix.results):
        alone = Server(OracleBackend(), hbm_budget=10 ** 9, chunk_steps=1000,
                       keep_moments=True).run([s]).results[0]
        assert r.status == alone.status == "done"
        for k in ("rho", "u", "pineq"):
            assert np.array_equal(r.moments[k], alone.moments[k])


class BlowUpBackend(CountingBackend):
    """Job `bad` blows up after `at` steps; blown_up() reports it from then on."""

    def __init__(self, clock, bad, at, **kw):
        super().__init__(clock, **kw)
        self.bad, self.at = bad, at
        self.done = {}
        self.stepped_after_failure = 0

    def step(self, handles, nsteps):
        super().step(handles, nsteps)
        for h, k in zip(handles, nsteps):
            if h.job_id == self.bad and self.done.get(h.job_id, 0) >= self.at:
                self.stepped_after_failure += 1
            self.done[h.job_id] = self.done.get(h.job_id, 0) + k

    def blown_up(self, handles):
        return [i for i, h in enumerate(handles)
                if h.job_id == self.bad and self.done[h.job_id] >= self.at]


@pytest.mark.parametrize("overlap", [False, True])
def test_blown_up_job_fails_at_the_next_chunk_and_frees_its_slot(overlap):
    clk = FakeClock()
    be = BlowUpBackend(clk, bad=1, at=130)
    specs = _specs(4, steps=1000)
    need = specs[0].nodes * 100
    rep = Server(be, hbm_budget=int(3.5 * need), chunk_steps=100, clock=clk, sleep=clk.sleep,
                 overlap=overlap).run(specs)
    r = {x.job_id: x for x in rep.results}
    assert r[1].status == "failed" and "within 200 steps" in r[1].error
    assert be.stepped_after_failure == 0     # never stepped again once detected
    assert all(r[i].status == "done" for i in (0, 2, 3))
    assert be.live == 0
    assert r[1].finished < r[2].finished     # stopped early, not after its 1000 steps


def test_blow_up_check_can_be_switched_off():
    clk = FakeClock()
    be = BlowUpBackend(clk, bad=0, at=50)
    rep = Server(be, hbm_budget=10 ** 12, chunk_steps=100, clock=clk, sleep=clk.sleep,
                 check_finite=False).run(_specs(1, steps=300))
    assert rep.results[0].status == "done"
