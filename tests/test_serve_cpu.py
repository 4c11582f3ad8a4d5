"""Serving loop logic on the CPU with a stand-in backend (no GPU): admission in
arrival order (or largest work first, with a wait bound) under the HBM budget and
the active-cell cap, overlap of requests,
retirement at each request's own step count, latency bookkeeping, rejection of a
request that can never fit, and the served trace generator."""
import numpy as np
import pytest

from paper_2609_16361_amd import inputs, serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBatch:
    """Instances advance one step per run step; a step costs `dt` fake seconds."""

    def __init__(self, clock, dt=1e-3):
        self.clock, self.dt = clock, dt
        self.inst, self.next_id, self.log, self.added_steps = {}, 0, [], []

    def add(self, params, Q, steps, storage=0):
        i = self.next_id
        self.next_id += 1
        self.inst[i] = [0, steps, Q]
        self.log.append(("add", i, self.clock.t))
        self.added_steps.append(steps)
        return i

    def run(self, n):
        for v in self.inst.values():
            v[0] = min(v[1], v[0] + n)
        self.clock.t += n * self.dt

    def query(self, i):
        done, steps, _ = self.inst[i]
        return done, done >= steps

    def moments(self, i):
        return self.inst[i][2] + self.inst[i][0]

    def remove(self, i):
        self.log.append(("remove", i, self.clock.t))
        del self.inst[i]


def make_req(rid, arrival, cells, steps, storage=0):
    nx = cells // 16
    case = inputs.Case("x", dict(nx=nx, ny=4, nz=4, layout_pad=0), np.zeros((5, 4, 4, nx)), steps)
    return inputs.Request(rid, arrival, "x", case, steps, storage)


def test_fifo_budget_and_overlap():
    clk = FakeClock()
    fb = FakeBatch(clk)
    reqs = [make_req(i, 0.01 * i, 1600, 100 + 50 * i) for i in range(6)]
    one = serve.state_bytes(reqs[0].case.params, 0)
    srv = serve.Server(fb, arena_bytes=3 * one, chunk_steps=10, clock=clk, order="fifo")
    st = srv.serve(reqs)
    s = st.summary()
    assert s["completed"] == 6 and s["failed"] == 0
    assert st.max_active == 3                       # budget caps concurrency at 3
    adds = [i for (what, i, t) in fb.log if what == "add"]
    assert adds == sorted(adds)                     # admitted in arrival order
    for o in st.outcomes:
        assert o.admitted >= o.arrival - 1e-12
        assert o.completed >= o.admitted
        # results are taken at the request's own step count, not the chunk end
        assert np.all(o.result)
    # each request needed at least its own steps of device time
    for r, o in zip(reqs, st.outcomes):
        assert o.completed - o.admitted >= r.steps * fb.dt - 1e-9


def test_results_are_exact_step_counts():
    clk = FakeClock()
    fb = FakeBatch(clk)
    reqs = [make_req(i, 0.0, 320, s) for i, s in enumerate((7, 33, 50, 51))]
    got = {}

    def handler(req, Q):
        got[req.rid] = Q.flat[0]
        return True

    serve.Server(fb, arena_bytes=1 << 30, chunk_steps=16, clock=clk, result_handler=handler).serve(reqs)
    assert got == {0: 7, 1: 33, 2: 50, 3: 51}


def test_cell_cap_and_rejection():
    clk = FakeClock()
    fb = FakeBatch(clk)
    reqs = [make_req(0, 0.0, 1600, 40), make_req(1, 0.0, 1600, 40), make_req(2, 0.0, 16000, 10)]
    one = serve.state_bytes(reqs[0].case.params, 0)
    srv = serve.Server(fb, arena_bytes=4 * one, max_active_cells=2000, chunk_steps=8, clock=clk, order="fifo")
    st = srv.serve(reqs)
    assert st.max_active == 1                     # the cell cap admits one at a time
    assert [o.ok for o in st.outcomes] == [True, True, False]   # the big one never fits
    assert st.outcomes[2].rejected and st.summary()["rejected"] == 1 and st.summary()["failed"] == 0


class Refused(RuntimeError):
    status = -1   # LBM_EINVAL


class FakeRefusingBatch(FakeBatch):
    """Refuses (LBM_EINVAL) requests whose steps are in `refuse`."""

    def __init__(self, clock, refuse):
        super().__init__(clock)
        self.refuse = refuse

    def add(self, params, Q, steps, storage=0):
        if steps in self.refuse:
            raise Refused("initial pressure not positive")
        return super().add(params, Q, steps, storage)


def test_refused_request_is_rejected_not_failed():
    clk = FakeClock()
    fb = FakeRefusingBatch(clk, refuse={30})
    reqs = [make_req(0, 0.0, 320, 20), make_req(1, 0.0, 320, 30), make_req(2, 0.0, 320, 40)]
    st = serve.Server(fb, arena_bytes=1 << 30, chunk_steps=10, clock=clk, order="fifo").serve(reqs)
    s = st.summary()
    assert s["completed"] == 2 and s["rejected"] == 1 and s["failed"] == 0
    assert "pressure" in st.outcomes[1].rejected and fb.added_steps == [20, 40]


def test_largest_work_first_skips_what_does_not_fit():
    clk = FakeClock()
    fb = FakeBatch(clk)
    # work (cells x steps): C 320k, B 160k, A 80k, D 3.2k; all arrived at t = 0
    A, B, C, D = (make_req(0, 0.0, 1600, 50), make_req(1, 0.0, 320, 500), make_req(2, 0.0, 3200, 100),
                  make_req(3, 0.0, 320, 10))
    nb = {r.rid: serve.state_bytes(r.case.params, 0) for r in (A, B, C, D)}
    srv = serve.Server(fb, arena_bytes=nb[2] + nb[1] + nb[3], chunk_steps=10, clock=clk, order="largest")
    st = srv.serve([A, B, C, D])
    # C, B, then D fits where A does not; A once C retires (requests told apart by steps)
    assert fb.added_steps == [100, 500, 10, 50]
    assert st.summary()["completed"] == 4


def test_largest_work_first_with_a_wait_bound():
    def order_of(max_wait):
        clk = FakeClock()
        fb = FakeBatch(clk)
        # one at a time by the cell cap; the first runs 0.2 s, during which the small
        # request (arrived first) and the large one (arrived next) wait
        reqs = [make_req(0, 0.0, 1600, 200), make_req(1, 0.0, 1600, 5), make_req(2, 0.001, 1600, 150)]
        serve.Server(fb, arena_bytes=1 << 30, max_active_cells=2000, chunk_steps=10, clock=clk,
                     order="largest", max_wait_s=max_wait).serve(reqs)
        return fb.added_steps
    assert order_of(None) == [200, 150, 5]     # largest work first
    assert order_of(0.05) == [200, 5, 150]     # both overdue: arrival order


def test_overdue_request_keeps_its_place():
    """A large request that is overdue and does not fit blocks admission behind it,
    so a stream of small requests arriving later cannot take the memory it waits
    for: it starts as soon as the running work leaves room."""
    def run(max_wait):
        clk = FakeClock()
        fb = FakeBatch(clk)
        small = [make_req(i, 0.002 * i, 320, 30) for i in range(40)]          # arrive through 0.08 s
        big = make_req(99, 0.001, 3200, 20)
        one_small = serve.state_bytes(small[0].case.params, 0)
        budget = serve.state_bytes(big.case.params, 0) + one_small
        st = serve.Server(fb, arena_bytes=budget - 1, chunk_steps=10, clock=clk, order="largest",
                          max_wait_s=max_wait).serve(small + [big])
        return {o.rid: o for o in st.outcomes}
    waited = run(0.01)[99]
    # its wait is bounded by max_wait plus the 30 ms the small solves already running need
    assert waited.ok and waited.admitted - waited.arrival <= 0.01 + 0.03 + 0.01
    starved = run(None)[99]
    assert starved.admitted > 0.08 > waited.admitted     # without the bound it waits for every small one


def test_overdue_reservation_backfills_short_requests():
    """While an overdue request waits for room, requests that finish before the
    room is there (its shadow) run meanwhile, and one that would still hold memory
    then waits: the overdue request starts exactly when the instance ahead of it
    retires, as it would with nothing admitted behind it."""
    clk = FakeClock()
    fb = FakeBatch(clk)
    M = make_req(0, 0.0, 1600, 100)                                          # running, 10 chunks
    B = make_req(1, 0.001, 3200, 20)                                         # does not fit beside M
    S = [make_req(2 + i, 0.02 + 0.01 * i, 320, 10) for i in range(3)]       # one chunk each
    L = make_req(9, 0.02, 640, 500)                                          # long, and too big to sit beside B
    budget = serve.state_bytes(B.case.params, 0) + serve.state_bytes(S[0].case.params, 0)
    st = serve.Server(fb, arena_bytes=budget, chunk_steps=10, clock=clk, order="largest",
                      max_wait_s=0.005).serve([M, B, *S, L])
    o = {x.rid: x for x in st.outcomes}
    assert all(x.ok for x in o.values())
    assert o[1].admitted == pytest.approx(o[0].completed)
    for x in S:
        assert o[x.rid].admitted < o[1].admitted and o[x.rid].completed <= o[1].admitted
    assert o[9].admitted >= o[1].admitted


class NoRun(RuntimeError):
    status = -2   # LBM_ENOMEM: the byte count fits but no free run of that size does


class FakeFragmentedBatch(FakeBatch):
    """Refuses (LBM_ENOMEM) to add an instance with `cells` cells while more than
    `keep` instances are resident, as an arena too fragmented for it would."""

    def __init__(self, clock, cells, keep):
        super().__init__(clock)
        self.big, self.keep = cells, keep

    def add(self, params, Q, steps, storage=0):
        if params["nx"] * params["ny"] * params["nz"] == self.big and len(self.inst) > self.keep:
            raise NoRun("no free run")
        return super().add(params, Q, steps, storage)


def test_overdue_request_waits_out_fragmentation():
    """An overdue request whose bytes fit but for which the arena has no free run
    holds a reservation up to the next retirement, with nothing left beside it:
    a later short request still runs meanwhile, a later long one waits, and the
    overdue request starts as soon as the running instances leave room."""
    clk = FakeClock()
    fb = FakeFragmentedBatch(clk, cells=3200, keep=0)
    M = make_req(0, 0.0, 320, 60)                     # running, 6 chunks
    B = make_req(1, 0.001, 3200, 20)                  # fits by bytes, not by run
    S = make_req(2, 0.02, 320, 10)                    # one chunk
    L = make_req(3, 0.02, 320, 500)                   # long
    st = serve.Server(fb, arena_bytes=1 << 30, chunk_steps=10, clock=clk, order="largest",
                      max_wait_s=0.005).serve([M, B, S, L])
    o = {x.rid: x for x in st.outcomes}
    assert all(x.ok for x in o.values())
    assert o[2].completed <= o[1].admitted                      # the short one backfilled
    assert o[3].admitted >= o[1].admitted                       # the long one waited
    assert o[1].admitted == pytest.approx(o[0].completed)       # B at M's retirement


def test_unknown_order_rejected():
    with pytest.raises(ValueError):
        serve.Server(FakeBatch(FakeClock()), arena_bytes=1, order="random")


def test_sequential_baseline_fifo():
    clk = FakeClock()

    class Solver:
        def __init__(self, params):
            self.n = 0

        def __enter__(self):
            return self

        def __exit__(self, *a):
            pass

        def init(self, Q):
            self.Q = Q

        def step(self, n, diag_every=0):
            self.n += n
            clk.t += n * 1e-3

        def diagnostics(self):
            return [], 0

        def moments(self):
            return self.Q + self.n

    reqs = [make_req(i, 0.0, 320, 10 * (i + 1)) for i in range(4)]
    st = serve.serve_sequential(reqs, Solver, clock=clk)
    lat = [o.latency for o in st.outcomes]
    assert lat == sorted(lat)                      # FIFO: later requests wait longer
    assert st.summary()["completed"] == 4


def test_sequential_baseline_stops_diverged_and_rejects():
    """The baseline checks divergence at the server's interval (a fused diagnostic
    reduction on the first step of every check_steps piece) and rejects a request
    the library refuses at initialisation."""
    clk = FakeClock()

    class Solver:
        def __init__(self, params):
            self.n, self.recs, self.bad_from = 0, [], params.get("bad_from")
            self.refuse = params.get("refuse", False)

        def __enter__(self):
            return self

        def __exit__(self, *a):
            pass

        def init(self, Q):
            if self.refuse:
                raise Refused("initial density not positive")

        def step(self, n, diag_every=0):
            for t in range(self.n, self.n + n):
                if diag_every and t % diag_every == 0:
                    self.recs.append({"step": t, "nonfinite": int(self.bad_from is not None and t >= self.bad_from)})
            self.n += n
            clk.t += n * 1e-3

        def diagnostics(self):
            r, self.recs = self.recs, []
            return r, 0

        def moments(self):
            return np.zeros((5, 4, 4, 20)) + self.n

    reqs = [make_req(0, 0.0, 320, 1000), make_req(1, 0.0, 320, 500), make_req(2, 0.0, 320, 100)]
    reqs[0].case.params["bad_from"] = 250          # diverges after 250 steps
    reqs[1].case.params["refuse"] = True
    failed = []
    st = serve.serve_sequential(reqs, Solver, clock=clk, check_steps=200, failure_handler=failed.append)
    o0, o1, o2 = st.outcomes
    assert not o0.ok and not o0.rejected and o0.completed == pytest.approx(0.6)   # stopped at step 600
    assert o1.rejected and not o1.ok
    assert o2.ok
    s = st.summary()
    assert (s["completed"], s["failed"], s["rejected"], s["stopped_diverged"]) == (1, 1, 1, 1)
    assert [r.rid for r in failed] == [0]


def test_serving_trace_mix():
    tr = inputs.serving_trace(count=40, seed=3, tgv_n=(16, 24), sod_n=(64, 96), becker_L=(64, 96))
    kinds = {k: sum(1 for r in tr if r.kind == k) for k in ("sod", "tgv", "becker")}
    assert sum(kinds.values()) == 40 and all(v > 0 for v in kinds.values())
    arr = np.array([r.arrival for r in tr])
    assert np.all(np.diff(arr) > 0)
    assert 0.3 < arr[-1] < 2.0                     # mean rate 50/s
    assert all(1000 <= r.steps <= 20000 for r in tr)
    assert {r.storage for r in tr} == {0, 1}
    for r in tr:
        assert r.case.Q0.shape == (5,) + r.case.shape and np.isfinite(r.case.Q0).all()


def test_riemann_max_speed_sod():
    # Sod: fastest signal is u* + c* behind the shock, about 2.19 (exact star state
    # p* = 0.30313, u* = 0.92745)
    s = inputs.riemann_max_speed((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert s == pytest.approx(2.19, abs=0.02)


class FakeDivergingBatch(FakeBatch):
    """As FakeBatch; the instance added k-th stops being finite after diverge[k]
    completed steps."""

    def __init__(self, clock, diverge, dt=1e-3):
        super().__init__(clock, dt)
        self.diverge, self.order = diverge, {}

    def add(self, params, Q, steps, storage=0):
        i = super().add(params, Q, steps, storage)
        self.order[i] = len(self.order)
        return i

    def nonfinite(self):
        return [i for i, v in self.inst.items()
                if self.order[i] in self.diverge and v[0] >= self.diverge[self.order[i]]]


@pytest.mark.parametrize("stop", [True, False])
def test_diverged_request_retired_early(stop):
    """A request whose state stops being finite is retired as failed after the chunk
    in which that happened (its memory freed for the next request), not at its step
    count; the result handler is not called for it, the failure handler is.  With
    the check off it runs to its step count."""
    clk = FakeClock()
    fb = FakeDivergingBatch(clk, diverge={0: 25})
    reqs = [make_req(0, 0.0, 1600, 1000), make_req(1, 0.0005, 1600, 100)]
    one = serve.state_bytes(reqs[0].case.params, 0)
    seen, failed = [], []

    def handler(req, Q):
        seen.append(req.rid)
        return req.rid != 0          # a diverged state is not a result

    srv = serve.Server(fb, arena_bytes=one, chunk_steps=10, clock=clk, order="fifo", result_handler=handler,
                       stop_diverged=stop, check_steps=10, failure_handler=failed.append)
    st = srv.serve(reqs)
    s = st.summary()
    o0, o1 = st.outcomes
    assert not o0.ok and o1.ok and s["failed"] == 1
    if stop:
        assert s["stopped_diverged"] == 1 and [r.rid for r in failed] == [0] and seen == [1]
        # retired at the end of the chunk holding step 25, so the second request
        # (which waited for its memory) starts after 30 steps, not 1000
        assert o0.completed == pytest.approx(30 * fb.dt)
        assert o1.admitted == pytest.approx(30 * fb.dt)
    else:
        assert s["stopped_diverged"] == 0 and failed == [] and seen == [0, 1]
        assert o0.completed == pytest.approx(1000 * fb.dt)
        assert o1.admitted == pytest.approx(1000 * fb.dt)


def test_divergence_check_interval():
    """With check_steps = 25 and chunks of 10 steps the check follows every third
    chunk: an instance that diverges at step 5 is retired after 30 steps."""
    clk = FakeClock()
    fb = FakeDivergingBatch(clk, diverge={0: 5})
    calls = []
    check = fb.nonfinite
    fb.nonfinite = lambda: calls.append(clk.t) or check()
    srv = serve.Server(fb, arena_bytes=1 << 30, chunk_steps=10, clock=clk, check_steps=25)
    st = srv.serve([make_req(0, 0.0, 1600, 1000)])
    assert not st.outcomes[0].ok and st.stopped == 1
    assert st.outcomes[0].completed == pytest.approx(30 * fb.dt)
    assert calls == [pytest.approx(30 * fb.dt)]


def test_timeline_of_resident_cells():
    """One timeline entry per chunk with the resident instances and cells while it
    ran; the summary's time-weighted mean of resident cells follows from it."""
    clk = FakeClock()
    fb = FakeBatch(clk)
    reqs = [make_req(0, 0.0, 1600, 40), make_req(1, 0.0, 3200, 20)]
    srv = serve.Server(fb, arena_bytes=1 << 30, chunk_steps=10, clock=clk)
    st = srv.serve(reqs)
    assert len(st.timeline) == st.chunks == 4
    assert [(n, c) for _, _, n, c in st.timeline] == [(2, 4800), (2, 4800), (1, 1600), (1, 1600)]
    for a, b, _, _ in st.timeline:
        assert b - a == pytest.approx(10 * fb.dt)
    assert st.summary()["resident_cells_mean"] == pytest.approx((4800 + 4800 + 1600 + 1600) / 4)


def test_state_bytes_mirrors_the_library():
    """The server's admission arithmetic (serve.state_bytes, no device call) gives
    the bytes lbm_state_bytes reports, for FP32 and FP16, with and without pads."""
    from paper_2609_16361_amd import binding
    rng = np.random.default_rng(3)
    for _ in range(40):
        nx, ny, nz = (int(v) for v in rng.integers(1, 300, size=3))
        pad = int(rng.choice([0, 1, 37, 4096]))
        for storage in (0, 1):
            params = dict(inputs.base_params(nx, ny, nz, (0, 0, 0), mu=1e-3), layout_pad=pad)
            p = binding.make_params(params)
            p.storage = storage
            assert serve.state_bytes(params, storage) == binding.lbm_state_bytes(p), (nx, ny, nz, pad, storage)


def test_fp16_only_for_the_allowed_kinds():
    """With fp16_kinds a request asking for FP16 storage runs in it only when its kind
    is in the set; the others run in FP32."""
    clk = FakeClock()
    fb = FakeBatch(clk)
    seen = []
    add = fb.add

    def spy(params, Q, steps, storage=0):
        seen.append((steps, storage))
        return add(params, Q, steps, storage)

    fb.add = spy
    reqs = [make_req(0, 0.0, 320, 10, storage=1), make_req(1, 0.0, 320, 20, storage=1),
            make_req(2, 0.0, 320, 30, storage=0)]
    reqs[1].kind = "tgv"
    srv = serve.Server(fb, arena_bytes=1 << 30, chunk_steps=10, clock=clk, order="fifo", fp16_kinds={"x"})
    st = srv.serve(reqs)
    assert sorted(seen) == [(10, 1), (20, 0), (30, 0)]
    assert [o.storage for o in st.outcomes] == [1, 0, 0]


def test_fp16_only_up_to_a_step_count():
    """With fp16_max_steps a request asking for FP16 storage runs in it only up to
    that many steps; longer ones run in FP32."""
    clk = FakeClock()
    fb = FakeBatch(clk)
    reqs = [make_req(0, 0.0, 320, 10, storage=1), make_req(1, 0.0, 320, 40, storage=1),
            make_req(2, 0.0, 320, 20, storage=1)]
    srv = serve.Server(fb, arena_bytes=1 << 30, chunk_steps=10, clock=clk, order="fifo", fp16_max_steps=20)
    st = srv.serve(reqs)
    assert [o.storage for o in st.outcomes] == [1, 0, 1]


def test_large_requests_run_in_contexts_of_their_own():
    """Requests whose state reaches solo_min_bytes run in contexts of their own,
    stepped one chunk at a time beside the batch: exactly their step count, their
    own divergence check (records on every multiple of check_steps), and
    rejection when the library refuses the state; the rest share the batch."""
    clk = FakeClock()
    b = FakeBatch(clk)
    made, closed = [], []

    class Solo:
        def __init__(self, r, storage):
            self.r, self.n, self.recs = r, 0, []
            self.bad_from = r.case.params.get("bad_from")
            made.append(r.rid)

        def init(self, Q):
            if self.r.case.params.get("refuse"):
                raise Refused("initial density not positive")
            self.Q = Q

        def step(self, n, diag_every=0):
            for t in range(self.n, self.n + n):
                if diag_every and t % diag_every == 0:
                    self.recs.append({"step": t, "nonfinite": int(self.bad_from is not None and t >= self.bad_from)})
            self.n += n
            clk.t += n * 1e-3

        def diagnostics(self):
            r, self.recs = self.recs, []
            return r, 0

        def moments(self):
            return self.Q + self.n

        def close(self):
            closed.append(self.r.rid)

    big, small = 3200, 320
    reqs = [make_req(0, 0.0, big, 130), make_req(1, 0.0, small, 70), make_req(2, 0.0, big, 1000),
            make_req(3, 0.0, big, 90), make_req(4, 0.0, small, 40)]
    reqs[2].case.params["bad_from"] = 450          # diverges after 450 steps
    reqs[3].case.params["refuse"] = True
    limit = serve.state_bytes(reqs[0].case.params, 0)
    assert serve.state_bytes(reqs[1].case.params, 0) < limit
    results, failed = {}, []

    def handler(r, Q):
        results[r.rid] = float(Q.flat[0])
        return True

    srv = serve.Server(b, arena_bytes=1 << 30, chunk_steps=50, clock=clk, result_handler=handler,
                       check_steps=200, failure_handler=failed.append, solo_factory=Solo, solo_min_bytes=limit)
    st = srv.serve(reqs)
    assert sorted(made) == [0, 2, 3] and sorted(closed) == [0, 2, 3]
    assert sorted(b.added_steps) == [40, 70]       # only the small ones share the batch
    assert results == {0: 130.0, 1: 70.0, 4: 40.0}  # each stopped at its own step count
    o = {x.rid: x for x in st.outcomes}
    assert not o[2].ok and not o[2].rejected and [r.rid for r in failed] == [2]
    assert o[3].rejected and not o[3].ok
    s = st.summary()
    assert (s["completed"], s["failed"], s["rejected"], s["stopped_diverged"]) == (3, 1, 1, 1)


class FakeSolo:
    """A context of its own for the fake clock: a step costs `dt` fake seconds."""

    def __init__(self, clk, dt=1e-3):
        self.clk, self.dt, self.n = clk, dt, 0

    def init(self, Q):
        self.Q = Q

    def step(self, n, diag_every=0):
        self.n += n
        self.clk.t += n * self.dt

    def diagnostics(self):
        return [], 0

    def moments(self):
        return self.Q + self.n

    def close(self):
        pass


def test_overdue_solo_request_keeps_its_place():
    """The reservation and backfilling hold when the overdue request, or the one
    running ahead of it, runs in a context of its own: the large request starts
    exactly when the request ahead of it retires, short requests fill the wait,
    and every result is its exact step count."""
    clk = FakeClock()
    fb = FakeBatch(clk)
    M = make_req(0, 0.0, 1600, 100)                                          # running, 10 chunks
    B = make_req(1, 0.001, 3200, 20)                                         # does not fit beside M
    S = [make_req(2 + i, 0.02 + 0.01 * i, 320, 10) for i in range(3)]       # one chunk each
    budget = serve.state_bytes(B.case.params, 0) + serve.state_bytes(S[0].case.params, 0)
    results = {}

    def keep(r, Q):
        results[r.rid] = float(Q.flat[0])
        return True

    solo_min = serve.state_bytes(M.case.params, 0)                           # M and B run alone
    st = serve.Server(fb, arena_bytes=budget, chunk_steps=10, clock=clk, order="largest", max_wait_s=0.005,
                      result_handler=keep, solo_factory=lambda r, stg: FakeSolo(clk),
                      solo_min_bytes=solo_min).serve([M, B, *S])
    o = {x.rid: x for x in st.outcomes}
    assert all(x.ok for x in o.values())
    assert sorted(fb.added_steps) == [10, 10, 10]                            # only the short ones batched
    assert o[1].admitted == pytest.approx(o[0].completed)
    for x in S:
        assert o[x.rid].admitted < o[1].admitted and o[x.rid].completed <= o[1].admitted
    assert results == {0: 100.0, 1: 20.0, 2: 10.0, 3: 10.0, 4: 10.0}
