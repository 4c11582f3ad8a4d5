"""Continuous-batching server on the GPU: requests of the served mix (Sod variants,
Taylor-Green vortices, Becker shocks; FP32 and FP16 storage) arrive while others
run, overlap on the device, and each result equals -- bitwise -- the same request
run alone in a single context."""
import numpy as np
import pytest
import torch

from paper_2609_16361_amd import binding, inputs, serve

pytestmark = pytest.mark.gpu


def test_results_alone_equal_in_mix():
    trace = inputs.serving_trace(count=12, rate=400.0, seed=5, steps_range=(40, 400),
                                 tgv_n=(12, 20), sod_n=(64, 300), becker_L=(64, 200))
    results = {}

    def keep(req, Q):
        results[req.rid] = Q
        return bool(np.isfinite(Q).all())

    with binding.Batch(1 << 28, graph_steps=16) as b:
        srv = serve.Server(b, arena_bytes=(1 << 28) - (1 << 20), chunk_steps=16,
                           result_handler=keep, sync=torch.cuda.synchronize)
        st = srv.serve(trace)
    s = st.summary()
    print(s, flush=True)
    assert s["completed"] == len(trace) and st.max_active >= 3    # requests overlapped
    for r in trace:
        with binding.Solver(r.case.params, storage=r.storage) as one:
            one.init(r.case.Q0)
            one.step(r.steps)
            Q = one.moments()
        assert np.array_equal(Q, results[r.rid]), (r.rid, r.kind)
