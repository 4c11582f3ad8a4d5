#!/usr/bin/env python3
"""Benchmark of the fused collide-and-stream update on one MI355X.

Workload: the supersonic compressible Taylor-Green vortex on a 256^3 periodic grid
in FP32 (Mach 1.25, Re 1600, Pr 0.71, gamma 1.4, Sutherland viscosity, regularized
collision with the compression sensor), kinetic energy and solenoidal/dilatational
dissipation reduced every 50 steps.  One "step" is one lattice update of every
cell.  Inputs are synthetic (the analytic initial field) and resident in HBM
before the timed region starts.

Prints one JSON line with the metric, a `roofline` object for the collide-and-
stream kernel (HBM bound: 280 algorithmic bytes per cell update) measured with HIP
events on the stream the kernel runs on, and a `cpu_baseline` object: the FP64
oracle timed on a bounded sample of the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
BYTES_PER_LUP_F32 = 280.0    # 35 populations x 4 B, read and written once


def _oracle_rate(params, f, steps):
    """Oracle cell updates per second over `steps` steps after one warm-up step."""
    import oracle
    f, _ = oracle.run(params, f, 1)
    t0 = time.perf_counter()
    oracle.run(params, f, steps)
    return oracle.cells(params) * steps / (time.perf_counter() - t0)


def cpu_baseline(target_s=15.0):
    """The oracle as it stands on a slab of the 256^3 workload (full x-y planes,
    32 z-planes, periodic), stepped for about target_s of wall time; then the oracle's
    rate on the other configurations: the Sod tube in full (256x4x4, 400 steps), the
    first two tubes of the Becker batch (50 steps) and the 128^3 vortex of the
    precision study (3 steps)."""
    import numpy as np
    import oracle
    from paper_2609_16361_amd import inputs
    case = inputs.tgv(n=256, dims=(256, 256, 32))
    f = oracle.init(case.params, case.Q0)
    cells = case.cells
    f, _ = oracle.run(case.params, f, 1)  # thread start-up
    t0 = time.perf_counter()
    f, _ = oracle.run(case.params, f, 2)
    one = (time.perf_counter() - t0) / 2
    steps = max(1, int(target_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    f, _ = oracle.run(case.params, f, steps)
    dt = time.perf_counter() - t0
    assert np.isfinite(f).all()
    glups = cells * steps / dt / 1e9
    cores = oracle.num_threads()
    # one thread on the same slab, two steps after one warm-up step
    oracle.set_num_threads(1)
    try:
        f, _ = oracle.run(case.params, f, 1)
        t0 = time.perf_counter()
        f, _ = oracle.run(case.params, f, 2)
        glups_1 = cells * 2 / (time.perf_counter() - t0) / 1e9
    finally:
        oracle.set_num_threads(cores)
    del f
    configs = {}
    sod = inputs.sod(n=256, ny=4, nz=4, steps=400)
    t0 = time.perf_counter()
    oracle.run(sod.params, oracle.init(sod.params, sod.Q0), sod.steps)
    configs["sod_256x4x4_400_steps"] = {"mlups": sod.cells * sod.steps / (time.perf_counter() - t0) / 1e6,
                                        "sample": "full run"}
    tubes = inputs.becker_batch(2)
    t_b, lup_b = 0.0, 0
    for c in tubes:
        t0 = time.perf_counter()
        oracle.run(c.params, oracle.init(c.params, c.Q0), 50)
        t_b += time.perf_counter() - t0
        lup_b += c.cells * 50
    configs["becker_batch"] = {"mlups": lup_b / t_b / 1e6,
                               "sample": f"first 2 of the 64 tubes ({sum(c.cells for c in tubes)} cells), 50 steps"}
    v = inputs.tgv(n=128, steps=3)
    rate = _oracle_rate(v.params, oracle.init(v.params, v.Q0), 3)
    configs["tgv_128"] = {"mlups": rate / 1e6, "sample": "128^3, 3 steps after 1 warm-up step"}
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": glups, "unit": "GLUP/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, 256x256x32 slab of the 256^3 cTGV initial field, {steps} steps "
                      f"after 3 warm-up steps, {dt:.1f} s",
            "one_thread_value": glups_1, "cpu_model": model, "other_configs": configs}


def becker_linf(case, Q):
    """L-inf error of the density profile (row y = z = 0) against the closed-form
    Becker shock, relative to the density jump, after the best sub-cell shift of the
    exact profile (the discrete shock may settle a fraction of a cell away)."""
    import numpy as np
    from paper_2609_16361_amd import inputs
    m = case.meta
    rho = Q[0, 0, 0, :]
    # closed form once on a grid 1/20 cell fine, shifted copies by interpolation
    xf = np.arange(m["x"][0] - 3.0, m["x"][-1] + 3.0, 0.05)
    rf = inputs.becker_profile(xf, m["mach"], m["mu"], m["x_shock"], m["gamma"], 1.0, m["c1"])[0]
    jump = rf.max() - rf.min()
    best = None
    for sh in np.linspace(-2.0, 2.0, 81):
        re = np.interp(m["x"] - sh, xf, rf)
        e = np.abs(rho - re).max() / jump
        if best is None or e < best[0]:
            best = (e, sh)
    return best


def bench_batch(count=64, steps=5000, seed=0, stream=None, tuning=None, sequential=True):
    """Batched Becker shocks (seeded lengths 512-8192 x 4 x 4, Mach 1.5-5, FP32,
    regularized collision with sensor): autotuned batch kernel + graphs, against
    the same solves run one after another in single contexts.  A given tuning
    (block, nontemporal, blocks_per_cu, grid) replaces the autotuner; sequential=False
    skips the single-context baseline (counter runs of the batch kernel alone)."""
    import numpy as np
    import torch
    from paper_2609_16361_amd import binding, inputs
    cases = inputs.becker_batch(count, seed=seed)
    cells = sum(c.cells for c in cases)
    nbytes = sum(binding.lbm_state_bytes(binding.make_params(c.params)) for c in cases)
    out = {"instances": count, "steps": steps, "cells": cells, "seed": seed}
    t_wall = time.perf_counter()
    with binding.Batch(int(nbytes * 1.05) + (64 << 20), max_instances=count, graph_steps=50,
                       stream=stream.cuda_stream) as b:
        ids = [b.add(c.params, c.Q0, steps) for c in cases]
        if tuning is None:
            best, best_us, tried = b.autotune(trial_steps=50)
        else:
            b.set_tuning(*tuning)
            best, best_us, tried = b.info()["tuning"], None, []
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.run(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        t_batch = e0.elapsed_time(e1) * 1e-3
        errs = []
        for i, c in zip(ids, cases):
            done, fin = b.query(i)
            assert fin and done == steps
            errs.append(becker_linf(c, b.moments(i))[0])
    t_wall = time.perf_counter() - t_wall
    out["batched"] = {"solves_per_s": count / t_batch, "run_s": t_batch, "glups": cells * steps / t_batch / 1e9,
                      "hbm_frac": 280.0 * cells * steps / t_batch / 1e9 / HBM_PEAK_GBS,
                      "tuning": best, "tuned_us_per_step": best_us, "candidates": len(tried),
                      "wall_s_incl_init_readout": t_wall}
    out["linf_rel_error"] = {"median": float(np.median(errs)), "max": float(np.max(errs)),
                             "mach_of_max": float(cases[int(np.argmax(errs))].meta["mach"])}
    if not sequential:
        return out
    # the same solves one at a time, plain FP32 single contexts
    t_seq = 0.0
    t_wall = time.perf_counter()
    for c in cases:
        with binding.Solver(c.params, stream=stream.cuda_stream) as s:
            s.init(c.Q0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.step(steps)
            e1.record(stream)
            torch.cuda.synchronize()
            t_seq += e0.elapsed_time(e1) * 1e-3
    t_wall = time.perf_counter() - t_wall
    out["sequential"] = {"solves_per_s": count / t_seq, "run_s": t_seq, "glups": cells * steps / t_seq / 1e9,
                         "wall_s_incl_init_readout": t_wall}
    out["speedup"] = t_seq / t_batch
    return out


def bench_precision(stream, n=128, steps=4000, diag_every=50):
    """FP16 shifted storage against FP32 storage (both FP32 arithmetic) on the
    compressible Taylor-Green vortex at n^3: throughput of each, relative L2 over the
    diagnostic time series of E_k, eps_s and eps_d, and of the conserved fields at
    the end.  (Both against the FP64 oracle: tests/test_gpu_fp16.py.)"""
    import numpy as np
    import torch
    from paper_2609_16361_amd import binding, inputs
    case = inputs.tgv(n=n, steps=steps, diag_every=diag_every)
    series, fields, rates = {}, {}, {}
    for name, stg in (("f32", binding.LBM_STORE_F32), ("f16", binding.LBM_STORE_F16)):
        with binding.Solver(case.params, storage=stg, stream=stream.cuda_stream) as s:
            s.init(case.Q0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.step(steps, diag_every)
            e1.record(stream)
            torch.cuda.synchronize()
            rates[name] = case.cells * steps / (e0.elapsed_time(e1) * 1e-3) / 1e9
            recs, st = s.diagnostics()
            assert st == binding.LBM_OK
            series[name] = np.array([[r["Ek"], r["eps_s"], r["eps_d"]] for r in recs]) / case.cells
            fields[name] = s.moments()

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    k0 = 1  # the first record holds the start's central-difference gradients, not the update's
    out = {"workload": f"compressible Taylor-Green {n}^3, {steps} steps, diagnostics every {diag_every}",
           "glups": rates,
           "f16_vs_f32_series": {q: rel(series["f16"][k0:, i], series["f32"][k0:, i])
                                 for i, q in enumerate(("Ek", "eps_s", "eps_d"))},
           "f16_vs_f32_fields": [rel(fields["f16"][k], fields["f32"][k]) for k in range(5)],
           "Ek_final": {name: float(series[name][-1, 0] * case.meta["ek_scale"]) for name in series},
           "tc_final": steps * case.meta["tc_per_step"]}
    # against the FP64 oracle's series of the same workload (tests/golden, written
    # by make_tgv128_oracle_series.py from the oracle alone)
    gold = os.path.join(ROOT, "tests", "golden", f"tgv{n}_oracle_series.json")
    if os.path.exists(gold) and steps == 4000 and diag_every == 50:
        ref = json.load(open(gold))
        o = np.stack([np.array(ref[q]) for q in ("Ek", "eps_s", "eps_d")], axis=1)
        assert o.shape == series["f32"].shape, (o.shape, series["f32"].shape)
        for name in ("f32", "f16"):
            out[f"{name}_vs_oracle_series"] = {q: rel(series[name][k0:, i], o[k0:, i])
                                              for i, q in enumerate(("Ek", "eps_s", "eps_d"))}
    return out


def bench_mms(stream, sizes=(64, 128, 256), frac=0.5):
    """Order of accuracy on the manufactured solution of Sec. 3.1 (eq. 8), FP32 on the
    GPU: relative L2 error of each conserved field at t = 1 against the exact field
    at n^3 for each n, the empirical order of convergence from each pair, and the
    throughput.  The source is evaluated on the GPU each step at the step's mid-time."""
    import numpy as np
    import torch
    from paper_2609_16361_amd import binding, inputs
    out = {"sizes": list(sizes), "errors": {}, "eoc": {}, "glups": {}, "omega": {}, "steps": {}}
    prev = None
    for n in sizes:
        case = inputs.mms(n)
        S = torch.empty(5 * n ** 3, dtype=torch.float32, device="cuda")
        with binding.Solver(case.params, stream=stream.cuda_stream) as s:
            s.init(case.Q0)
            s.set_source(S.data_ptr())
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for step in range(case.steps):
                binding.lbm_mms_source(case.meta["mms"], n, n, n, step + frac, S.data_ptr(), stream.cuda_stream)
                s.step(1)
            e1.record(stream)
            torch.cuda.synchronize()
            Q = s.moments()
        del S
        Qe = inputs.mms_exact(case, case.steps)
        err = [float(np.linalg.norm(Q[k] - Qe[k]) / np.linalg.norm(Qe[k])) for k in range(5)]
        out["errors"][n] = err
        out["omega"][n] = case.meta["omega"]
        out["steps"][n] = case.steps
        out["glups"][n] = case.cells * case.steps / (e0.elapsed_time(e1) * 1e-3) / 1e9
        if prev is not None:
            out["eoc"][f"{prev[0]}->{n}"] = [float(np.log2(a / b)) for a, b in zip(prev[1], err)]
        prev = (n, err)
        print(f"mms {n}^3: errors {['%.3e' % e for e in err]}", file=sys.stderr, flush=True)
    return out


def bench_spectral(stream, n=128, tc_samples=(1.0, 2.0, 3.0, 4.0, 5.0)):
    """The dissipation channels of the compressible Taylor-Green vortex at n^3: the
    fused in-collision values (reconstructed gradients) against the spectral values
    of the same state (Fourier derivatives of lbm_moments output, Sec. 3.3), at
    several convective times, in the paper's units (divided by rho0, converted)."""
    from paper_2609_16361_amd import binding, inputs, spectral
    case = inputs.tgv(n=n, diag_every=0)
    scale = case.meta["eps_scale"]
    rows = []
    with binding.Solver(case.params, stream=stream.cuda_stream) as s:
        s.init(case.Q0)
        done = 0
        for tc in tc_samples:
            target = int(round(tc / case.meta["tc_per_step"]))
            s.step(target - done)
            Q = s.moments()
            s.step(1, 1)                  # the fused record of this state
            done = target + 1
            recs, st = s.diagnostics()
            assert st == binding.LBM_OK and recs[-1]["step"] == target
            ek, es, ed = spectral.channels(Q, case.params)
            fs, fd = recs[-1]["eps_s"] / case.cells, recs[-1]["eps_d"] / case.cells
            rows.append({"tc": target * case.meta["tc_per_step"], "step": target,
                         "eps_s": {"fused": fs * scale, "spectral": es * scale, "ratio": fs / es},
                         "eps_d": {"fused": fd * scale, "spectral": ed * scale, "ratio": fd / ed}})
            print(f"spectral t_c {rows[-1]['tc']:.2f}: eps_s ratio {fs / es:.3f} eps_d ratio {fd / ed:.3f}",
                  file=sys.stderr, flush=True)
    return {"workload": f"compressible Taylor-Green {n}^3", "samples": rows}


# Kinds whose FP16-served results meet the 1e-2 bar against FP32 (relative L2 of
# rho, rho u, E).  Vortices run near omega = 2, where the regularized collision
# amplifies FP16 rounding (measured 0.10 median, 0.52 worst on the 64-request
# mix); they are served in FP32.
FP16_KINDS = ("sod", "becker")
# FP16 rounding error grows about as the square root of the step count: the worst
# FP16 Sod tubes of the 1000-request trace reached about 8.2e-5 sqrt(steps) against
# FP32, which passes the 1e-2 bar at about 15000 steps; longer requests run in FP32
FP16_MAX_STEPS = 12000
# Requests whose state takes this much or more run in contexts of their own beside
# the batch: from about this size the single-context kernels, with plain access up
# to 320 MB and nontemporal beyond, move a state faster than the batch kernel does
# (the mix's vortices of 63^3-127^3 alone at 17.9-22.6 GLUP/s against 17.4 for all
# of its vortices in one batch), while smaller states are launch-bound alone.
SOLO_MIN_BYTES = 24 << 20


def bench_serve(stream, count=64, rate=50.0, seed=1, budget_bytes=200 * 10 ** 9, chunk=50,
                max_active_cells=8 * 2 ** 20):
    """Serving mix (Poisson arrivals at `rate`, 40% Sod variants, 40% Taylor-Green,
    20% Becker; 1000-20000 steps; FP32 or FP16 storage per request) through the
    continuous-batching server under an HBM budget (its default admission order),
    against the same requests served one at a time, in arrival order, in plain FP32
    single contexts."""
    import numpy as np
    import torch
    from paper_2609_16361_amd import binding, inputs, serve
    trace = inputs.serving_trace(count=count, rate=rate, seed=seed)
    work = sum(r.case.cells * r.steps for r in trace)
    out = {"requests": count, "rate_per_s": rate, "seed": seed, "budget_bytes": budget_bytes,
           "admission": "largest work first among arrived requests, any request waiting over 2 s first",
           "divergence": "checked every 200 steps in every leg; a diverged request stops at once as failed",
           "rejection": "a request whose initial density or pressure is not positive is refused by the "
                        "library (LBM_EINVAL) in every leg and counted as rejected",
           "solo": f"batched legs: requests of {SOLO_MIN_BYTES >> 20} MiB of state or more run in contexts of "
                   "their own beside the batch, one chunk at a time",
           "offered_glup": work / 1e9,
           "mix": {k: sum(1 for r in trace if r.kind == k) for k in ("sod", "tgv", "becker")},
           "fp16_share": sum(r.storage for r in trace) / count,
           "fp16_served": {"kinds": list(FP16_KINDS), "max_steps": FP16_MAX_STEPS,
                           "requests": sum(1 for r in trace if r.storage and r.kind in FP16_KINDS and
                                           r.steps <= FP16_MAX_STEPS),
                           "note": "FP16 requested by vortices is served in FP32: near omega = 2 their FP16 "
                                   "results miss the 1e-2 bar against FP32; so are requests of more than "
                                   "max_steps steps, whose FP16 rounding error grows past it"}}

    failures = {}
    progress = {"leg": "", "done": 0}  # long traces report every 100 results on stderr
    f16_results = {}                   # FP16-served results of the mixed leg, by request
    f16_err = {}                       # kind -> per request, max over rho, rho u, E of rel. L2

    def failed(req):
        failures[req.rid] = {"kind": req.kind, "shape": list(req.case.shape), "steps": req.steps,
                             "storage": req.storage,
                             **{k: req.case.meta[k] for k in ("mach", "left", "right", "r") if k in req.case.meta}}

    def finished(req, ok):
        progress["done"] += 1
        if count >= 200 and progress["done"] % 100 == 0:
            print(f"serve {progress['leg']}: {progress['done']}/{count} results", file=sys.stderr, flush=True)
        if not ok:
            failed(req)
        return ok

    def finite(req, Q):
        return finished(req, bool(np.isfinite(Q).all()))

    def keep_f16(req, Q):
        ok = finite(req, Q)
        if ok and req.storage == binding.LBM_STORE_F16 and req.kind in FP16_KINDS and req.steps <= FP16_MAX_STEPS:
            f16_results[req.rid] = Q.astype(np.float32)
        return ok

    def compare_f32(req, Q):
        # FP32 results of the batch are bitwise those of the sequential FP32 solves
        ok = finite(req, Q)
        a = f16_results.pop(req.rid, None)
        if ok and a is not None:
            # the momentum against the larger of its own norm and the acoustic
            # momentum scale rho_ref c_ref sqrt(N): a weak tube's momentum decays
            # towards zero over its run, and relative to a vanishing field any
            # rounding is a large fraction
            p = req.case.params
            mscale = p["rho_ref"] * np.sqrt(p["gamma"] * (p["gamma"] - 1.0) * p["E_ref"] / p["rho_ref"]) * \
                np.sqrt(req.case.cells)
            m, ma = Q[1:4], a[1:4].astype(np.float64)
            errs = [np.linalg.norm(a[0] - Q[0]) / np.linalg.norm(Q[0]),
                    np.linalg.norm(ma - m) / max(np.linalg.norm(m), mscale),
                    np.linalg.norm(a[4] - Q[4]) / np.linalg.norm(Q[4])]
            f16_err.setdefault(req.kind, []).append((float(max(errs)), req))
        return ok

    def batched(storage_override, handler):
        progress.update(leg="batched" if storage_override is None else "batched fp32", done=0)
        with binding.Batch(budget_bytes, max_instances=4096, max_tiles=1 << 22, graph_steps=chunk,
                           stream=stream.cuda_stream) as b:
            srv = serve.Server(b, arena_bytes=budget_bytes, chunk_steps=chunk, result_handler=handler,
                               sync=torch.cuda.synchronize, max_active_cells=max_active_cells,
                               storage_override=storage_override, fp16_kinds=FP16_KINDS,
                               fp16_max_steps=FP16_MAX_STEPS,
                               failure_handler=lambda req: finished(req, False),
                               solo_factory=lambda req, stg: binding.Solver(req.case.params, stream=stream.cuda_stream,
                                                                            storage=stg),
                               solo_min_bytes=SOLO_MIN_BYTES)
            return srv.serve(trace)

    # storage as requested (FP16 for about half the requests), then every request in
    # FP32: the latter's results are bitwise those of the sequential FP32 solves, and
    # each FP16 result is compared with the FP32 result of the same request
    st = batched(None, keep_f16)
    out["batched"] = st.summary()
    out["batched"]["max_active_cells"] = max_active_cells
    out["failures"] = failures
    out["batched_fp32"] = batched(binding.LBM_STORE_F32, compare_f32).summary()
    out["accuracy"] = {
        "bar": "max over rho, rho u, E of the relative L2 against the FP32 result of the same request <= 1e-2 "
               "(rho u against the larger of its norm and rho_ref c_ref sqrt(cells))",
        "batched_fp32_vs_sequential_fp32": "bitwise equal (same kernels and arithmetic per instance)",
        "fp16_vs_fp32_max_rel_l2": {k: {"requests": len(v), "median": float(np.median([e for e, _ in v])),
                                        "max": float(max(e for e, _ in v)),
                                        "above_bar": sum(1 for e, _ in v if e > 1e-2),
                                        "err_and_steps": [[round(e, 6), r.steps] for e, r in v],
                                        "worst": [{"rid": r.rid, "err": e, "shape": list(r.case.shape), "steps": r.steps,
                                                   **{m: r.case.meta[m] for m in ("mach", "left", "right")
                                                      if m in r.case.meta}}
                                                  for e, r in sorted(v, key=lambda t: -t[0])[:3]]}
                                    for k, v in sorted(f16_err.items())},
        "fp16_served_within_bar": bool(all(e <= 1e-2 for v in f16_err.values() for e, _ in v))}

    def fp32_solver(params):
        return binding.Solver(params, stream=stream.cuda_stream)

    progress.update(leg="sequential fp32", done=0)
    st2 = serve.serve_sequential(trace, fp32_solver, result_handler=finite, sync=torch.cuda.synchronize,
                                 failure_handler=lambda req: finished(req, False))
    out["sequential_fp32"] = st2.summary()
    out["speedup_solves_per_s"] = out["batched"]["solves_per_s"] / out["sequential_fp32"]["solves_per_s"]
    out["speedup_fp32_solves_per_s"] = (out["batched_fp32"]["solves_per_s"] /
                                        out["sequential_fp32"]["solves_per_s"])
    return out


def measured_traffic():
    """HBM bytes per launch of the collide-and-stream kernel from the committed
    FETCH_SIZE/WRITE_SIZE counter runs, or None if the kernel sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_step_tgv256_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for p in rec["sources"]:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=256, help="grid edge (default 256)")
    ap.add_argument("--diag-every", type=int, default=50)
    ap.add_argument("--block", type=int, default=None)
    ap.add_argument("--nontemporal", type=int, default=None)
    ap.add_argument("--autotune", type=int, default=0, metavar="STEPS",
                    help="time the launch shapes for STEPS steps each before the run and keep the fastest")
    ap.add_argument("--blocks-per-cu", type=int, default=None,
                    help="even-step occupancy cap in blocks per CU (0 = none; default 4 FP32, none FP16)")
    ap.add_argument("--layout-pad", type=int, default=0)
    ap.add_argument("--odd-lds", type=int, default=1,
                    help="1: odd step shifts the +-x populations in LDS (default); 0: direct")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bw-probe", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched Becker workload")
    ap.add_argument("--batch-only", action="store_true", help="only the batched Becker workload")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--batch-tuning", type=str, default=None, metavar="B,NT,BPC,GRID",
                    help="fixed batch launch shape instead of the autotuner")
    ap.add_argument("--batch-no-seq", action="store_true", help="skip the single-context batch baseline")
    ap.add_argument("--precision-only", action="store_true",
                    help="only the FP16-storage precision study (128^3 vortex)")
    ap.add_argument("--fp16", action="store_true", help="FP16 population storage for the main workload")
    ap.add_argument("--serve-only", action="store_true", help="only the serving mix")
    ap.add_argument("--spectral-only", action="store_true",
                    help="only the fused vs spectral dissipation comparison (cTGV 128^3)")
    ap.add_argument("--mms-only", action="store_true",
                    help="only the manufactured-solution convergence study (64^3-256^3)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving mix")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-rate", type=float, default=50.0,
                    help="mean Poisson arrival rate of the serving mix, requests per second")
    ap.add_argument("--copy-only", type=int, default=0, metavar="BYTES",
                    help="only run the streaming-copy probe on BYTES bytes (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2609_16361_amd import binding, inputs

    binding.load()  # fails loudly if the HIP library has not been built
    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_only:
        gbs = binding.lbm_bw_probe(args.copy_only, 3)
        print(json.dumps({"copy_bytes": args.copy_only, "copy_launches": 4, "copy_gbs": round(gbs, 1)}))
        return
    if args.batch_only:
        tun = None if args.batch_tuning is None else [int(v) for v in args.batch_tuning.split(",")]
        print(json.dumps({"batch": bench_batch(steps=args.batch_steps, stream=stream, tuning=tun,
                                               sequential=not args.batch_no_seq)}), flush=True)
        return
    if args.precision_only:
        print(json.dumps({"precision": bench_precision(stream)}), flush=True)
        return
    if args.spectral_only:
        print(json.dumps({"spectral": bench_spectral(stream)}), flush=True)
        return
    if args.mms_only:
        print(json.dumps({"mms": bench_mms(stream)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serve": bench_serve(stream, count=args.serve_requests, rate=args.serve_rate)}), flush=True)
        return

    case = inputs.tgv(n=args.n, diag_every=args.diag_every)
    cells = case.cells
    storage = binding.LBM_STORE_F16 if args.fp16 else binding.LBM_STORE_F32
    bytes_per_lup = BYTES_PER_LUP_F32 / 2 if args.fp16 else BYTES_PER_LUP_F32
    solver = binding.Solver(case.params, stream=stream.cuda_stream, block=args.block,
                            nontemporal=None if args.nontemporal is None else bool(args.nontemporal),
                            layout_pad=args.layout_pad, storage=storage, odd_lds=bool(args.odd_lds),
                            blocks_per_cu=args.blocks_per_cu)
    solver.init(case.Q0)
    del case.Q0

    solver.step(args.warmup, args.diag_every)
    torch.cuda.synchronize()
    solver.diagnostics()
    tuned = None
    if args.autotune:
        best, best_us, tried = solver.autotune(trial_steps=args.autotune)
        tuned = {"us_per_step": round(best_us, 2), "candidates": len(tried)}
    launch = solver.launch()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_host = time.perf_counter()
    ev0.record(stream)
    solver.step(args.steps, args.diag_every)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    ms = ev0.elapsed_time(ev1)

    recs, status = solver.diagnostics()
    assert status == binding.LBM_OK and all(r["nonfinite"] == 0 for r in recs), "state diverged"
    solver.close()
    if tuned is not None:
        launch["autotuned"] = tuned

    glups = cells * args.steps / (ms * 1e-3) / 1e9
    # lbm_step reduces the diagnostics on the steps t with t % diag_every == 0
    diag_timed = (sum(1 for t in range(args.warmup, args.warmup + args.steps) if t % args.diag_every == 0)
                  if args.diag_every > 0 else 0)
    avg_launch_ms = ms / args.steps
    achieved_gbs = bytes_per_lup * cells / (avg_launch_ms * 1e-3) / 1e9

    bw = None
    if not args.no_bw_probe:
        bw = binding.lbm_bw_probe(2 * 1024 ** 3, 10)

    out = {
        "metric": "GLUP/s + % HBM roofline (256^3 TGV fp32); batched solves/s, p99 latency",
        "value": round(glups, 4),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if not args.fp16 else "f32 arithmetic, f16 storage",
        "data": "synthetic (analytic compressible Taylor-Green initial field)",
        "config": {"workload": f"compressible Taylor-Green vortex {args.n}^3 periodic "
                               f"{'FP16-storage' if args.fp16 else 'FP32'}, Mach 1.25, "
                               f"Re 1600, regularized collision + sensor, diagnostics every "
                               f"{args.diag_every} steps ({diag_timed} of the {args.steps} timed steps)",
                   "cells": cells, "steps": args.steps, "diag_every": args.diag_every,
                   "diag_steps_timed": diag_timed,
                   **launch,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                     "traffic": None if args.fp16 or args.n != 256 else measured_traffic(),
                     "traffic_unit": "bytes per launch",
                     "bytes_per_lup": bytes_per_lup, "avg_launch_ms": round(avg_launch_ms, 5)},
        "host_wall_s": round(t_host, 3),
        "copy_bw_gbs": None if bw is None else round(bw, 1),
        "frac_of_copy_bw": None if bw is None else round(achieved_gbs / bw, 4),
        "diag_records": len(recs),
        "Ek_last": recs[-1]["Ek"] / cells if recs else None,
    }
    if not args.no_batch:
        out["batch"] = bench_batch(stream=stream)
    if not args.no_serve:
        out["serve"] = bench_serve(stream, count=args.serve_requests, rate=args.serve_rate)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
