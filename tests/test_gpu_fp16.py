"""FP16 population storage (shifted by w_i Q_ref and scaled per field by a power
of two) with FP32 moments, reconstruction and collision, against the FP64 oracle.

Tolerance: each stored value is rounded stochastically to FP16 (after the exact
power-of-two scaling), so a store errs by less than one FP16 ulp, a relative
2^-10 = 9.8e-4 of the field's largest shifted population, with zero mean; a
handful of steps therefore stays within a few such ulps per step, and the
conserved fields after 100 smooth steps within about 1e-3 relative L2.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2609_16361_amd import binding, inputs

pytestmark = pytest.mark.gpu
F16 = binding.LBM_STORE_F16
W = np.array([0.25] + [0.125] * 6)


def say(msg):
    print(msg, flush=True)


def shift(params):
    qref = np.array([params["rho_ref"], 0, 0, 0, params["E_ref"]])
    return (qref[:, None] * W[None, :]).reshape(35)


@pytest.mark.parametrize("dims,bc", [((4, 4, 4), (0, 0, 0)), ((70, 3, 2), (1, 0, 0)),
                                     ((6, 2, 3), (1, 1, 1)), ((1, 1, 1), (0, 0, 0))])
def test_fp16_tiny_grids(dims, bc):
    case = inputs.random_smooth(*dims, seed=sum(dims), amp=0.08, mach=1.2, bc=bc, J_min=1e-3,
                                sensor_gain=20.0, omega_min=1.0)
    sh = shift(case.params)
    f_or = oracle.init(case.params, case.Q0)
    for steps in (1, 2, 3):
        say(f"fp16 tiny {dims} steps={steps}")
        f_or, _ = oracle.run(case.params, f_or, 1)
        with binding.Solver(case.params, storage=F16) as s:
            s.init(case.Q0)
            s.step(steps)
            f16, _ = s.populations()
        g_gpu = f16.reshape(35, -1).astype(np.float64)
        g_ora = f_or - sh[:, None]
        for k in range(5):
            sl = slice(7 * k, 7 * k + 7)
            err = np.abs(g_gpu[sl] - g_ora[sl]).max() / np.abs(g_ora[sl]).max()
            say(f"   field {k}: {err:.2e}")
            assert err <= 4 * 2.0 ** -10 * steps, (dims, steps, k, err)


def test_fp16_vortex_100_steps():
    case = inputs.tgv(n=32, steps=100)
    say("fp16 tgv 32^3 100 steps")
    with binding.Solver(case.params, storage=F16) as s:
        s.init(case.Q0)
        s.step(100)
        Q16 = s.moments()
    with binding.Solver(case.params) as s:
        s.init(case.Q0)
        s.step(100)
        Q32 = s.moments()
    f, _ = oracle.run(case.params, oracle.init(case.params, case.Q0), 100)
    Qo = oracle.moments(case.params, f)
    N = case.cells
    c_ref = math.sqrt(1.4 * 0.4 * case.params["E_ref"] / case.params["rho_ref"])
    for k in range(5):
        scale = max(np.linalg.norm(Qo[k]), case.params["rho_ref"] * c_ref * math.sqrt(N))
        e16 = np.linalg.norm(Q16[k] - Qo[k]) / scale
        e32 = np.linalg.norm(Q32[k] - Qo[k]) / scale
        say(f"   field {k}: fp16 {e16:.2e} fp32 {e32:.2e}")
        assert e16 <= 1e-3, (k, e16)


def test_fp16_stochastic_rounding_is_unbiased():
    """FP16 stores round stochastically with zero mean.  In a uniform state at rest
    every cell computes the same post-collision value of each slot, and the dither
    of its cell and slot rounds it to one of the two FP16 neighbours; the share of
    cells rounded up then places the value between them.  The value itself comes
    from the FP64 oracle stepping the state the GPU holds after its start (read
    back, so the start's own rounding is in it).  Bar: 5 standard errors of the
    share (sqrt(p (1 - p) / N) of the FP16 spacing) plus 1e-3 of the spacing for
    the FP32 arithmetic.  At rest the density and energy slots come back exactly
    as stored; the six momentum slots that carry the pressure round, each over
    262144 cells.  A biased or non-uniform dither fails it (a first 24-bit dither
    that took the multiply's sign into the shift turned a vortex non-finite in
    one step)."""
    n = 64
    p = inputs.tgv(n=n, steps=1).params
    Q0 = np.zeros((5, n, n, n))
    Q0[0] = p["rho_ref"] * 1.0123457
    Q0[4] = p["E_ref"] * 1.0234567
    sh = shift(p)
    with binding.Solver(p, storage=F16) as s:
        s.init(Q0)
        g0, st0 = s.populations()
        s.step(1)
        g1, st1 = s.populations()
    assert st0 == 0 and st1 == 1
    g0 = g0.reshape(35, -1).astype(np.float64)
    g1 = g1.reshape(35, -1).astype(np.float64)
    N = g1.shape[1]
    assert np.all(g0 == g0[:, :1])          # the start is uniform as well
    one = dict(p, nx=1, ny=1, nz=1)         # one periodic cell holds the uniform state
    f, _ = oracle.run(one, g0[:, :1] + sh[:, None], 1)
    exact = f[:, 0] - sh
    rounded = 0
    for i in range(35):
        vals = np.unique(g1[i])
        assert len(vals) <= 2, (i, vals)
        if len(vals) == 1:
            # exactly representable (zero, for instance): no rounding at all
            scale = np.abs(exact[7 * (i // 7):7 * (i // 7) + 7]).max()
            assert abs(vals[0] - exact[i]) <= 1e-6 * scale, (i, vals, exact[i])
            continue
        a, b = vals
        assert a < exact[i] < b, (i, a, exact[i], b)
        share = np.mean(g1[i] == b)
        est = a + share * (b - a)
        tol = (5.0 * np.sqrt(max(share * (1 - share), 1e-12) / N) + 1e-3) * (b - a)
        say(f"   slot {i}: exact at {(exact[i] - a) / (b - a):.4f} of the spacing, rounded up {share:.4f}")
        assert abs(est - exact[i]) <= tol, (i, est, exact[i], tol)
        rounded += 1
    assert rounded >= 6


def test_fp16_checkpoint_roundtrip():
    case = inputs.random_smooth(20, 6, 5, seed=3, amp=0.06, bc=(1, 0, 0))
    with binding.Solver(case.params, storage=F16) as s:
        s.init(case.Q0)
        s.step(5)
        fa, st = s.populations()
        s.set_populations(fa, st)
        fb, _ = s.populations()
        assert np.array_equal(fa, fb)
        s.step(4)
        f1, _ = s.populations()
    with binding.Solver(case.params, storage=F16) as s2:
        s2.set_populations(fa, 5)
        s2.step(4)
        f2, _ = s2.populations()
    assert np.array_equal(f1, f2)


def test_precision_workload_against_oracle():
    """The FP16 precision workload (cTGV 128^3, f_mu 0.9) over its first 100 steps:
    the E_k / eps_s / eps_d series (every 10 steps) and the conserved fields of FP32
    and FP16 storage against the FP64 oracle.  Bars: FP32 at its smooth-data level;
    FP16 a few times the relative FP16 step 2^-11 (and ~10x the measured values).
    Over these steps the dilatational dissipation is about 1e-4 of the solenoidal
    one, below what FP16 populations resolve on their own scale (measured 12%), so
    its FP16 bar is taken against the total dissipation eps_s + eps_d."""
    case = inputs.tgv(n=128, steps=100, diag_every=10)
    out = {}
    for name, stg in (("f32", binding.LBM_STORE_F32), ("f16", F16)):
        say(f"precision workload 128^3 {name}")
        with binding.Solver(case.params, storage=stg) as s:
            s.init(case.Q0)
            s.step(100, 10)
            recs, st = s.diagnostics()
            assert st == binding.LBM_OK
            out[name] = (np.array([[r["Ek"], r["eps_s"], r["eps_d"]] for r in recs]), s.moments())
    say("precision workload 128^3 oracle")
    f, d = oracle.run(case.params, oracle.init(case.params, case.Q0), 100, 10)
    Qo = oracle.moments(case.params, f)
    so = d[:, :3]
    bars = {"f32": ((1e-6, 1e-4, 1e-4), 2e-5), "f16": ((1e-3, 3e-2, 2e-3), 1e-2)}
    total = np.linalg.norm(so[1:, 1] + so[1:, 2])
    say(f"   oracle eps_d / eps_s over the series: {np.linalg.norm(so[1:, 2]) / np.linalg.norm(so[1:, 1]):.2e}")
    for name, (ser, Q) in out.items():
        for i, q in enumerate(("Ek", "eps_s", "eps_d")):
            d_ = np.linalg.norm(ser[1:, i] - so[1:, i])
            e = d_ / np.linalg.norm(so[1:, i])
            say(f"   {name} {q} series vs oracle {e:.2e} (of the total dissipation {d_ / total:.2e})")
            if name == "f16" and q == "eps_d":
                e = d_ / total
            assert e <= bars[name][0][i], (name, q, e)
        for k in range(5):
            e = np.linalg.norm(Q[k] - Qo[k]) / np.linalg.norm(Qo[k])
            say(f"   {name} field {k} vs oracle {e:.2e}")
            assert e <= bars[name][1], (name, k, e)


def test_precision_workload_full_run_against_oracle_series():
    """The precision workload over its whole run (cTGV 128^3, 4000 steps, records
    every 50) against the FP64 oracle's series of the same run, stored in
    tests/golden/tgv128_oracle_series.json by make_tgv128_oracle_series.py (which
    calls only the oracle).  Relative L2 over the series, per quantity, from the
    second record on (the first is the same initial state on both sides).  Bars:
    FP32 storage 1e-5 (E_k) and 1e-4 (the dissipation rates), the FP32 rounding
    of 4000 steps with room; FP16 storage the 1e-2 accuracy stated for FP16 on the
    rates and 1e-4 on E_k, a volume sum in which the zero-mean rounding errors of
    the 2 M cells average out.  By t_c = 5.45 the dilatational rate has grown to a
    tenth of the solenoidal one, so here it is measured against itself."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tgv128_oracle_series.json")))
    case = inputs.tgv(n=128, steps=4000, diag_every=50)
    assert gold["cells"] == case.cells and gold["r"] == case.meta["r"] and gold["omega"] == case.params["omega"][0]
    o = np.stack([np.array(gold[q]) for q in ("Ek", "eps_s", "eps_d")], axis=1)
    bars = {"f32": (1e-5, 1e-4, 1e-4), "f16": (1e-4, 1e-2, 1e-2)}
    for name, stg in (("f32", binding.LBM_STORE_F32), ("f16", F16)):
        say(f"precision workload 128^3 {name}, 4000 steps")
        with binding.Solver(case.params, storage=stg) as s:
            s.init(case.Q0)
            s.step(4000, 50)
            recs, st = s.diagnostics()
            assert st == binding.LBM_OK
        ser = np.array([[r["Ek"], r["eps_s"], r["eps_d"]] for r in recs]) / case.cells
        assert ser.shape == o.shape
        for i, q in enumerate(("Ek", "eps_s", "eps_d")):
            e = np.linalg.norm(ser[1:, i] - o[1:, i]) / np.linalg.norm(o[1:, i])
            say(f"   {name} {q} series vs oracle over 4000 steps {e:.2e}")
            assert e <= bars[name][i], (name, q, e)


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 1)])
def test_even_step_cell_pairs_bitwise(bc):
    """From 2^23 cells on, FP16 even steps with blocks of up to 256 threads take two
    consecutive cells per lane (4-byte accesses); 512-thread blocks take one.  Both
    give the same bits, diagnostics to FP32 summation order."""
    case = inputs.random_smooth(256, 256, 128, seed=21, amp=0.05, bc=bc)
    out = []
    for block in (256, 512):
        say(f"FP16 256x256x128 bc={bc} block={block}")
        with binding.Solver(case.params, storage=binding.LBM_STORE_F16, block=block) as s:
            s.init(case.Q0)
            s.step(4, 2)
            f, st = s.populations()
            recs, status = s.diagnostics()
        out.append((f, recs, status))
    (fa, ra, sa), (fb, rb, sb) = out
    assert sa == sb == binding.LBM_OK
    assert np.array_equal(fa, fb)
    for a, b in zip(ra, rb):
        assert a["Ek"] == pytest.approx(b["Ek"], rel=1e-5)


@pytest.mark.parametrize("dims,bc,coll", [((384, 192, 128), (0, 1, 1), inputs.RLB_SENSOR),
                                          ((512, 128, 128), (1, 1, 0), inputs.BGK),
                                          ((512, 256, 64), (1, 0, 1), inputs.RLB_SENSOR),
                                          ((1024, 64, 128), (1, 0, 1), inputs.RLB_SENSOR)])
def test_odd_step_row_pairs_bitwise(dims, bc, coll):
    """From 2^23 cells on, FP16 odd steps on rows of 384 or 512 cells take two
    consecutive cells per lane, one row per block; the direct odd step (one cell per
    lane, no LDS) gives the same bits, diagnostics to FP32 summation order.  (The
    1024-cell rows take the one-cell LDS odd step.)"""
    case = inputs.random_smooth(*dims, seed=sum(dims) + sum(bc), amp=0.05, bc=bc, collision=coll)
    out = []
    for staged in (True, False):
        say(f"FP16 {dims} bc={bc} coll={coll} odd_lds={staged}")
        with binding.Solver(case.params, storage=binding.LBM_STORE_F16, odd_lds=staged) as s:
            s.init(case.Q0)
            s.step(5, 2)
            f, st = s.populations()
            recs, status = s.diagnostics()
        out.append((f, recs, status))
    (fa, ra, sa), (fb, rb, sb) = out
    assert sa == sb == binding.LBM_OK and len(ra) == len(rb) == 3  # steps 0, 2, 4
    assert np.array_equal(fa, fb)
    for a, b in zip(ra, rb):
        for key in ("Ek", "eps_s", "eps_d"):
            assert a[key] == pytest.approx(b[key], rel=1e-5, abs=1e-30), key


def test_fp16_scale_headroom_for_a_growing_field():
    """A Sod tube with nearly equal densities (ratio 1.025) and a pressure ratio of
    90: the density populations start tiny, so the density field takes a large
    FP16 scale, and the shock raises them more than 160-fold by step 1000 (FP64
    oracle).  The scale leaves 1024x headroom below the FP16 maximum (64x overflowed
    at step 200), so the FP16 run stays finite and within the FP16 shock-tube bar
    of the serving tests (1e-2 relative L2) of FP32."""
    case = inputs.sod_variant(3061, 1.0247, 90.23)
    out = {}
    for stg in (binding.LBM_STORE_F32, binding.LBM_STORE_F16):
        say(f"Sod 3061x4x4 rho ratio 1.0247 p ratio 90.23 storage {stg}, 2000 steps")
        with binding.Solver(case.params, storage=stg) as s:
            s.init(case.Q0)
            s.step(2000)
            out[stg] = s.moments()
    Q32, Q16 = out[binding.LBM_STORE_F32], out[binding.LBM_STORE_F16]
    assert np.isfinite(Q32).all() and np.isfinite(Q16).all()
    for k in (0, 1, 4):
        e = np.linalg.norm(Q16[k] - Q32[k]) / np.linalg.norm(Q32[k])
        say(f"   field {k}: FP16 vs FP32 {e:.2e}")
        assert e <= 1e-2, (k, e)
