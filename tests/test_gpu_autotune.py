"""lbm_autotune on a single context: it times launch shapes on the live state and
must leave that state bitwise as it found it (populations and step count), so a
run with an autotune in the middle ends exactly where the same run without one
ends.  Results never depend on the launch shape, so the tuned shape changes
nothing but the speed."""
import numpy as np
import pytest

from paper_2609_16361_amd import binding, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("storage", [None, binding.LBM_STORE_F16])
def test_autotune_keeps_state_and_results(storage):
    case = inputs.random_smooth(80, 24, 12, seed=7, amp=0.05, bc=(1, 0, 0))
    with binding.Solver(case.params, storage=storage) as ref:
        ref.init(case.Q0)
        ref.step(31, 10)
        f_ref, st_ref = ref.populations()
        rec_ref, _ = ref.diagnostics()
    with binding.Solver(case.params, storage=storage) as s:
        s.init(case.Q0)
        s.step(13, 10)                      # odd step count: autotune starts mid-pair
        say(f"autotune storage={storage}")
        best, us, tried = s.autotune(trial_steps=6)
        assert len(tried) == 12 and us > 0
        assert s.launch() == best
        assert min(t for _, t in tried) == us
        f_mid, st_mid = s.populations()
        assert st_mid == 13
        s.step(18, 10)
        f, st = s.populations()
        rec, _ = s.diagnostics()
    assert st == st_ref == 31
    assert np.array_equal(f, f_ref)
    # the diagnostics are block-wise reductions, so their rounding follows the
    # block count of the launch shape: steps exact, values to FP32 summation error
    assert [r["step"] for r in rec] == [r["step"] for r in rec_ref] == [0, 10, 20, 30]
    for a, b in zip(rec, rec_ref):
        for k in ("Ek", "eps_s", "eps_d"):
            assert a[k] == pytest.approx(b[k], rel=1e-5, abs=1e-12)
        assert a["nonfinite"] == b["nonfinite"] == 0


def test_default_launch_shapes():
    case = inputs.random_smooth(16, 8, 4, seed=1)
    with binding.Solver(case.params) as s:
        assert s.launch() == dict(block=256, nontemporal=1, blocks_per_cu=4, odd_lds=1)
    with binding.Solver(case.params, storage=binding.LBM_STORE_F16) as s:
        assert s.launch() == dict(block=256, nontemporal=1, blocks_per_cu=0, odd_lds=1)
    with binding.Batch(1 << 24) as b:
        assert b.info()["tuning"] == dict(block=256, nontemporal=0, blocks_per_cu=2, grid=0)
    # states of 24 MB up to 320 MB default to plain access; smaller and larger ones
    # to nontemporal access
    F16 = binding.LBM_STORE_F16
    for dims, stg, nt in (((96, 96, 96), None, 0), ((136, 136, 136), None, 1), ((128, 128, 128), F16, 0),
                          ((48, 48, 48), F16, 1), ((256, 256, 256), None, 1)):
        p = dict(case.params, nx=dims[0], ny=dims[1], nz=dims[2])
        with binding.Solver(p, storage=stg) as s:
            assert s.launch()["nontemporal"] == nt, (dims, stg)
        # a partial override keeps the grid's default for the rest
        with binding.Solver(p, storage=stg, block=512) as s:
            assert s.launch()["nontemporal"] == nt and s.launch()["block"] == 512, (dims, stg)


def test_autotune_before_init_is_an_error():
    case = inputs.random_smooth(16, 8, 4, seed=1)
    with binding.Solver(case.params) as s:
        with pytest.raises(binding.LbmError) as e:
            s.autotune()
        assert e.value.status == binding.LBM_ESTATE
