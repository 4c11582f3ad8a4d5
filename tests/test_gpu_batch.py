"""GPU tests of the batched path (lbm_batch_*): uneven instances stepped by one
kernel launch over a tile work-list, time loops replayed from a captured graph.

The bar is bitwise: an instance inside a batch must end exactly where the same
instance run alone in a context (lbm_create/lbm_step) ends, whatever the other
instances, its admission time, the graph length or the tuned launch shape; the
single-context path is itself checked against the oracle in test_gpu_parity.py.
A Becker mix is also checked directly against the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2609_16361_amd import binding, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def alone(case, steps, storage=None):
    with binding.Solver(case.params, storage=storage) as s:
        s.init(case.Q0)
        s.step(steps)
        f, st = s.populations()
    assert st == steps
    return f


def mix():
    """Uneven instances: sizes, both boundary kinds, both collisions, FP32 and FP16."""
    cases = [
        (inputs.random_smooth(300, 3, 2, seed=1, amp=0.06, bc=(1, 0, 0)), None),
        (inputs.random_smooth(17, 9, 5, seed=2, amp=0.05), None),
        (inputs.random_smooth(64, 4, 4, seed=3, amp=0.05, collision=inputs.BGK), None),
        (inputs.becker(L=200, mach=2.5, ny=4, nz=4), None),
        (inputs.random_smooth(33, 7, 3, seed=4, amp=0.05, bc=(1, 1, 0)), binding.LBM_STORE_F16),
        (inputs.sod(n=128, ny=2, nz=3), None),
    ]
    return cases


# launch shapes: (block, nontemporal, blocks_per_cu, grid); None keeps the default.
# grid 0 is one block per tile: the 36864-cell instance takes its group past 256
# tiles of 128 cells and back, so the rounded grid changes and the graph is
# captured again on the way.
SHAPES = [(1, None), (16, None), (16, (512, 1, 0, 0)), (16, (128, 0, 0, 0)), (1, (128, 1, 0, 0)),
          (16, (256, 0, 4, 7)), (16, (256, 1, 4, 0))]


@pytest.mark.parametrize("graph_steps,shape", SHAPES)
def test_batch_equals_single_contexts_bitwise(graph_steps, shape):
    # the last two hold 2^20 cells or more (thousands of tiles each, beside
    # instances of a few tiles)
    cases = mix() + [(inputs.random_smooth(48, 32, 24, seed=5, amp=0.05), None),
                     (inputs.random_smooth(40, 6, 5, seed=6, amp=0.05, collision=inputs.BGK, bc=(0, 1, 0)),
                      binding.LBM_STORE_F16),
                     (inputs.random_smooth(128, 96, 86, seed=7, amp=0.05), None),
                     (inputs.random_smooth(96, 110, 100, seed=8, amp=0.05, bc=(1, 0, 1)), binding.LBM_STORE_F16)]
    assert all(c.cells >= 1 << 20 for c, _ in cases[-2:]) and all(c.cells < 1 << 20 for c, _ in cases[:-2])
    steps = [37, 20, 41, 25, 30, 18, 12, 27, 15, 22]
    admit = [0, 0, 5, 9, 9, 23, 9, 2, 9, 0]    # clock at which each instance joins
    with binding.Batch(1 << 29, graph_steps=graph_steps) as b:
        if shape is not None:
            b.set_tuning(*shape)
            assert b.info()["tuning"] == dict(zip(("block", "nontemporal", "blocks_per_cu", "grid"), shape))
        ids = {}
        clock = 0
        for t_admit in sorted(set(admit)):
            if t_admit > clock:
                say(f"batch run {t_admit - clock} steps (graph {graph_steps})")
                b.run(t_admit - clock)
                clock = t_admit
            for k, (c, stg) in enumerate(cases):
                if admit[k] == t_admit:
                    ids[k] = b.add(c.params, c.Q0, steps[k], storage=stg)
        say("batch run to the end")
        b.run(max(a + s for a, s in zip(admit, steps)) - clock + 3)
        for k, (c, stg) in enumerate(cases):
            done, fin = b.query(ids[k])
            assert fin and done == steps[k]
            fb, st = b.populations(ids[k])
            assert st == steps[k]
            say(f"compare instance {k}")
            fa = alone(c, steps[k], storage=stg)
            assert np.array_equal(fa, fb), k
            Qb = b.moments(ids[k])
            with binding.Solver(c.params, storage=stg) as s:
                s.init(c.Q0)
                s.step(steps[k])
                assert np.array_equal(s.moments(), Qb)


def test_batch_degenerate_instances_bitwise():
    """A single periodic cell (its own neighbour on every axis) and one-cell rows
    beside an ordinary instance, in FP32 and FP16: each ends bitwise where it ends
    alone."""
    cases = [(inputs.random_smooth(1, 1, 1, seed=11, amp=0.05), None),
             (inputs.random_smooth(1, 4, 3, seed=12, amp=0.05), binding.LBM_STORE_F16),
             (inputs.random_smooth(1, 5, 2, seed=13, amp=0.05, bc=(0, 1, 1)), None),
             (inputs.random_smooth(24, 6, 5, seed=14, amp=0.05), None)]
    steps = [9, 14, 11, 7]
    with binding.Batch(1 << 26, graph_steps=4) as b:
        ids = [b.add(c.params, c.Q0, n, storage=stg) for (c, stg), n in zip(cases, steps)]
        b.run(max(steps) + 2)
        for k, ((c, stg), n) in enumerate(zip(cases, steps)):
            fb, st = b.populations(ids[k])
            assert st == n
            say(f"compare degenerate instance {k} {c.shape}")
            assert np.array_equal(alone(c, n, storage=stg), fb), k


def test_batch_autotune_keeps_state():
    cases = mix()[:4]
    with binding.Batch(1 << 26, graph_steps=8) as b:
        ids = [b.add(c.params, c.Q0, 40) for c, _ in cases]
        b.run(6)
        say("autotune")
        best, us, tried = b.autotune(trial_steps=8)
        assert len(tried) >= 8 and us > 0
        assert b.info()["tuning"] == best
        assert b.info()["clock"] == 6
        b.run(40)
        for i, (c, _) in zip(ids, cases):
            fb, st = b.populations(i)
            assert st == 40
            assert np.array_equal(fb, alone(c, 40)), i


def test_batch_remove_and_reuse():
    c1 = inputs.random_smooth(40, 5, 4, seed=8, amp=0.05)
    c2 = inputs.random_smooth(30, 6, 4, seed=9, amp=0.05, bc=(0, 1, 0))
    c3 = inputs.random_smooth(20, 5, 4, seed=10, amp=0.05)
    p1 = binding.make_params(c1.params)
    arena = binding.lbm_state_bytes(p1) * 2 + (1 << 20)
    with binding.Batch(arena, max_instances=2) as b:
        i1 = b.add(c1.params, c1.Q0, 10)
        i2 = b.add(c2.params, c2.Q0, 25)
        with pytest.raises(binding.LbmError) as e:
            b.add(c3.params, c3.Q0, 5)          # descriptor table full
        assert e.value.status == binding.LBM_ENOMEM
        b.run(12)
        assert b.query(i1) == (10, True) and b.query(i2) == (12, False)
        b.remove(i1)
        i3 = b.add(c3.params, c3.Q0, 9)          # reuses the freed slot and arena run
        b.run(13)
        assert b.query(i2) == (25, True) and b.query(i3) == (9, True)
        assert np.array_equal(b.populations(i2)[0], alone(c2, 25))
        assert np.array_equal(b.populations(i3)[0], alone(c3, 9))
        with pytest.raises(binding.LbmError):
            b.query(i1 + 7)
        info = b.info()
        assert info["live_instances"] == 2 and info["active_instances"] == 0


def test_batch_nonfinite_flags_diverged_instances():
    """lbm_batch_nonfinite reports exactly the instances whose stored rest
    populations (slot 0 of each field) are not all finite: a Mach 1.25 vortex on
    16^3 run at 0.5 cells per step near omega = 2 (the FP64 oracle's state stops
    being finite at step 30), in FP32 and FP16 storage, next to smooth states that
    stay finite."""
    bad = inputs.tgv(n=16, mach=1.25, cfl=0.5, steps=60, diag_every=0)
    g0 = inputs.random_smooth(40, 5, 4, seed=8, amp=0.05)
    g1 = inputs.random_smooth(30, 6, 4, seed=9, amp=0.05, bc=(0, 1, 0))
    with binding.Batch(1 << 28) as b:
        ids = {"bad32": b.add(bad.params, bad.Q0, 60),
               "good32": b.add(g0.params, g0.Q0, 60),
               "bad16": b.add(bad.params, bad.Q0, 60, storage=binding.LBM_STORE_F16),
               "good16": b.add(g1.params, g1.Q0, 60, storage=binding.LBM_STORE_F16)}

        def expected():
            return sorted(i for i in ids.values()
                          if not np.isfinite(b.populations(i)[0][[0, 7, 14, 21, 28]]).all())

        assert b.nonfinite() == expected()
        b.run(60)
        flagged = b.nonfinite()
        say(f"flagged after 60 steps: {[k for k, i in ids.items() if i in flagged]}")
        assert flagged == expected()
        assert ids["bad32"] in flagged
        assert ids["good32"] not in flagged and ids["good16"] not in flagged
        b.remove(ids["bad32"])
        assert ids["bad32"] not in b.nonfinite()


def test_batch_arena_full():
    c = inputs.random_smooth(64, 8, 8, seed=1)
    need = binding.lbm_state_bytes(binding.make_params(c.params))
    with binding.Batch(need + need // 2) as b:
        b.add(c.params, c.Q0, 3)
        with pytest.raises(binding.LbmError) as e:
            b.add(c.params, c.Q0, 3)
        assert e.value.status == binding.LBM_ENOMEM


def test_becker_mix_against_oracle():
    """Small Becker tubes of the batched workload's kind (zero-gradient ends,
    regularized collision with sensor, Pr = 3/4) against the FP64 oracle."""
    cases = [inputs.becker(L=L, mach=m, ny=4, nz=4) for L, m in ((96, 1.5), (160, 3.0), (128, 5.0))]
    with binding.Batch(1 << 26, graph_steps=16) as b:
        ids = [b.add(c.params, c.Q0, 300) for c in cases]
        b.run(300)
        for i, c in zip(ids, cases):
            say(f"becker L={c.params['nx']} vs oracle")
            Q = b.moments(i)
            f, _ = oracle.run(c.params, oracle.init(c.params, c.Q0), 300)
            Qo = oracle.moments(c.params, f)
            for k in (0, 1, 4):
                e = np.linalg.norm(Q[k] - Qo[k]) / np.linalg.norm(Qo[k])
                assert e <= 2e-5, (c.params["nx"], k, e)


def test_full_becker_batch_sampled_against_oracle():
    """The batched workload at its full size and in the launch configuration the
    benchmark times: all 64 seeded tubes (4.5 M cells) in one batch, graphs of 50
    steps, autotuned shape, 5000 steps.  Three instances (the shortest, and two near
    the top of the Mach range) are checked against the FP64 oracle: uniform across
    the tube, relative L2 <= 1e-3 in shocked cells (oracle sensor active at the end,
    dilated by 4 cells) and over the tube for rho, rho u_x and E."""
    cases = inputs.becker_batch(64, seed=0)
    steps = 5000
    nbytes = sum(binding.lbm_state_bytes(binding.make_params(c.params)) for c in cases)
    sample = (23, 41, 6)
    with binding.Batch(int(nbytes * 1.05) + (64 << 20), max_instances=64, graph_steps=50) as b:
        ids = [b.add(c.params, c.Q0, steps) for c in cases]
        say("autotune the full Becker batch")
        b.autotune(trial_steps=50)
        say("run 5000 steps")
        b.run(steps)
        Qs = {j: b.moments(ids[j]) for j in sample}
    for j in sample:
        c = cases[j]
        nx = c.params["nx"]
        Q = Qs[j]
        say(f"becker instance {j}: L={nx} M={c.meta['mach']:.2f} vs oracle, {steps} steps")
        assert np.array_equal(Q, np.broadcast_to(Q[:, :1, :1, :], Q.shape))
        f, _ = oracle.run(c.params, oracle.init(c.params, c.Q0), steps)
        Qo = oracle.moments(c.params, f)
        fo = f.reshape(35, 4, 4, nx)[:, 0, 0, :]
        chi = np.array([oracle.collide(c.params, fo[:, x])[1]["chi"] for x in range(nx)])
        mask = np.convolve((chi > 0).astype(float), np.ones(9), mode="same") > 0
        for k in (0, 1, 4):
            e_all = np.linalg.norm(Q[k] - Qo[k]) / np.linalg.norm(Qo[k])
            e_sh = (np.linalg.norm(Q[k][..., mask] - Qo[k][..., mask]) / np.linalg.norm(Qo[k][..., mask])
                    if mask.any() else 0.0)
            say(f"   field {k}: overall {e_all:.2e} shocked {e_sh:.2e} ({int(mask.sum())} cells)")
            assert e_all <= 1e-3 and e_sh <= 1e-3, (j, k, e_all, e_sh)
