"""lbm_step_noalloc (no device allocation, fixed scratch for the diagnostic
partials) against lbm_step on a context over the same state: the same kernels and
launch shape, so populations and diagnostic records must agree bit for bit.  Two
calls in a row share the scratch array; the second runs a smaller grid."""
import numpy as np
import pytest
import torch

from paper_2609_16361_amd import binding, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def compare(case, warm, n, diag_every):
    """Bring a context to `warm` completed steps, copy its buffer, advance the
    context by lbm_step and the copy by lbm_step_noalloc, compare both."""
    prm = binding.make_params(case.params)
    nbytes = binding.lbm_state_bytes(prm)
    stream = torch.cuda.current_stream()
    A = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    B = torch.empty_like(A)
    ctx = binding.lbm_create_in(prm, A.data_ptr(), nbytes, stream.cuda_stream)
    try:
        binding.lbm_init_fields(ctx, case.Q0)
        binding.lbm_step(ctx, warm)
        torch.cuda.synchronize()
        B.copy_(A)
        binding.lbm_step(ctx, n, diag_every)
        recs, st = binding.lbm_diagnostics(ctx)
        assert st == binding.LBM_OK
        torch.cuda.synchronize()
    finally:
        binding.lbm_destroy(ctx)
    R = torch.full((max(len(recs), 1) * 9,), float("nan"), dtype=torch.float32, device="cuda")
    binding.lbm_step_noalloc(prm, B.data_ptr(), warm, n, diag_every, R.data_ptr(), len(recs),
                             stream.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(A.view(torch.int32), B.view(torch.int32))
    R = R.cpu().numpy()
    assert len(recs) == (sum(1 for t in range(warm, warm + n) if t % diag_every == 0) if diag_every else 0)
    for i, r in enumerate(recs):
        v = R[9 * i: 9 * i + 9]
        assert float(v[0]) == r["Ek"] and float(v[1]) == r["eps_s"] and float(v[2]) == r["eps_d"], (i, v, r)
        assert [float(x) for x in v[3:8]] == r["dtotal"], (i, v, r)
        assert int(round(float(v[8]))) == r["nonfinite"] == 0
    return prm, B


def test_noalloc_matches_lbm_step_two_calls():
    say("noalloc: 48x20x12 zero-gradient x, 3 + 9 steps, diagnostics every 4")
    big = inputs.random_smooth(48, 20, 12, seed=21, amp=0.07, mach=1.2, bc=(1, 0, 0))
    compare(big, 3, 9, 4)
    say("noalloc: 20x9x6 periodic, 0 + 6 steps, diagnostics every 2 (smaller, same scratch)")
    small = inputs.random_smooth(20, 9, 6, seed=22, amp=0.06)
    compare(small, 0, 6, 2)
    say("noalloc: 20x9x6 BGK, 1 + 5 steps, no diagnostics")
    bgk = inputs.random_smooth(20, 9, 6, seed=23, amp=0.06, collision=inputs.BGK)
    compare(bgk, 1, 5, 0)


def test_noalloc_rejects_what_it_cannot_do():
    case = inputs.random_smooth(16, 8, 4, seed=24)
    prm = binding.make_params(case.params)
    nbytes = binding.lbm_state_bytes(prm)
    A = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    R = torch.zeros(9, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    with pytest.raises(binding.LbmError) as e:   # two records, room for one
        binding.lbm_step_noalloc(prm, A.data_ptr(), 0, 4, 2, R.data_ptr(), 1, s)
    assert e.value.status == binding.LBM_EINVAL
    with pytest.raises(binding.LbmError) as e:   # FP16 storage
        binding.lbm_step_noalloc(binding.make_params(case.params, storage=binding.LBM_STORE_F16),
                                 A.data_ptr(), 0, 1, 0, None, 0, s)
    assert e.value.status == binding.LBM_EINVAL
    with pytest.raises(binding.LbmError) as e:   # misaligned buffer
        binding.lbm_step_noalloc(prm, A.data_ptr() + 4, 0, 1, 0, None, 0, s)
    assert e.value.status == binding.LBM_EINVAL
    torch.cuda.synchronize()
    assert torch.count_nonzero(A).item() == 0   # nothing was launched
