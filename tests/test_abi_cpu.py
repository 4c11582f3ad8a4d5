"""Host-side checks of the C ABI (no GPU needed).

* the HIP library loads and exports every function the headers in include/ declare
* the ctypes mirrors of lbm_params / lbm_diag / lbm_launch / lbm_batch_tuning match
  the C layout (checked with a
  small C program compiled by gcc against the header)
* lbm_state_bytes: 35 padded arrays; 140 B/cell FP32 and 70 B/cell FP16 (Sec. 4:
  the five-field state of a 512^3 grid is about 19 GB)
* parameter validation returns LBM_EINVAL with a message, before any device call
"""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2609_16361_amd import binding, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grlbm.h")
HEADERS = sorted(os.path.join(ROOT, "include", h) for h in os.listdir(os.path.join(ROOT, "include"))
                 if h.endswith(".h"))


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(lbm_\w+)\s*\(", src, flags=re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = declared_functions()
    assert len(names) >= 15, names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.SIGNATURES), set(names) ^ set(binding.SIGNATURES)


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "grlbm.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(lbm_params),"
        " offsetof(lbm_params, gamma), offsetof(lbm_params, omega), offsetof(lbm_params, E_ref),"
        " sizeof(lbm_diag), offsetof(lbm_diag, nonfinite), sizeof(lbm_launch), offsetof(lbm_launch, odd_lds),"
        " sizeof(lbm_batch_tuning), offsetof(lbm_batch_tuning, grid)); return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)], check=True)
    vals = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True,
                                        check=True).stdout.split()))
    P, D, L, T = binding.lbm_params, binding.lbm_diag, binding.lbm_launch, binding.lbm_batch_tuning
    assert vals == [ctypes.sizeof(P), P.gamma.offset, P.omega.offset, P.E_ref.offset,
                    ctypes.sizeof(D), D.nonfinite.offset, ctypes.sizeof(L), L.odd_lds.offset,
                    ctypes.sizeof(T), T.grid.offset]


def test_mms_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "mms.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "grlbm_mms.h"\n'
                    'int main(void){printf("%zu %zu\\n", sizeof(lbm_mms), offsetof(lbm_mms, kappa));'
                    ' return 0;}\n')
    exe = tmp_path / "mms"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)], check=True)
    vals = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()))
    M = binding.lbm_mms
    assert vals == [ctypes.sizeof(M), M.kappa.offset]


def test_generated_mms_kernel_is_current():
    """csrc/grlbm_mms.hip is what the generator produces from eq. 2 and eq. 8."""
    from paper_2609_16361_amd import mms_codegen
    assert open(mms_codegen.OUT).read() == mms_codegen.generate()


def test_generator_source_matches_oracle():
    """The SymPy source behind the generated kernel and the oracle's hand-written
    source are two derivations of the same residual of eq. 2."""
    import numpy as np
    import sympy as sp
    import oracle
    from paper_2609_16361_amd import mms_codegen
    (x, y, z, t), c, S = mms_codegen.source_expressions()
    case = inputs.mms(n=10)
    m = case.meta["mms"]
    sub = {c[k]: m[k] for k in mms_codegen.CONSTS}
    f = sp.lambdify((x, y, z, t), [e.subs(sub) for e in S], "math")
    So = oracle.mms_source(case.params, m, 3.5)
    for i, j, l in ((0, 0, 0), (3, 7, 1), (9, 2, 5)):
        ref = f(float(i), float(j), float(l), 3.5)
        for k in range(5):
            assert abs(So[k, l, j, i] - ref[k]) <= 1e-11 * max(abs(ref[k]), 1e-3 * np.abs(So[k]).max())


def test_state_bytes():
    c = inputs.tgv(n=512, dims=(512, 512, 512))
    p = binding.make_params(c.params)
    n = 512 ** 3
    assert binding.lbm_state_bytes(p) == 35 * 4 * n
    assert abs(35 * 4 * n / 1e9 - 19) < 0.5          # "19 GB" at 512^3
    p16 = binding.make_params(c.params, storage=binding.LBM_STORE_F16)
    assert binding.lbm_state_bytes(p16) == 35 * 2 * n
    small = binding.make_params(inputs.sod(n=100, ny=3, nz=1).params)
    per = (300 + 63) // 64 * 64                      # arrays padded to 256 bytes
    assert binding.lbm_state_bytes(small) == 35 * 4 * per   # 28 of 100 would be too much row padding
    # rows padded to whole 128-byte lines when that adds at most a sixteenth: a
    # 1000-cell row to 1024 in FP32 and FP16; 144 -> 160 would add a ninth, so none
    odd = binding.make_params(inputs.tgv(n=144, dims=(1000, 12, 10)).params)
    assert binding.lbm_state_bytes(odd) == 35 * 4 * ((1024 * 120 + 63) // 64 * 64)
    odd.storage = binding.LBM_STORE_F16
    assert binding.lbm_state_bytes(odd) == 35 * 2 * ((1024 * 120 + 127) // 128 * 128)
    cube = binding.make_params(inputs.tgv(n=144, dims=(144, 144, 144)).params)
    assert binding.lbm_state_bytes(cube) == 35 * 4 * ((144 ** 3 + 63) // 64 * 64)
    one_row = binding.make_params(inputs.sod(n=1000, ny=1, nz=1).params)   # nothing to align
    assert binding.lbm_state_bytes(one_row) == 35 * 4 * ((1000 + 63) // 64 * 64)
    small.layout_pad = 1000
    assert binding.lbm_state_bytes(small) == 35 * 4 * ((1300 + 63) // 64 * 64)
    # one MI355X holds a 1024^3 FP32 state (150 GB of its 288 GB); 32-bit cell
    # indices allow up to 2^31 - 2^16 cells (1290^3 keeps unpadded rows: padded to
    # 1312 they would leave that range)
    big = binding.make_params(inputs.tgv(n=8, dims=(8, 8, 8)).params)
    big.nx = big.ny = big.nz = 1024
    assert binding.lbm_state_bytes(big) == 35 * 4 * 1024 ** 3
    big.nx = big.ny = big.nz = 1290
    assert binding.lbm_state_bytes(big) == 35 * 4 * ((1290 ** 3 + 63) // 64 * 64)


@pytest.mark.parametrize("mutate,needle", [
    (lambda p: setattr(p, "nx", 0), "dims"),
    (lambda p: p.bc.__setitem__(0, 7), "bc[0]"),
    (lambda p: (p.bc.__setitem__(2, 1), setattr(p, "nz", 1)), "zero-gradient"),
    (lambda p: p.omega.__setitem__(1, 2.5), "omega[1]"),
    (lambda p: p.omega.__setitem__(4, 0.0), "omega[4]"),
    (lambda p: p.omega.__setitem__(2, 1.5), "momentum"),
    (lambda p: setattr(p, "gamma", 1.0), "gamma"),
    (lambda p: setattr(p, "collision", 3), "collision"),
    (lambda p: setattr(p, "storage", 9), "storage"),
    (lambda p: setattr(p, "rho_min", 0.0), "rho_min"),
    (lambda p: setattr(p, "layout_pad", -1), "layout_pad"),
    (lambda p: setattr(p, "start", 2), "start"),
    (lambda p: setattr(p, "T_ref", float("nan")), "T_ref"),
    (lambda p: (setattr(p, "nx", 1291), setattr(p, "ny", 1291), setattr(p, "nz", 1291)), "32-bit"),
])
def test_validation_rejects(mutate, needle):
    p = binding.make_params(inputs.tgv(n=8, dims=(8, 8, 8)).params)
    mutate(p)
    assert binding.lbm_state_bytes(p) == 0
    with pytest.raises(binding.LbmError) as e:
        binding.lbm_create(p)
    assert e.value.status == binding.LBM_EINVAL
    assert needle in str(e.value)


def test_null_arguments():
    lib = binding.load()
    assert lib.lbm_destroy(None) == 0
    assert lib.lbm_step(None, 1, 0) == binding.LBM_EINVAL
    assert "NULL" in binding.lbm_last_error()
    cnt = ctypes.c_int32(5)
    assert lib.lbm_diagnostics(None, None, 0, ctypes.byref(cnt)) == binding.LBM_EINVAL
    best = binding.lbm_launch()
    assert lib.lbm_autotune(None, 10, ctypes.byref(best), None, None, None, 0, None) == binding.LBM_EINVAL
    assert lib.lbm_get_launch(None, ctypes.byref(best)) == binding.LBM_EINVAL
    assert lib.lbm_batch_nonfinite(None, None, 0, ctypes.byref(cnt)) == binding.LBM_EINVAL
