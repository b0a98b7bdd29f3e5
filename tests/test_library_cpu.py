"""Host-side checks of the C ABI that need no GPU: the built library loads,
exports every entry point include/turboadmm.h declares, and rejects bad
arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "turboadmm.h")

tadmm = pytest.importorskip("paper_2602_15838_amd")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tadmm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = tadmm.lib()
    names = _declared()
    assert "tadmm_solve" in names and "tadmm_adjoint" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(tadmm.EXPORTED_SYMBOLS)


def test_version_and_status_strings():
    L = tadmm.lib()
    assert L.tadmm_version().decode().startswith("turboadmm")
    assert L.tadmm_status_string(0) == b"ok"
    assert L.tadmm_status_string(3) == b"non-finite input"
    assert L.tadmm_status_string(99) == b"unknown status"


def _ws(prm, N, T):
    N = np.asarray(N, np.int32)
    T = np.asarray(T, np.int32)
    nb = C.c_size_t(0)
    rc = tadmm.lib().tadmm_workspace_size(C.byref(prm), int(N.size), N.ctypes.data_as(tadmm._ip),
                                          T.ctypes.data_as(tadmm._ip), C.byref(nb))
    return rc, nb.value


def test_workspace_size_scales_with_batch():
    p = synth.ProblemParams()
    prm = tadmm.make_params(p)
    rc1, b1 = _ws(prm, [2], [20])
    rc2, b2 = _ws(prm, [2, 14, 32], [20, 20, 40])
    assert rc1 == 0 and rc2 == 0 and 0 < b1 < b2
    rc0, b0 = _ws(prm, [], [])
    assert rc0 == 0
    p3 = synth.ProblemParams(dp=3, u_max=3.0)
    rc3, b3 = _ws(tadmm.make_params(p3), [2], [20])
    assert rc3 == 0 and b3 > b1


@pytest.mark.parametrize("field,value", [("rho", 0.0), ("rho", -1.0), ("max_iter", 0), ("nx", 5),
                                         ("qT_scale", 0.0), ("eps_abs", -1.0), ("normal_mode", 7),
                                         ("block_threads", 100), ("block_threads", 512), ("mu_tol", float("nan")),
                                         ("refine_band", -1.0)])
def test_bad_params_rejected(field, value):
    prm = tadmm.make_params(synth.ProblemParams())
    setattr(prm, field, value)
    rc, _ = _ws(prm, [2], [20])
    assert rc == 1


def test_inverted_box_rejected():
    prm = tadmm.make_params(synth.ProblemParams())
    prm.u_lo[0], prm.u_hi[0] = 1.0, -1.0
    assert _ws(prm, [2], [20])[0] == 1


@pytest.mark.parametrize("field, value", [("rho_mu", 0.5), ("rho_tau", 1.0), ("rho_every", 0),
                                          ("rho_tau", float("nan"))])
def test_bad_adaptive_rho_params_rejected(field, value):
    prm = tadmm.make_params(synth.ProblemParams(), adaptive_rho=True)
    assert _ws(prm, [2], [20])[0] == 0
    setattr(prm, field, value)
    rc, _ = _ws(prm, [2], [20])
    assert rc == 1
    prm.adaptive_rho = 0          # the fields are not read with a fixed penalty
    assert _ws(prm, [2], [20])[0] == 0


@pytest.mark.parametrize("lo, hi", [(1.0, 1.0), (2.0, -2.0), (float("nan"), 1.0), (float("inf"), float("inf"))])
def test_bad_state_box_rejected(lo, hi):
    prm = tadmm.make_params(synth.ProblemParams(), state_box=True, s_lo=(-1.0, -1.0), s_hi=(1.0, 1.0))
    assert _ws(prm, [2], [20])[0] == 0
    prm.s_lo[1], prm.s_hi[1] = lo, hi
    assert _ws(prm, [2], [20])[0] == 1
    prm.state_box = 0             # the bounds are not read without the box
    assert _ws(prm, [2], [20])[0] == 0
    prm = tadmm.make_params(synth.ProblemParams(), state_box=True, p_lo=(-1.0, -1.0), p_hi=(1.0, 1.0))
    assert _ws(prm, [2], [20])[0] == 0
    prm.p_lo[0], prm.p_hi[0] = lo, hi
    assert _ws(prm, [2], [20])[0] == 1
    # a one-sided box (an infinite end) is allowed; the unused third slot is not read in 2-D
    prm = tadmm.make_params(synth.ProblemParams(), state_box=True, s_lo=(-1.0, -np.inf), s_hi=(np.inf, 1.0))
    prm.s_lo[2] = prm.s_hi[2] = float("nan")
    assert _ws(prm, [2], [20])[0] == 0


@pytest.mark.parametrize("extra", [dict(mom_eta=1.0), dict(mom_eta=0.0), dict(adaptive_rho=True), dict(alpha=1.5),
                                   dict(state_box=True, s_lo=(-1.0, -1.0), s_hi=(1.0, 1.0))])
def test_bad_momentum_params_rejected(extra):
    prm = tadmm.make_params(synth.ProblemParams(), momentum=True)
    assert _ws(prm, [2], [20])[0] == 0
    assert _ws(tadmm.make_params(synth.ProblemParams(), momentum=True, **extra), [2], [20])[0] == 1
    assert _ws(tadmm.make_params(synth.ProblemParams(), **extra), [2], [20])[0] == 0   # valid without momentum


@pytest.mark.parametrize("alpha", [-0.5, 2.0, float("nan"), float("inf")])
def test_bad_relaxation_rejected(alpha):
    prm = tadmm.make_params(synth.ProblemParams(), alpha=1.5)
    assert _ws(prm, [2], [20])[0] == 0
    prm.alpha = alpha
    assert _ws(prm, [2], [20])[0] == 1


def test_relaxation_workspace_holds_the_copies():
    """alpha != 1 adds 2 nu floats per ordered pair copy and step (rounded
    up to the region alignment); alpha = 0 reads as plain ADMM."""
    sizes = {}
    for a in (1.0, 0.0, 1.5):
        rc, b = _ws(tadmm.make_params(synth.ProblemParams(), alpha=a), [5, 3], [20, 11])
        assert rc == 0
        sizes[a] = b
    assert sizes[0.0] == sizes[1.0]
    extra = 4 * 2 * 2 * (20 * 5 * 5 + 11 * 3 * 3)
    assert extra <= sizes[1.5] - sizes[1.0] <= extra + 512


@pytest.mark.parametrize("N,T", [([0], [20]), ([2], [0]), ([5000], [10])])
def test_bad_shapes_rejected(N, T):
    prm = tadmm.make_params(synth.ProblemParams())
    assert _ws(prm, N, T)[0] == 2


def test_null_arguments():
    L = tadmm.lib()
    prm = tadmm.make_params(synth.ProblemParams())
    assert L.tadmm_workspace_size(C.byref(prm), 1, None, None, None) == 1
    assert L.tadmm_create(None, C.byref(prm), None) == 1
    assert L.tadmm_solve(None, None, None, None, 0, 0) == 1
    assert L.tadmm_destroy(None) == 1
    assert L.tadmm_last_kernel_ms(None) == -1.0


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the header's sizes and field
    offsets (a C program compiled against include/turboadmm.h prints them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no C compiler or HIP headers")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    fields = {"tadmm_params": [n for n, _ in tadmm.Params._fields_],
              "tadmm_batch": [n for n, _ in tadmm.Batch._fields_],
              "tadmm_out": [n for n, _ in tadmm.Out._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "turboadmm.h"', 'int main(void) {']
    for st, names in fields.items():
        lines.append(f'  printf("{st} %zu\\n", sizeof({st}));')
        for n in names:
            lines.append(f'  printf("{st}.{n} %zu\\n", offsetof({st}, {n}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", inc, "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                              text=True).stdout.split("\n") if line)
    for st, cls in (("tadmm_params", tadmm.Params), ("tadmm_batch", tadmm.Batch), ("tadmm_out", tadmm.Out)):
        assert int(got[st]) == C.sizeof(cls), st
        for n in fields[st]:
            assert int(got[f"{st}.{n}"]) == getattr(cls, n).offset, (st, n)
