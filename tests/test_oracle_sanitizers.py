"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code, gcc), run under the fast oracle pins: no out-of-bounds access,
use after free or undefined operation on any of their paths (the pins'
scenarios reach the active set, every ADMM variant, the state boxes, the
per-agent data and the fallback normals).  Runs in a child process with the
sanitizer runtimes preloaded; any report aborts it."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "tadmm_oracle.c")

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import oracle
oracle._lib = None
oracle.build = lambda force=False: {lib!r}
oracle.lib()
from tests import test_oracle_mutants as m
failed = [fn.__name__ for fn in m.PIN_FUNCS if not m._call_pin(fn)]
print("pins failed:", failed, flush=True)
sys.exit(1 if failed else 0)
"""


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_oracle_clean_under_address_and_undefined_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fPIC", "-shared", "-fopenmp", SRC, "-o", lib, "-lm"],
                   check=True, capture_output=True)
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], env=env, capture_output=True,
                       text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
