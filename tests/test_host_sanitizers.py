"""CPU: the host C code (the oracle's hopping term and the input generator) built with
AddressSanitizer and UndefinedBehaviorSanitizer, and the oracle's pins and property tests
run against those builds in a child process.  Any out-of-bounds access, use after free or
undefined operation in the C code stops the child with a sanitizer report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fopenmp", "-fPIC", "-shared"]


def _gcc_runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], stdout=subprocess.PIPE, text=True).stdout.strip()
    return os.path.realpath(p) if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    libs = {}
    for env, src, extra in (("ORACLE_WREF_LIB", "oracle/wref.c", []),
                            ("ORACLE_WREF32_LIB", "oracle/wref.c", ["-DWREF_FP32"]),
                            ("LATTICE_SYNTH_LIB", "lattice_synth/synth.c", [])):
        out = str(tmp_path / (env.lower() + ".so"))
        subprocess.check_call(["gcc"] + FLAGS + extra + ["-o", out, os.path.join(ROOT, src), "-lm"])
        libs[env] = out
    env = dict(os.environ, **libs)
    env["LD_PRELOAD"] = asan   # the ASan runtime must come first in a process that is not itself built with it
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"   # the interpreter keeps its objects to the end
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-s", "-x", "-p", "no:cacheprovider", "-m", "not gpu and not slow",
                        "tests/test_oracle_pins.py", "tests/test_oracle_properties.py"],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=1200)
    tail = r.stdout[-3000:]
    assert "AddressSanitizer" not in r.stdout and "runtime error" not in r.stdout, tail
    assert r.returncode == 0, tail
    assert " passed" in tail, tail
