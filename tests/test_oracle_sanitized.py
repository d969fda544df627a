"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is built again from the same source with ``-fsanitize=address,undefined``
(no recovery: the first finding aborts), and every oracle pin in
``test_oracle_pins.py`` runs against that build in a child process with the
sanitizer runtimes preloaded.  A pass means no out-of-bounds access, use after
free or undefined operation on any path those pins take.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _runtime(name):
    if not shutil.which("gcc"):
        return None
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not available")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-o", lib, os.path.join(ROOT, "oracle", "ibm_oracle.c"), "-lm"])
    env = dict(os.environ)
    env.update({"LD_PRELOAD": asan + ":" + ubsan, "IBM_ORACLE_LIB": lib, "OMP_NUM_THREADS": "4",
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    probe = "import oracle, sys; sys.exit(0 if oracle._LIB == %r else 3)" % lib
    assert subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env).returncode == 0
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"), "-x", "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
