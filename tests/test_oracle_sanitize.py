"""The FP64 reference under AddressSanitizer and UndefinedBehaviorSanitizer.

afr_oracle.c is rebuilt with ``-fsanitize=address,undefined`` (every report fatal) and the reference's
own pins (the ``tests/test_oracle_*.py`` files) are run against that build in a child process, so an
out-of-bounds access, a use after free or undefined arithmetic anywhere the pins reach fails here.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if out.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_pass_under_sanitizers(oracle, tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_asan.so")
    flags = [f for f in oracle.CFLAGS if f != "-O2"]
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", *flags, "-o", lib, oracle.source_path(), "-lm"])
    env = dict(os.environ)
    env.update(AFR_ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=97",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=98")
    pins = sorted(f for f in os.listdir(os.path.join(ROOT, "tests"))
                  if f.startswith("test_oracle_") and f != os.path.basename(__file__))
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           *(os.path.join("tests", f) for f in pins)]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    log = r.stdout + r.stderr
    assert "runtime error" not in log and "AddressSanitizer" not in log, log[-4000:]
    assert r.returncode == 0, log[-4000:]
    assert " passed" in log
