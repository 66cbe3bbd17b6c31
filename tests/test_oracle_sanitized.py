"""The oracle's pin suite run against an AddressSanitizer + UndefinedBehavior-
Sanitizer build of the oracle (host code only, gcc): out-of-bounds reads or
writes, use after free, signed overflow, bad shifts and misaligned accesses in
the C oracle fail the run.  The suite runs in a child interpreter that preloads
the sanitizer runtimes and loads the instrumented library (SADREF_LIB)."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not available")
    lib = str(tmp_path / "libsad_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-pthread",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "sad_oracle.c"),
                           "-o", lib])
    env = dict(os.environ)
    env.update(SADREF_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=87",
               SAD_GEN_WORKERS="1")
    pins = sorted(glob.glob(os.path.join(HERE, "test_oracle_*.py")))
    pins = [p for p in pins if not p.endswith("test_oracle_sanitized.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *pins], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
