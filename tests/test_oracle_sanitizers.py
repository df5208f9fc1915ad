"""The oracle's pins, run again against a build of oracle/orc.c with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code only): any
out-of-bounds access, use after free, signed overflow, misaligned or null
access or invalid shift in the oracle aborts the run.  The oracle is built
into a temporary directory and loaded by the pin tests through
CAMG_ORACLE_LIB; the ASan runtime is preloaded into the child interpreter.
Leak checking is off (the interpreter itself does not free everything at
exit)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle.py", "tests/test_oracle_fsai.py", "tests/test_oracle_afsai.py",
             "tests/test_oracle_interp.py", "tests/test_oracle_bamg.py", "tests/test_oracle_srqm.py"]


def _asan_runtime():
    gcc = shutil.which("gcc")
    if not gcc:
        return None
    p = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_clean_under_asan_ubsan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc with the AddressSanitizer runtime is not available")
    lib = str(tmp_path / "liborc_san.so")
    build = subprocess.run(
        ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fPIC", "-shared", "-o", lib,
         os.path.join(ROOT, "oracle", "orc.c"), "-lm"], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "CAMG_ORACLE_LIB": lib,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    r = subprocess.run([sys.executable, "-m", "pytest", *PIN_FILES, "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out and "failed" not in out
