"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The FP64 oracle (oracle/mpc_oracle.c) is rebuilt with
  -fsanitize=address,undefined and the whole pin suite
  (tests/test_oracle_pins.py) runs against that build in a child interpreter
  with the sanitizer runtimes preloaded; any report aborts the child.
* The served loop's arena allocator (csrc/server_arena.h) runs its host check
  (tests/arena_check.cpp) built with the same sanitizers.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2510_12717_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _runtime(cc, name):
    p = subprocess.run([cc, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_under_sanitizers(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    asan, ubsan = _runtime(cc, "libasan.so"), _runtime(cc, "libubsan.so")
    if not (asan and ubsan):
        pytest.skip("sanitizer runtimes not installed")
    so = str(tmp_path / "libmpc_oracle_san.so")
    src = os.path.join(ROOT, "oracle", "mpc_oracle.c")
    subprocess.run([cc, "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                    "-shared", "-fPIC", "-Wall", *SAN, "-I", os.path.join(ROOT, "oracle"), "-o", so,
                    src, "-lm"], check=True)
    env = dict(os.environ, MPC_ORACLE_LIB=so, LD_PRELOAD=f"{asan}:{ubsan}", **SAN_ENV)
    out = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"),
                          "-q", "-x", "-p", "no:cacheprovider"], cwd=ROOT, env=env,
                         capture_output=True, text=True, timeout=900)
    text = out.stdout + out.stderr
    assert out.returncode == 0, text[-4000:]
    assert "ERROR: AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    assert " passed" in out.stdout


def test_arena_allocator_under_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "arena_check_san")
    subprocess.run([cxx, "-O1", "-std=c++17", *SAN, "-I", CSRC,
                    os.path.join(HERE, "arena_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                         env=dict(os.environ, **SAN_ENV))
    assert out.returncode == 0 and "arena ok" in out.stdout, out.stdout + out.stderr
