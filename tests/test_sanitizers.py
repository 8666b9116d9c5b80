"""Sanitizer runs on the CPU: the oracle's pin tests against an oracle built
with AddressSanitizer and UndefinedBehaviorSanitizer (gcc), and the C ABI's
host-side argument checks against a library whose host code carries the
same sanitizers (hipcc, host code only).  Every finding is fatal, so a
memory error or undefined behaviour fails the child test run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["test_oracle_pins.py", "test_oracle_readings.py", "test_oracle_curved.py",
                "test_oracle_halfstep.py", "test_oracle_mhd_variants.py", "test_oracle_porous.py",
                "test_oracle_adjoint.py"]
MAPS = "import sys; print('\\n'.join(l for l in open('/proc/self/maps') if sys.argv[1] in l))"


def child_env(**extra):
    env = {k: v for k, v in os.environ.items() if k not in ("LBM_LIBRARY", "ORACLE_LIB_DIR", "LD_PRELOAD")}
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    env.update(extra)
    return env


def run(cmd, env, timeout):
    p = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    return p.returncode, p.stdout + p.stderr


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    import oracle.build as ob
    ob.build(outdir=str(tmp_path), sanitize=True)
    gcc_asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    env = child_env(ORACLE_LIB_DIR=str(tmp_path), LD_PRELOAD=gcc_asan)
    # the child loads the sanitized build, not the in-tree one
    rc, out = run([sys.executable, "-c", "import oracle; oracle.Oracle(0, 8, 8, 1, 0.8, 1.0, 1.0, 4); " + MAPS,
                   "liboracle"], env, 120)
    assert rc == 0, out
    assert str(tmp_path) in out and os.path.join(ROOT, "oracle") not in out, out
    rc, out = run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                   *[os.path.join("tests", t) for t in ORACLE_TESTS]], env, 900)
    assert rc == 0, out[-4000:]
    assert " passed" in out and "ERROR: AddressSanitizer" not in out and "runtime error" not in out


def test_host_argument_checks_under_asan_and_ubsan(tmp_path):
    from paper_2512_12213_amd import build as pb
    lib = pb.build_host_sanitized(str(tmp_path))
    # the host code is instrumented: without the runtime the library does not load
    rc, out = run([sys.executable, "-c", "import ctypes, sys; ctypes.CDLL(sys.argv[1])", lib], child_env(), 120)
    assert rc != 0 and "asan" in out.lower(), out
    env = child_env(LBM_LIBRARY=lib, LD_PRELOAD=pb.asan_runtime())
    rc, out = run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                   os.path.join("tests", "test_abi.py")], env, 600)
    assert rc == 0, out[-4000:]
    assert " passed" in out and "ERROR: AddressSanitizer" not in out and "runtime error" not in out
