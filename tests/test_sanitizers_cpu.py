"""The host code under AddressSanitizer and UBSan (no GPU): the host-only build of the library
(builder, planner, primal search, C-ABI checks; device calls stubbed to fail) and the oracle, both
compiled with -fsanitize=address,undefined and no recovery, run the CPU tests of the planner, the
boundary, the primal search, the dataflow schedule and the oracle's pins in a child process with
libasan preloaded. Any sanitizer report aborts that process."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SUITES = ["tests/test_plan_cpu.py", "tests/test_boundary_cpu.py", "tests/test_primal_cpu.py", "tests/test_batch_cpu.py",
          "tests/test_dataflow_protocol.py", "tests/test_oracle_pins.py", "tests/test_residual_oracle.py",
          "tests/test_smooth_oracle.py", "tests/test_split_oracle.py"]


def _libasan():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(_libasan() is None, reason="gcc's libasan is not available")
def test_cpu_suites_under_address_and_undefined_sanitizers():
    from paper_2009_00481_amd import build

    lib = build.build_host_only()
    env = dict(os.environ)
    env["BDDMP_SANITIZE"] = "1"
    subprocess.run([sys.executable, os.path.join(ROOT, "oracle", "build.py")], check=True, env=env, cwd=ROOT)
    env.update(LD_PRELOAD=_libasan(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", BDDMP_HOST_ONLY_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", *SUITES],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "Sanitizer" not in r.stdout + r.stderr, tail
    assert " passed" in r.stdout, tail
