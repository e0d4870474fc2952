"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the oracle's pins (residual,
tangent and adjoint, growth matrix and sigma_1, energies and objectives, codec, Roe flux and
characteristic boundaries) run in a child process against a sanitized build of the same source,
with every sanitizer report fatal.  A memory error or undefined behaviour anywhere in the oracle
fails this test, whatever the pins' own tolerances."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_growth_energy.py", "tests/test_oracle_roe.py",
        "tests/test_oracle_char.py", "tests/test_oracle_energy.py"]


def test_oracle_pins_under_sanitizers():
    import oracle
    so = oracle.build_sanitized()
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ)
    env.update(ADJNS_ORACLE_SO=so, LD_PRELOAD=asan, OMP_NUM_THREADS="4",
               # the interpreter is not instrumented: leaks of its own and of numpy are not the oracle's
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu and not slow"]
                       + PINS, cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=1500)
    tail = "\n".join(r.stdout.splitlines()[-30:])
    assert r.returncode == 0, tail
    assert "passed" in tail and "ERROR: AddressSanitizer" not in r.stdout and "runtime error" not in r.stdout, tail
