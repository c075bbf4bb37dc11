"""The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer: the oracle (gcc build with
-fsanitize=address,undefined, gcc's runtimes preloaded) runs its pins, and the library's host code
(hipcc build with the sanitizers on the host side only, clang's runtime preloaded) builds and checks
its tables; each in a process of its own, failing on the first report."""
import os
import subprocess
import sys

import pytest

import oracle
from paper_2403_15051_amd import build as lbe_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _stale(lib, sources):
    return not os.path.exists(lib) or any(os.path.getmtime(s) > os.path.getmtime(lib) for s in sources)


def _run(env_extra, args):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *args],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0


@pytest.mark.slow
def test_oracle_pins_under_sanitizers():
    lib = oracle.build(force=_stale(oracle.SAN_LIB, [oracle._SRC]), sanitize=True)
    pre = ":".join(subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True,
                                  check=True).stdout.strip() for n in ("libasan.so", "libubsan.so"))
    _run({"LD_PRELOAD": pre, "LBE_ORACLE_LIB": lib, "OMP_NUM_THREADS": "2"},
         ["tests/test_oracle_pins.py", "-k", "not rest_state"])


@pytest.mark.slow
def test_host_tables_under_sanitizers():
    srcs = [os.path.join(lbe_build.CSRC, s) for s in lbe_build.SOURCES]
    lib = lbe_build.SAN_LIB if not _stale(lbe_build.SAN_LIB, srcs) else lbe_build.build(sanitize=True)
    _run({"LD_PRELOAD": lbe_build.san_runtime(), "LBE_LIB": lib}, ["tests/test_host_tables.py"])
