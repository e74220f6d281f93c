"""The oracle's pins on an AddressSanitizer + UndefinedBehaviorSanitizer build
of oracle/cfo.c: an out-of-bounds access, a use of freed memory or undefined
arithmetic anywhere on the paths the pins drive ends the run with the
sanitizer's report instead of passing silently."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_oracle_box_pins.py", "tests/test_oracle_tree_pins.py",
             "tests/test_oracle_learned_pins.py", "tests/test_adjoint_fd_pins.py"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_clean_under_asan_and_ubsan(tmp_path):
    from oracle import cfo
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc's sanitizer runtimes are not installed")
    lib = cfo.build(force=True, path=str(tmp_path / "libcfo_san.so"), sanitize=True)
    env = dict(os.environ, CFO_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = "from oracle import cfo; import sys; sys.exit(0 if cfo.lib()._name == sys.argv[1] else 3)"
    r = subprocess.run([sys.executable, "-c", probe, lib], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, ("the child did not load the sanitizer build", r.stderr[-2000:])
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "--capture=sys",
                        "-m", "not gpu",
                        *PIN_FILES], env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    log = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, log
    for mark in ("AddressSanitizer", "runtime error:"):
        assert mark not in r.stdout + r.stderr, log
