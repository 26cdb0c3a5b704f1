"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only), run over every pin, single-threaded and with 4 OpenMP
threads: no out-of-bounds access, use after free or undefined behaviour on
the pins' inputs.  Runs in a subprocess with the sanitizer runtime
preloaded (the Python interpreter itself is not instrumented)."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    except OSError:
        return None
    return p if p and os.path.exists(p) else None


@pytest.mark.skipif(_runtime() is None, reason="gcc's AddressSanitizer runtime is not installed")
def test_oracle_pins_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        so = os.path.join(d, "liboracle_san.so")
        cmd = ["gcc", "-O1", "-g", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
               "-o", so, os.path.join(oracle.HERE, "oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
        code = ("import sys; sys.path[:0] = [%r, %r]\n"
                "import oracle, pins\n"
                "L = oracle.lib(%r)\n"
                "for p in pins.ALL_PINS + [pins.pin_stencil_closed_form]:\n"
                "    p(L)\n"
                "pins.NTHREADS = 4\n"
                "for p in pins.ALL_PINS:\n"
                "    p(L)\n"
                "print('sanitized pins ok')\n") % (ROOT, os.path.join(ROOT, "tests"), so)
        env = dict(os.environ, LD_PRELOAD=_runtime(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0 and "sanitized pins ok" in r.stdout, r.stderr[-4000:]
