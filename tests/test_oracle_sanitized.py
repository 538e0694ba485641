"""The CPU reference built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only), running every pin: an out-of-bounds access, a use after free or
undefined arithmetic in the reference would abort the run."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]

RUNNER = r"""
import sys
sys.path.insert(0, %(root)r)
sys.path.insert(0, %(tests)r)
import numpy as np
import oracle
import pins
from paper_1911_09340_amd import synth

o = oracle.Oracle(oracle.load(%(lib)r))
ev, ev_exact = synth.event_plain(0), synth.event_plain(0, sigma=0.0)
for check in pins.ALL_SIMPLE:
    check(o)
for check, e in [(pins.pin_far_seed, ev), (pins.pin_truth_seed, ev_exact),
                 (pins.pin_grid_argmin, ev_exact), (pins.pin_rotation, ev),
                 (pins.pin_brute_force, ev), (pins.pin_gradient_fd, ev),
                 (pins.pin_lm_truth, ev_exact)]:
    check(o, e)
print("SANITIZED PINS OK", flush=True)
"""


def _runtime(name):
    path = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_pins_under_address_and_ub_sanitizers():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    with tempfile.TemporaryDirectory() as d:
        lib = oracle.build(out=os.path.join(d, "liboracle_san.so"), extra=SAN_FLAGS)
        env = dict(os.environ)
        env["LD_PRELOAD"] = asan
        # the interpreter's own allocations are not the reference's: leaks are not checked
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
        env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
        env["OMP_NUM_THREADS"] = "4"
        code = RUNNER % {"root": ROOT, "tests": HERE, "lib": lib}
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=1500)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "SANITIZED PINS OK" in r.stdout, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
