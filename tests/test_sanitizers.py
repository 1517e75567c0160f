"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle (oracle/oracle.c) is built with -fsanitize=address,undefined and
every pin runs against that build in a process that preloads the sanitizer
runtimes; an out-of-bounds access, a use after free or an undefined operation
(signed overflow, a bad shift, ...) aborts it.  A copy with a planted
out-of-bounds read shows that the instrumented run does catch one."""
import os
import subprocess
import sys

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


def runtimes():
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                           text=True).stdout.strip()
        if not os.path.isabs(p) or not os.path.exists(p):
            pytest.skip(f"{name} not available")
        libs.append(p)
    return ":".join(libs)


def build_oracle(src, out):
    subprocess.check_call(["gcc", *SAN, "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", out, src, "-lm"])


def run_pins(lib):
    env = dict(os.environ, LD_PRELOAD=runtimes(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize",
                                                        "run_oracle_pins.py"), lib],
                          capture_output=True, text=True, env=env, timeout=900)


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    build_oracle(O.SRC, lib)
    r = run_pins(lib)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert r.stdout.count(": ok") == 19, r.stdout


def test_sanitizers_catch_a_planted_overread(tmp_path):
    src = open(O.SRC).read()
    old = "    y[i] = s + c;\n"
    assert src.count(old) == 1
    planted = tmp_path / "oracle_oob.c"
    planted.write_text(src.replace(old, "    y[i] = s + c + 0.0 * x[A->n];\n"))  # one past the end
    lib = str(tmp_path / "liboracle_oob.so")
    build_oracle(str(planted), lib)
    r = run_pins(lib)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]


def test_layout_builders_round_trip_under_sanitizers(tmp_path):
    """The host layout builders of the GPU library (csrc/layout.cpp: CSR row blocks, row
    order, gather order, 16-bit offsets at and past +-32767, sliced slices and padding,
    batch padding of uneven systems) decode back to the input on the CPU, built with the
    address and undefined-behaviour sanitizers (tests/sanitize/layout_check.cpp)."""
    csrc = os.path.join(ROOT, "paper_2108_10591_amd", "csrc")
    exe = str(tmp_path / "layout_check")
    subprocess.check_call(["g++", "-std=c++17", *SAN, f"-I{csrc}",
                           os.path.join(ROOT, "tests", "sanitize", "layout_check.cpp"),
                           os.path.join(csrc, "layout.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stderr[-3000:]
    assert "layout round trips: ok" in r.stdout
