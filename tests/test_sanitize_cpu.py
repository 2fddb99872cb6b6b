"""The library's host-only code (paper_1501_03105_amd/csrc/host_graph.cpp:
graph validation and set-up, the fixed-point conversions of the sweep cut,
the coarse max-flow of the two-level rounding, option checks) and the oracle,
built on the CPU with AddressSanitizer and UndefinedBehaviorSanitizer into
tests/sanitize/driver.cpp and run on small seeded inputs; the max-flows are
checked against exhaustive search there.  The build goes to a temporary
directory."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
# the sanitizer runtimes are linked into the executable, so it needs no
# preloading and comes first whatever else the environment loads
LINK = ["-static-libasan", "-static-libubsan"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="needs gcc and g++")
def test_host_code_and_oracle_under_sanitizers(tmp_path):
    objs = []
    for c in ("graph.c", "irls.c", "sweep.c", "maxflow.c"):
        o = str(tmp_path / (c + ".o"))
        subprocess.run(["gcc", "-std=gnu11", "-fopenmp", "-ffp-contract=off", *SAN, "-c",
                        os.path.join(ROOT, "oracle", c), "-o", o], check=True)
        objs.append(o)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", "-std=c++17", "-fopenmp", *SAN, "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "sanitize", "driver.cpp"),
                    os.path.join(ROOT, "paper_1501_03105_amd", "csrc", "host_graph.cpp"),
                    *objs, *LINK, "-o", exe, "-lm", "-lpthread"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "0 failures" in out
