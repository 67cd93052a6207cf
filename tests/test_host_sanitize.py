"""The host planning code (circuit -> network -> sliced contraction plan:
csrc/network.cpp and csrc/planner.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, host code only) and run on seeded grid
circuits under several option sets; any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

import rqcgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_14502_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_planner_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "plan_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-pthread",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "sanitize", "plan_driver.cpp"),
           os.path.join(CSRC, "network.cpp"), os.path.join(CSRC, "planner.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    circuits = str(tmp_path / "circuits.txt")
    with open(circuits, "w") as f:
        for (rows, cols, depth, seed, n_open) in ((3, 4, 6, 1, 2), (4, 4, 8, 2, 4), (5, 5, 8, 3, 0)):
            c = rqcgen.grid_rqc(rows, cols, depth, seed)
            n = rows * cols
            openq = list(range(n - n_open, n))
            f.write(f"circuit {n} {len(c.gates)} {n_open} {' '.join(map(str, openq))}\n")
            for g in c.gates:
                f.write(f"{int(g.kind)} {int(g.q0)} {int(g.q1) if g.q1 is not None else -1} "
                        f"{float(g.theta)!r} {float(g.phi)!r}\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, circuits], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    # the 3x4 circuit needs no slicing at a 2^10 bound, so its slice-share
    # option set is refused (EINVAL); every other option set plans
    assert "plans 14 rejected 1" in r.stdout, r.stdout[-2000:]
    assert "rejected -1 n_local_sliced exceeds the number of sliced wires" in r.stdout
