"""The host geometry plans (csrc/plan.cpp, csrc/plan3.cpp) built with
AddressSanitizer and UndefinedBehaviorSanitizer (g++, no GPU) and run on the
curve and surface workloads, on a mix of seeded serving shapes, and on
geometry the plan must refuse.  Any out-of-bounds access, leak or undefined
behaviour aborts the driver; its own checks keep every stored index inside the
arrays it refers to.  The counts it prints are compared with the oracle's plan.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import kfbi_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_15249_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("asan") / "plan_asan")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(ROOT, "tests", "native", "plan_asan_main.cpp"),
           os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "plan3.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("the sanitizer runtime is not installed")
    assert r.returncode == 0, r.stderr
    return exe


def run(exe, lines):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout.split("\n")[:len(lines)]


def curve_line(xy, n, lo=synth.BOX_LO, hi=synth.BOX_HI):
    return f"2 {n} {lo!r} {hi!r} {len(xy)} " + " ".join(repr(float(v)) for v in np.asarray(xy).ravel())


def test_curves_and_surfaces_under_sanitizers(driver):
    cases = [(synth.circle_points(128), 64), (synth.star_points(256), 512), (synth.star_points(512), 1024)]
    for seed, n in ((7, 256), (8, 256), (9, 512)):
        sp = synth.serving_spec(seed, n)
        cases.append((sp.xy, sp.n))
    lines = [curve_line(xy, n) for xy, n in cases]
    lines += ["3 64 -1.2 1.2 0.9 0.7 0.5", "3 128 -1.2 1.2 0.9 0.7 0.5"]
    out = run(driver, lines)
    for (xy, n), got in zip(cases, out):
        assert got.startswith("ok "), got
        q, i = map(int, got.split()[1:])
        plan = O.build_plan(xy, n, synth.BOX_LO, synth.BOX_HI)
        assert (q, i) == (len(plan.q_axis), len(plan.irr)), (n, q, i, len(plan.q_axis), len(plan.irr))
    # the circle r = 0.8 on the 64^2 grid: 172 crossings, 244 irregular nodes (the counts a
    # brute-force scan of the grid edges gives, pinned in the oracle's tests too)
    assert out[0] == "ok 172 244"
    # the ellipsoid (0.9, 0.7, 0.5) at 64^3 and 128^3: control points (= grid-edge crossings)
    # and irregular nodes, as the oracle's 3D pins count them
    assert out[-2:] == ["ok 6394 7352", "ok 25514 29360"]


def test_refused_geometry_under_sanitizers(driver):
    lines = [
        curve_line(synth.circle_points(256, r=1.18), 128),           # within 2h of the box
        curve_line(synth.circle_points(16, r=0.005) + 0.01, 64),     # between grid lines: no crossing
        curve_line(synth.circle_points(128) * [1.0, 0.0125] + [0.0, 0.01], 64),   # thinner than h: edges crossed twice
        curve_line(np.where(np.arange(128)[:, None] == 5, np.nan, synth.circle_points(128)), 64),   # NaN sample
        "3 64 -1.2 1.2 1.19 0.7 0.5",                                # ellipsoid touching the box
        "3 100 -1.2 1.2 0.9 0.7 0.5",                                # not a supported grid
    ]
    out = run(driver, lines)
    for line, got in zip(lines, out):
        assert got.startswith("geometry "), (line[:40], got)
