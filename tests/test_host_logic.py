"""The library's host-side scan-path and geometry logic (tl_host.cpp:
laser position, window rule, swept source boxes, Gauss rules), built with
g++ under AddressSanitizer and UndefinedBehaviorSanitizer and driven on the
CPU, against the oracle's functions for the same inputs.  No GPU needed."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import laser as L
from oracle import twolevel as TW
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2110_12932_amd", "csrc")
UM = 1e-6


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("host") / "host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", f"-I{CSRC}",
           os.path.join(CSRC, "tl_host.cpp"), os.path.join(HERE, "host", "host_check.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-300:])
    return exe


def _run(exe, lines):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True,
                       text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    return r.stdout.split("\n")


def _tracks(scan):
    out = [f"T {len(scan.tracks)}"]
    for t in scan.tracks:
        out.append(" ".join(repr(float(v)) for v in (t.x0, t.y0, t.x1, t.y1, t.speed,
                                                      t.power, t.radius, t.absorptivity,
                                                      t.depth)))
    out.append(f"S {scan.t_start!r}")
    return out


@pytest.mark.parametrize("name", ["c0", "corner"])
def test_laser_position_and_window_rule(driver, name):
    wl = W.small_cases()[name]
    mesh, scan = wl.mesh, wl.scan
    coarse = TW.coarse_grid(mesh)
    starts, t_end = L.track_start_times(scan)
    times = [float(t) for t in np.linspace(scan.t_start - 20e-6, t_end + 20e-6, 61)]
    q = _tracks(scan)
    cur = (3, 2)
    for t in times:
        q.append(f"L {t!r}")
        q.append(f"W {t!r} {coarse.hx!r} {coarse.hy!r} {mesh.nx} {mesh.ny} "
                 f"{mesh.win_nx} {mesh.win_ny} 1 {cur[0]} {cur[1]}")
    out = [l for l in _run(driver, q) if l]
    for n, t in enumerate(times):
        lo = out[2 * n].split()
        ref = L.laser_at(scan, t)
        assert int(lo[1]) == (ref is not None)
        if ref is not None:
            got = [float(v) for v in lo[2:7]]
            assert got == pytest.approx(list(ref[:5]), rel=1e-14, abs=1e-18)
            assert int(lo[7]) == ref[5]
        wo = out[2 * n + 1].split()
        assert (int(wo[1]), int(wo[2])) == TW.window_origin(mesh, coarse, scan, t, current=cur)


def test_swept_boxes(driver):
    R, d, v, P, eta = 80 * UM, 40 * UM, 0.5, 200.0, 0.4
    scan = W.ScanPath([
        W.Track(0.1e-3, 0.5e-3, 0.3e-3, 0.5e-3, v, P, R, eta, d),
        W.Track(0.3e-3, 0.5e-3, 0.3e-3, 0.9e-3, v, P, R, eta, d),
        W.Track(0.3e-3, 0.9e-3, 0.1e-3, 0.9e-3, 2 * v, P, R, eta, d)], t_start=10e-6)
    z_top = 1e-3
    steps = [(0.0, 50e-6), (100e-6, 300e-6), (350e-6, 500e-6), (390e-6, 1.4e-3),
             (1.3e-3, 1.6e-3), (2e-3, 3e-3)]
    q = _tracks(scan) + [f"B {a!r} {b!r}" for a, b in steps]
    out = [l for l in _run(driver, q) if l]
    pos = 0
    for a, b in steps:
        head = out[pos].split()
        n = int(head[1])
        ref = L.swept_boxes(scan, a, b, z_top)
        assert n == len(ref)
        for k in range(n):
            got = [float(x) for x in out[pos + 1 + k].split()]
            x0, x1, y0, y1, z0, z1, qv = ref[k]
            assert got == pytest.approx([x0, x1, y0, y1, z1 - z0, qv], rel=1e-13, abs=1e-18)
        pos += 1 + n


@pytest.mark.parametrize("nq", [1, 2, 3, 4])
def test_gauss_rules(driver, nq):
    out = _run(driver, [f"G {nq}"])[0].split()[1:]
    got = np.array([float(v) for v in out]).reshape(nq, 2)
    x, w = L.gauss01(nq)
    assert np.allclose(got[:, 0], x, rtol=0, atol=1e-15)
    assert np.allclose(got[:, 1], w, rtol=0, atol=1e-15)
