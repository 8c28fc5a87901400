"""GPU parity at the workloads' full sizes, in the configuration bench.py
times (the workloads' default options).

* single_track_2mm (the benchmark workload): the first macro steps against FP64
  oracle fields stored by tests/golden/make_golden.py (oracle converged to
  1e-10 K): FP64 path <= 1e-9, mixed path <= 1e-6 relative max-norm.
* raster_5mm and raster_10mm (raster and large build, mixed precision): properties
  that hold at any size -- the mixed path agrees with the FP64 path to
  1e-6, the energy ledger closes, fields are finite and bounded below by
  the plate temperature -- plus oracle goldens when present.
"""
import os

import numpy as np
import pytest

import workloads as W
from tests._gpu import say, rel_maxerr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_12932_amd import tl  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tl.load()


def _run(wl, n):
    say("run", wl.name, "precision", wl.options.precision, "macro steps", n)
    sim = tl.Sim(wl)
    try:
        sim.step(n)
        Tc, _ = sim.temperature(0)
        Tf, origin = sim.temperature(1)
        return Tc, Tf, origin, sim.ledger(), sim.stats()
    finally:
        sim.close()


def _golden(name):
    files = sorted(f for f in os.listdir(GOLDEN) if f.startswith(name + "_n") and f.endswith(".npz"))
    if not files:
        pytest.skip(f"no golden data for {name}")
    return np.load(os.path.join(GOLDEN, files[-1]), allow_pickle=False)


def _ledger_closes(led):
    lhs = led["stored"] - led["stored0"]
    rhs = led["absorbed"] - led["bottom"] - led["surface"] + led["remap"]
    return abs(lhs - rhs) <= 1e-8 * abs(led["absorbed"])


@pytest.mark.parametrize("prec, tol", [(W.FP64, 1e-9), (W.MIXED, 1e-6)])
def test_single_track_2mm_against_oracle_golden(prec, tol):
    g = _golden("single_track_2mm")
    n = int(g["steps"])
    Tc, Tf, origin, led, st = _run(W.single_track_2mm(prec), n)
    assert tuple(origin) == tuple(int(v) for v in g["origin"])
    ec, ef = rel_maxerr(Tc, g["Tc"]), rel_maxerr(Tf, g["Tf"])
    say("  rel err coarse", ec, "fine", ef)
    assert ec <= tol and ef <= tol
    assert _ledger_closes(led)
    assert led["absorbed"] == pytest.approx(float(g["absorbed"]), rel=1e-12)
    assert led["stored"] == pytest.approx(float(g["stored"]), rel=tol)


@pytest.mark.parametrize("name, n", [("raster_5mm", 6), ("raster_10mm", 3)])
def test_mixed_matches_fp64_at_full_size(name, n):
    a = _run(W.by_name(name, precision=W.FP64), n)
    b = _run(W.by_name(name, precision=W.MIXED), n)
    assert a[2] == b[2]
    ec, ef = rel_maxerr(b[0], a[0]), rel_maxerr(b[1], a[1])
    say("  mixed vs fp64 coarse", ec, "fine", ef)
    assert ec <= 1e-6 and ef <= 1e-6
    for Tc, Tf, _, led, _ in (a, b):
        assert np.isfinite(Tc).all() and np.isfinite(Tf).all()
        assert Tc.min() > 299.0 and Tf.min() > 299.0
        assert _ledger_closes(led)


@pytest.mark.parametrize("name", ["raster_5mm", "raster_10mm"])
def test_large_against_oracle_golden(name):
    g = _golden(name)
    n = int(g["steps"])
    Tc, Tf, origin, led, _ = _run(W.by_name(name), n)
    assert tuple(origin) == tuple(int(v) for v in g["origin"])
    ec, ef = rel_maxerr(Tc, g["Tc"]), rel_maxerr(Tf, g["Tf"])
    say("  rel err coarse", ec, "fine", ef)
    assert ec <= 1e-6 and ef <= 1e-6
    assert _ledger_closes(led)
