"""GPU test of tl_create_static, the allocation-free variant of tl_create:
its handles give bitwise the results of tl_create handles (same kernels on
the library's static device workspace), on two creations in a row -- the
second with a smaller problem, on the array the first one left behind --
and a second live handle on the same device is refused with TL_EBUSY."""
import numpy as np
import pytest

import workloads as W
from tests._gpu import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_12932_amd import tl  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tl.load()


def _fields(sim, n):
    sim.step(n)
    Tc, _ = sim.temperature(0)
    Tf, origin = sim.temperature(1)
    return Tc, Tf, origin, sim.ledger(), sim.stats()


def _compare(wl, n):
    say("tl_create_static vs tl_create:", wl.name, "precision", wl.options.precision,
        "macro steps", n, "workspace bytes", tl.tl_workspace_bytes(wl.mesh, wl.options))
    assert tl.tl_workspace_bytes(wl.mesh, wl.options) <= tl.TL_STATIC_WORKSPACE_BYTES
    ref = tl.Sim(wl)
    try:
        a = _fields(ref, n)
    finally:
        ref.close()
    st = tl.Sim(wl, static=True)
    try:
        b = _fields(st, n)
    finally:
        st.close()
    assert a[2] == b[2]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[3] == b[3]
    for k in ("newton_fine", "cg_fine", "newton_coarse", "cg_coarse", "window_moves"):
        assert a[4][k] == b[4][k], k
    say("  bitwise equal; window moves", b[4]["window_moves"])


def test_static_matches_workspace_twice_second_smaller():
    # the benchmark-size single track (about 24 MB of workspace), then the
    # small single track (under 1 MB) on the same static array
    _compare(W.single_track_2mm(W.FP64), 3)
    _compare(W.single_track_1mm(W.MIXED), 6)


def test_second_live_handle_is_refused():
    wl = W.single_track_1mm()
    a = tl.Sim(wl, static=True)
    try:
        with pytest.raises(tl.TLError) as e:
            tl.Sim(wl, static=True)
        assert e.value.status == tl.TL_EBUSY
        # the first handle is untouched and still runs
        Tc, Tf, _, _, _ = _fields(a, 2)
        ref = tl.Sim(wl)
        try:
            Rc, Rf, _, _, _ = _fields(ref, 2)
        finally:
            ref.close()
        assert np.array_equal(Tc, Rc) and np.array_equal(Tf, Rf)
    finally:
        a.close()
    # released by tl_destroy: a new static handle can be made
    b = tl.Sim(wl, static=True)
    b.close()


def test_too_large_problem_is_refused():
    wl = W.raster_5mm(W.FP64)
    with pytest.raises(tl.TLError) as e:
        tl.Sim(wl, static=True)
    assert e.value.status == tl.TL_ENOMEM
