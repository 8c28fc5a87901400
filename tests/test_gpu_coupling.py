"""GPU parity of both forms of the two-level correction against the FP64
CPU oracle's Dirichlet-Neumann iteration (the paper's Section 3): the
composite-grid solve (one Newton solve over the free fine nodes and the
coarse nodes outside the window interior, the fine interface values slaved
to the coarse ones; the default) and the GPU's own Dirichlet-Neumann
iteration with interface quasi-Newton relaxation.  Both reach the oracle's
discrete solution.  Also the paper's alternate global formulation against
the oracle's.  Tolerances: 1e-9 (FP64), 1e-6 (mixed) relative max-norm."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
import workloads as W
from tests._gpu import say, rel_maxerr, oracle_fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_12932_amd import tl  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tl.load()
    yield
    torch.cuda.synchronize()


def _with(wl, coupling):
    return replace(wl, options=replace(wl.options, coupling=coupling))


def _run(wl, n_macro):
    say("case", wl.name, "precision", wl.options.precision, "coupling",
        wl.options.coupling, "macro steps", n_macro)
    sim = tl.Sim(wl)
    try:
        sim.step(n_macro)
        Tc, _ = sim.temperature(0)
        Tf, origin = sim.temperature(1)
        led, st = sim.ledger(), sim.stats()
    finally:
        sim.close()
    return Tc, Tf, origin, led, st


def _check_vs_oracle(wl, n_macro, tol, coupling):
    Tc, Tf, origin, led, st = _run(_with(wl, coupling), n_macro)
    # the oracle runs the Dirichlet-Neumann iteration (for either form of
    # the correction) or the alternate formulation, converged far below the
    # GPU path's tolerances
    orc = oracle.run(_with(wl, coupling), n_macro, newton_tol=1e-10, dn_tol=1e-10)
    oc, of, oorigin = oracle_fields(orc)
    assert origin == oorigin
    ec, ef = rel_maxerr(Tc, oc), rel_maxerr(Tf, of)
    say("  rel err coarse", ec, "fine", ef, "newton", st["newton_fine"],
        "cg", st["cg_fine"], "solves", st["fine_solves"])
    assert ec <= tol and ef <= tol
    lhs = led["stored"] - led["stored0"]
    rhs = led["absorbed"] - led["bottom"] - led["surface"] + led["remap"]
    assert abs(lhs - rhs) <= 1e-8 * abs(led["absorbed"])
    assert led["absorbed"] == pytest.approx(orc.ledger["absorbed"], rel=1e-12)
    assert led["stored"] == pytest.approx(orc.ledger["stored"], rel=max(tol, 1e-9))
    assert led["bottom"] == pytest.approx(orc.ledger["bottom"], rel=max(tol, 1e-7),
                                          abs=1e-9 * abs(led["absorbed"]))
    assert st["window_moves"] == orc.stats["moves"]
    if coupling == W.COMPOSITE:   # one solve per macro step
        assert st["dn_iters"] == n_macro
    elif coupling in (W.DN, W.CONSISTENT):
        assert st["dn_iters"] >= n_macro
    else:                         # no correction to iterate
        assert st["dn_iters"] == 0
    return led, orc


COUPLINGS = [pytest.param(W.COMPOSITE, id="composite"), pytest.param(W.DN, id="dn")]


@pytest.mark.parametrize("coupling", COUPLINGS)
def test_single_track_1mm_fp64(coupling):
    _check_vs_oracle(W.single_track_1mm(), 20, 1e-9, coupling)


@pytest.mark.parametrize("coupling", COUPLINGS)
def test_single_track_1mm_mixed(coupling):
    _check_vs_oracle(W.single_track_1mm(W.MIXED), 20, 1e-6, coupling)


@pytest.mark.parametrize("coupling", COUPLINGS)
@pytest.mark.parametrize("name", ["r1m1", "r3m2", "fulldepth", "corner"])
def test_small_cases_fp64(name, coupling):
    wl = W.small_cases()[name]
    _check_vs_oracle(wl, wl.n_macro, 1e-9, coupling)


# The path starts at t = 0.1 ms (beam off for the first two macro steps)
# and its track ends at 0.725 ms, partway through macro step 14: loads
# switch on and off inside macro steps, the window follows the beam five
# times and stays where it is while the beam is off.
@pytest.mark.parametrize("coupling", COUPLINGS)
def test_beam_off_before_and_after_the_path(coupling):
    base = W.single_track_1mm()
    tr = replace(base.scan.tracks[0], x1=0.6e-3)
    wl = replace(base, name="beam_off", n_macro=17,
                 scan=W.ScanPath([tr], t_start=0.1e-3))
    led, orc = _check_vs_oracle(wl, wl.n_macro, 1e-9, coupling)
    assert orc.stats["moves"] == 5
    # eta P over the 0.625 ms the beam is on (the face quadrature of a
    # 50 um spot on 31 um faces integrates it to within a few per cent)
    assert led["absorbed"] == pytest.approx(0.4 * 180.0 * 0.625e-3, rel=0.05)


# No heat input: every node keeps the plate temperature (the oracle's field
# is exactly 300 K), while the window still follows the beam.
@pytest.mark.parametrize("coupling", COUPLINGS)
def test_zero_power_keeps_the_plate_temperature(coupling):
    base = W.single_track_1mm()
    tr = replace(base.scan.tracks[0], power=0.0)
    wl = _with(replace(base, name="zero_power", scan=W.ScanPath([tr])), coupling)
    Tc, Tf, origin, led, st = _run(wl, 6)
    orc = oracle.run(wl, 6, newton_tol=1e-10, dn_tol=1e-10)
    oc, of, oorigin = oracle_fields(orc)
    assert origin == oorigin and st["window_moves"] == orc.stats["moves"] == 1
    T0 = wl.material.T_init
    assert np.all(oc == T0) and np.all(of == T0)
    assert np.abs(Tc - T0).max() <= 1e-9 and np.abs(Tf - T0).max() <= 1e-9
    assert led["absorbed"] == 0.0
    assert np.isfinite(led["stored"]) and np.isfinite(led["bottom"])


@pytest.mark.parametrize("coupling", COUPLINGS)
@pytest.mark.parametrize("prec, tol", [(W.FP64, 1e-9), (W.MIXED, 1e-6)])
def test_surface_loss(prec, tol, coupling):
    wl = W.single_track_1mm(prec)
    wl = replace(wl, material=replace(wl.material, h_conv=2.0e4, emissivity=0.8, T_amb=300.0))
    led, orc = _check_vs_oracle(wl, 12, tol, coupling)
    assert led["surface"] > 0.0
    assert led["surface"] == pytest.approx(orc.ledger["surface"], rel=max(tol, 1e-9))


# the paper's volumetric local source and smeared global source, on its 3D
# single-track example
@pytest.mark.parametrize("coupling", COUPLINGS)
@pytest.mark.parametrize("prec, tol", [(W.FP64, 1e-9), (W.MIXED, 1e-6)])
def test_single_track_3d_volume_sources(prec, tol, coupling):
    wl = W.single_track_3d(prec)
    led, orc = _check_vs_oracle(wl, wl.n_macro, tol, coupling)
    assert led["absorbed"] == pytest.approx(0.38 * 179.2 * 2.5e-3, rel=1e-4)


# the paper's alternate global formulation (a different discrete problem:
# the oracle runs the same formulation)
@pytest.mark.parametrize("prec, tol", [(W.FP64, 1e-9), (W.MIXED, 1e-6)])
@pytest.mark.parametrize("name", ["single_track_1mm", "single_track_3d"])
def test_alternate_formulation(name, prec, tol):
    wl = W.single_track_1mm(prec) if name == "single_track_1mm" else W.single_track_3d(prec)
    wl = replace(wl, material=replace(wl.material, h_conv=1.0e4))
    _check_vs_oracle(wl, min(wl.n_macro, 12), tol, W.ALTERNATE)


# degenerate window: it covers the whole plate, so there is no interface
# (the correction reduces to the fine solve; the composite pair's coarse
# side has no free node)
@pytest.mark.parametrize("coupling", COUPLINGS)
def test_whole_plate_window(coupling):
    UM = 1e-6
    wl = W.single_track_1mm()
    mesh = replace(wl.mesh, nx=6, ny=4, nz=3, lx=6 * 62.5 * UM, ly=4 * 62.5 * UM,
                   lz=3 * 62.5 * UM, win_nx=6, win_ny=4, win_nz=3)
    tr = W.Track(0.05e-3, 0.1e-3, 0.3e-3, 0.15e-3, 0.8, 150.0, 50 * UM, 0.4)
    wl = replace(wl, mesh=mesh, scan=W.ScanPath([tr]), n_macro=4)
    _check_vs_oracle(wl, 4, 1e-9, coupling)


# the largest micro-step count (the coarse load averages 32 laser positions)
@pytest.mark.parametrize("coupling", COUPLINGS)
def test_max_micro_steps(coupling):
    wl = W.single_track_1mm()
    wl = replace(wl, options=replace(wl.options, m_time=32, dt_coarse=64e-6), n_macro=3)
    _check_vs_oracle(wl, 3, 1e-9, coupling)


def test_composite_equals_dn_on_gpu():
    """The two GPU forms agree with each other (single_track_1mm, FP64)."""
    a = _run(_with(W.single_track_1mm(), W.COMPOSITE), 20)
    b = _run(_with(W.single_track_1mm(), W.DN), 20)
    assert rel_maxerr(a[0], b[0]) <= 1e-9 and rel_maxerr(a[1], b[1]) <= 1e-9


# every reduction sums in a fixed order (no atomics), so two runs agree bit
# for bit: a race in a kernel would show up here
@pytest.mark.parametrize("prec", [W.FP64, W.MIXED])
def test_run_to_run_bitwise(prec):
    wl = replace(W.small_cases()["corner"], options=replace(
        W.small_cases()["corner"].options, precision=prec))
    a = _run(wl, 8)
    b = _run(wl, 8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[3] == b[3]          # ledgers
    assert a[4]["cg_fine"] == b[4]["cg_fine"]


@pytest.mark.parametrize("coupling", COUPLINGS)
def test_checkpoint_roundtrip_bitwise(coupling):
    wl = _with(W.small_cases()["corner"], coupling)
    a = tl.Sim(wl)
    a.step(3)
    blob = tl.tl_save(a.h)
    a.step(4)
    Ta, _ = a.temperature(1)
    Ca, _ = a.temperature(0)
    b = tl.Sim(wl)
    tl.tl_load(b.h, blob)
    b.step(4)
    Tb, _ = b.temperature(1)
    Cb, _ = b.temperature(0)
    assert np.array_equal(Ta, Tb) and np.array_equal(Ca, Cb)
    a.close()
    b.close()



# tl_load rejects a damaged or foreign buffer before it changes anything:
# the handle then continues exactly like one that was never touched.
def test_checkpoint_rejects_damaged_or_foreign_data():
    import struct
    wl = _with(W.small_cases()["corner"], W.DN)
    a, b = tl.Sim(wl), tl.Sim(wl)
    a.step(3)
    b.step(3)
    blob = tl.tl_save(a.h)
    # header: magic[8], version, I0, J0, gc_n, gf_n, n_gamma, ncols (int32)
    n_gamma, ncols = struct.unpack_from("<ii", blob, 28)
    assert ncols > 0 and n_gamma > 0    # the DN iteration's secant pairs
    wrong_len = bytearray(blob)
    struct.pack_into("<i", wrong_len, 28, n_gamma - 1)
    bad_window = bytearray(blob)
    struct.pack_into("<i", bad_window, 12, 10 ** 6)
    damaged = [blob[:40], b"X" + blob[1:], blob[:-8], bytes(wrong_len), bytes(bad_window)]
    other = W.small_cases()["r3m2"]
    c = tl.Sim(_with(other, W.DN))
    c.step(1)
    damaged.append(tl.tl_save(c.h))     # another grid
    c.close()
    for data in damaged:
        with pytest.raises(tl.TLError) as e:
            tl.tl_load(b.h, data)
        assert e.value.status == tl.TL_EINVAL
    a.step(2)
    b.step(2)
    for level in (0, 1):
        assert np.array_equal(a.temperature(level)[0], b.temperature(level)[0])
    sa, sb = a.stats(), b.stats()
    for key in ("newton_fine", "newton_coarse", "cg_fine", "cg_coarse", "dn_iters",
                "window_moves", "fine_dof_steps"):
        assert sa[key] == sb[key], key
    a.close()
    b.close()

# CG budget of 2 iterations per direction (below what cg_rtol needs): every
# direction is cut, so Newton may stop only after two accepted steps within
# tol; the result still meets the FP64 bar
@pytest.mark.parametrize("coupling", COUPLINGS)
def test_small_cg_budget(coupling):
    wl = W.single_track_1mm()
    wl = replace(wl, options=replace(wl.options, cg_max=2))
    _check_vs_oracle(wl, 8, 1e-9, coupling)


# the consistent global formulation of Section 3: the global problem on
# every coarse element, with constant coefficients of its own inside the
# window (the law's values at T_init, or given ones), loaded there by the
# local solution
FICT = [pytest.param(0.0, 0.0, id="law-at-T_init"), pytest.param(50.0, 2.0e6, id="given")]


@pytest.mark.parametrize("k_fict, rhoc_fict", FICT)
@pytest.mark.parametrize("prec, tol", [(W.FP64, 1e-9), (W.MIXED, 1e-6)])
def test_consistent_formulation_single_track(prec, tol, k_fict, rhoc_fict):
    wl = W.single_track_1mm(prec)
    wl = replace(wl, material=replace(wl.material, h_conv=1.0e4, k_fict=k_fict,
                                      rhoc_fict=rhoc_fict))
    _check_vs_oracle(wl, 12, tol, W.CONSISTENT)


@pytest.mark.parametrize("name", ["r1m1", "r3m2", "fulldepth", "corner"])
def test_consistent_formulation_small_cases(name):
    wl = W.small_cases()[name]
    wl = replace(wl, material=replace(wl.material, k_fict=50.0, rhoc_fict=2.0e6))
    _check_vs_oracle(wl, wl.n_macro, 1e-9, W.CONSISTENT)


def test_consistent_formulation_volume_sources():
    wl = W.single_track_3d()
    _check_vs_oracle(wl, wl.n_macro, 1e-9, W.CONSISTENT)


def test_consistent_equal_levels_is_single_level():
    """r = 1, m = 1: the global field is the single-level solution on the
    whole plate, inside the window too (Section 3's stronger consistency)."""
    wl = W.small_cases()["r1m1"]
    wl = replace(wl, material=replace(wl.material, k_fict=50.0, rhoc_fict=2.0e6))
    Tc, Tf, _, _, st = _run(_with(wl, W.CONSISTENT), wl.n_macro)
    ref = oracle.twolevel.single_level_run(oracle.twolevel.coarse_grid(wl.mesh), wl.material,
                                           wl.scan, wl.options.dt_coarse, wl.n_macro,
                                           tol=1e-11)[-1]
    c = oracle.twolevel.coarse_grid(wl.mesh)
    e = rel_maxerr(Tc, ref.reshape(c.shape))
    say("  consistent r = 1, m = 1 vs single level:", e, "moves", st["window_moves"])
    assert e <= 1e-9
    assert st["window_moves"] >= 1
