"""GPU parity: the HIP path against the FP64 CPU oracle on the same seeded
inputs.  Tolerances: FP64 path 1e-9 and mixed path 1e-6 relative max-norm
temperature error (relative to the oracle's max temperature); the operator
apply 1e-12 (FP64) and 1e-5 (FP32) relative to the magnitude of its terms."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from oracle import grid as G
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


# the last shape has more tiles (2508) than workgroups, so every workgroup
# loops over several tiles
@pytest.mark.parametrize("cells", [(13, 9, 5), (40, 33, 21), (160, 150, 20)])
@pytest.mark.parametrize("prec", [W.FP64, W.MIXED])
def test_op_apply_matches_assembled_operator(cells, prec):
    nx, ny, nz = cells
    say("op_apply", cells, prec)
    h = (5.3e-6, 4.1e-6, 6.7e-6)
    g = G.Grid(nx, ny, nz, *h)
    rng = np.random.default_rng(7)
    d = rng.uniform(1e-4, 1e-3, g.n_nodes)
    kap = rng.uniform(10.0, 30.0, g.n_elems)
    v = rng.normal(300.0, 50.0, g.n_nodes)
    K = G.stiffness(g, kap)
    y_ref = d * v + K @ v
    scale = np.abs(d * v) + abs(K) @ np.abs(v)
    dt = torch.float64 if prec == W.FP64 else torch.float32
    grid = tl.to_grid(nx, ny, nz, *h)
    npad = tl.tl_op_padded_size(grid)
    dev = lambda a: torch.tensor(a, dtype=dt, device="cuda")
    pads = [torch.empty(npad, dtype=dt, device="cuda") for _ in range(4)]
    tl.tl_op_pack(grid, 0, dev(d), pads[0])
    tl.tl_op_pack(grid, 1, dev(kap), pads[1])
    tl.tl_op_pack(grid, 0, dev(v), pads[2])
    tl.tl_op_apply(grid, prec, pads[0], pads[1], pads[2], pads[3])
    y = torch.empty(g.n_nodes, dtype=dt, device="cuda")
    tl.tl_op_unpack(grid, 0, pads[3], y)
    err = np.abs(y.cpu().numpy().astype(np.float64) - y_ref) / scale
    tol = 1e-12 if prec == W.FP64 else 2e-6
    assert err.max() < tol, err.max()


def _op_rows(g, Ke, d, kap, v, nodes):
    """y_i = d_i v_i + sum over the elements e around node i of
    kap_e (K_e v_e)_i, one sampled node at a time (plain loops)."""
    out, scale = [], []
    for (i, j, k) in nodes:
        y = d[g.node(i, j, k)] * v[g.node(i, j, k)]
        s = abs(y)
        for ez in (0, 1):
            for ey in (0, 1):
                for ex in (0, 1):
                    ei, ej, ek = i - ex, j - ey, k - ez
                    if not (0 <= ei < g.nx and 0 <= ej < g.ny and 0 <= ek < g.nz):
                        continue
                    ke = kap[ei + g.nx * (ej + g.ny * ek)]
                    a = ex + 2 * ey + 4 * ez   # the node's corner in element e
                    for c in range(8):
                        cx, cy, cz = c & 1, (c >> 1) & 1, c >> 2
                        vc = v[g.node(ei + cx, ej + cy, ek + cz)]
                        y += ke * Ke[a, c] * vc
                        s += abs(ke * Ke[a, c] * vc)
        out.append(y)
        scale.append(s)
    return np.array(out), np.array(scale)


# more than 4M nodes: the z-marching kernel, with ragged column tiles in x
# (301 = 4 x 64 + 45) and y (121 = 30 x 4 + 1) and a short last z run
@pytest.mark.parametrize("prec", [W.FP64, W.MIXED])
def test_op_apply_large_grid_sampled(prec):
    nx, ny, nz = 300, 120, 118
    say("op_apply large", (nx, ny, nz), prec)
    h = (5.3e-6, 4.1e-6, 6.7e-6)
    g = G.Grid(nx, ny, nz, *h)
    assert g.n_nodes > 4 * 2**20
    rng = np.random.default_rng(11)
    d = rng.uniform(1e-4, 1e-3, g.n_nodes)
    kap = rng.uniform(10.0, 30.0, g.n_elems)
    v = rng.normal(300.0, 50.0, g.n_nodes)
    dt = torch.float64 if prec == W.FP64 else torch.float32
    grid = tl.to_grid(nx, ny, nz, *h)
    npad = tl.tl_op_padded_size(grid)
    dev = lambda a: torch.tensor(a, dtype=dt, device="cuda")
    pads = [torch.empty(npad, dtype=dt, device="cuda") for _ in range(4)]
    tl.tl_op_pack(grid, 0, dev(d), pads[0])
    tl.tl_op_pack(grid, 1, dev(kap), pads[1])
    tl.tl_op_pack(grid, 0, dev(v), pads[2])
    tl.tl_op_apply(grid, prec, pads[0], pads[1], pads[2], pads[3])
    y = torch.empty(g.n_nodes, dtype=dt, device="cuda")
    tl.tl_op_unpack(grid, 0, pads[3], y)
    y = y.cpu().numpy().astype(np.float64)
    if prec != W.FP64:   # the reference takes the inputs the kernel saw
        d, kap, v = (a.astype(np.float32).astype(np.float64) for a in (d, kap, v))
    # every corner and edge class of the domain and of the tiles, plus random
    xs = sorted({0, 1, 63, 64, 65, 127, 128, 255, 256, 299, 300})
    ys = sorted({0, 1, 3, 4, 5, 59, 60, 116, 119, 120})
    zs = sorted({0, 1, 8, 9, 17, 18, 116, 117, 118})
    nodes = [(i, j, k) for i in xs for j in ys for k in zs]
    nodes += [tuple(int(t) for t in rng.integers(0, (nx + 1, ny + 1, nz + 1)))
              for _ in range(300)]
    ref, scale = _op_rows(g, G.element_stiffness(*h), d, kap, v, nodes)
    got = np.array([y[g.node(*n)] for n in nodes])
    err = np.abs(got - ref) / scale
    tol = 1e-12 if prec == W.FP64 else 2e-6
    assert err.max() < tol, err.max()


def _run_pair(wl, n_macro):
    say("case", wl.name, "precision", wl.options.precision, "macro steps", n_macro)
    sim = tl.Sim(wl)
    try:
        sim.step(n_macro)
        Tc, _ = sim.temperature(0)
        Tf, origin = sim.temperature(1)
        led, st = sim.ledger(), sim.stats()
    finally:
        sim.close()
    # the reference is converged far below the GPU path's tolerances
    orc = oracle.run(wl, n_macro, newton_tol=1e-10, dn_tol=1e-10)
    oc, of, oorigin = oracle_fields(orc)
    return (Tc, Tf, origin, led, st), (oc, of, oorigin, orc)


def _check(gpu, ref, tol):
    Tc, Tf, origin, led, st = gpu
    oc, of, oorigin, orc = ref
    assert origin == oorigin
    ec, ef = rel_maxerr(Tc, oc), rel_maxerr(Tf, of)
    say("  rel err coarse", ec, "fine", ef, "dn", st["dn_iters"], orc.stats["dn_iters"])
    assert ec <= tol and ef <= tol
    # ledger identity on the device and agreement with the oracle's ledger
    lhs = led["stored"] - led["stored0"]
    rhs = led["absorbed"] - led["bottom"] - led["surface"] + led["remap"]
    assert abs(lhs - rhs) <= 1e-8 * abs(led["absorbed"])
    assert led["absorbed"] == pytest.approx(orc.ledger["absorbed"], rel=1e-12)
    # the stored energy is a mass-weighted sum of H(T), so it carries the
    # temperature bar of the path
    assert led["stored"] == pytest.approx(orc.ledger["stored"], rel=max(tol, 1e-9))
    assert st["window_moves"] == orc.stats["moves"]


def test_config0_fp64():
    gpu, ref = _run_pair(W.config0(), 20)
    _check(gpu, ref, 1e-9)


@pytest.mark.parametrize("name", ["r1m1", "r3m2", "fulldepth", "corner"])
def test_small_cases_fp64(name):
    wl = W.small_cases()[name]
    gpu, ref = _run_pair(wl, wl.n_macro)
    _check(gpu, ref, 1e-9)


def test_config0_mixed():
    gpu, ref = _run_pair(W.config0(W.MIXED), 20)
    _check(gpu, ref, 1e-6)


# Top-surface loss (convection on both levels, radiation on the fine one),
# strong enough to move the field well beyond the parity bar
@pytest.mark.parametrize("prec, tol", [(W.FP64, 1e-9), (W.MIXED, 1e-6)])
def test_config0_surface_loss(prec, tol):
    wl = W.config0(prec)
    wl = replace(wl, material=replace(wl.material, h_conv=2.0e4, emissivity=0.8, T_amb=300.0))
    gpu, ref = _run_pair(wl, 12)
    _check(gpu, ref, tol)
    led, orc = gpu[3], ref[3]
    assert led["surface"] > 0.0
    assert led["surface"] == pytest.approx(orc.ledger["surface"], rel=max(tol, 1e-9))


def test_checkpoint_roundtrip_bitwise():
    wl = W.small_cases()["corner"]
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
    assert tl.tl_get_time(b.h)[1] == 7
    a.close()
    b.close()


def test_nonconvergence_rolls_back():
    wl = W.config0()
    sim = tl.Sim(replace(wl, options=replace(wl.options, newton_max=1)))
    T0, _ = sim.temperature(1)
    with pytest.raises(tl.TLError) as e:
        sim.step(1)
    assert e.value.status == tl.TL_ENOCONV
    T1, _ = sim.temperature(1)
    assert np.array_equal(T0, T1)
    assert tl.tl_get_time(sim.h)[1] == 0
    sim.close()
