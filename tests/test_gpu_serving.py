"""Continuous batching (the served workload): each result is the same
alone and in the mix, requests arriving while others run are admitted as
slots and memory free up, and served results match the oracle."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
import workloads as W
from tests._gpu import say, rel_maxerr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2110_12932_amd import tl  # noqa: E402

UM = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tl.load()


def _requests():
    """Small two-level requests of different sizes, parameters and
    precisions."""
    base = W.single_track_1mm()
    cases = W.small_cases()
    a = replace(base, name="A", n_macro=6)
    b = replace(base, name="B", n_macro=4,
                mesh=replace(base.mesh, nx=20, lx=1.25e-3))
    c = replace(cases["corner"], name="C", n_macro=5)
    d = replace(cases["r3m2"], name="D", n_macro=5,
                options=replace(cases["r3m2"].options, precision=W.MIXED,
                                newton_tol=1e-6, dn_tol=1e-6))
    return {"A": a, "B": b, "C": c, "D": d}


def _drain(sv, max_ticks=200):
    log = []
    for _ in range(max_ticks):
        active, queued, finished = sv.tick()
        log.append((active, queued, finished))
        if active == 0 and queued == 0:
            return log
    raise AssertionError("server did not drain")


def _pool_bytes(reqs, extra=1 << 20):
    return sum(tl.tl_workspace_bytes(w.mesh, w.options) + 4096 for w in reqs) + extra


def test_result_same_alone_and_in_mix():
    R = _requests()
    say("alone: A")
    sv = tl.Server(_pool_bytes([R["A"]]), max_slots=4)
    ia = sv.submit(R["A"])
    _drain(sv)
    Ca, Fa, sa, la, _ = sv.result(ia)
    sv.close()
    say("mix: B, C first; A arrives after one tick; then D")
    sv = tl.Server(_pool_bytes(R.values()), max_slots=4)
    ib, ic = sv.submit(R["B"]), sv.submit(R["C"])
    sv.tick()
    ia2 = sv.submit(R["A"])
    sv.tick()
    idd = sv.submit(R["D"])
    log = _drain(sv)
    assert max(a for a, _, _ in log) >= 3          # their work overlapped
    Cm, Fm, sm, lm, info = sv.result(ia2)
    assert np.array_equal(Ca, Cm) and np.array_equal(Fa, Fm)
    assert la == lm
    assert sm["newton_fine"] == sa["newton_fine"] and sm["cg_fine"] == sa["cg_fine"]
    # every other request also equals its own run through a plain handle
    for rid, key in ((ib, "B"), (ic, "C"), (idd, "D")):
        Cs, Fs, _, _, _ = sv.result(rid)
        s = tl.Sim(R[key])
        s.step(R[key].n_macro)
        Cp, _ = s.temperature(0)
        Fp, _ = s.temperature(1)
        s.close()
        assert np.array_equal(Cs, Cp) and np.array_equal(Fs, Fp), key
    sv.close()


def test_heterogeneous_mix_equals_alone():
    """Requests with different two-level couplings (the consistent global
    formulation among them), laser models and precisions share the server's
    launches: each equals its own run through a plain handle."""
    base = W.single_track_1mm()
    reqs = {
        "dn": replace(base, name="dn", n_macro=4,
                      options=replace(base.options, coupling=W.DN)),
        "alt": replace(base, name="alt", n_macro=4,
                       options=replace(base.options, coupling=W.ALTERNATE)),
        "vol": replace(W.single_track_3d(), n_macro=3),
        "mixloss": replace(W.single_track_1mm(W.MIXED), name="mixloss", n_macro=4,
                           material=replace(base.material, h_conv=2e4, emissivity=0.8)),
        "cons": replace(base, name="cons", n_macro=4,
                        options=replace(base.options, coupling=W.CONSISTENT),
                        material=replace(base.material, k_fict=50.0, rhoc_fict=2.0e6)),
    }
    sv = tl.Server(_pool_bytes(reqs.values()), max_slots=5)
    ids = {k: sv.submit(w) for k, w in reqs.items()}
    log = _drain(sv)
    assert max(a for a, _, _ in log) >= 3
    for k, w in reqs.items():
        say("  heterogeneous:", k)
        Cs, Fs, _, _, _ = sv.result(ids[k])
        s = tl.Sim(w)
        s.step(w.n_macro)
        Cp, _ = s.temperature(0)
        Fp, _ = s.temperature(1)
        s.close()
        assert np.array_equal(Cs, Cp) and np.array_equal(Fs, Fp), k
    sv.close()


def test_served_results_match_oracle():
    R = _requests()
    sv = tl.Server(_pool_bytes(R.values()), max_slots=4)
    ids = {k: sv.submit(w) for k, w in R.items()}
    _drain(sv)
    for k, w in R.items():
        Cs, Fs, _, led, _ = sv.result(ids[k])
        ref = oracle.run(w, w.n_macro, newton_tol=1e-10, dn_tol=1e-10)
        ec = rel_maxerr(Cs, ref.Tc.reshape(ref.coarse.shape))
        ef = rel_maxerr(Fs, ref.Tf.reshape(ref.win.fine.shape))
        tol = 1e-9 if w.options.precision == W.FP64 else 1e-6
        say("  ", k, "rel err", ec, ef)
        assert ec <= tol and ef <= tol
        assert abs((led["stored"] - led["stored0"]) - (led["absorbed"] - led["bottom"] - led["surface"] + led["remap"])) \
            <= 1e-8 * led["absorbed"]
    sv.close()


def test_admission_respects_budget_and_drains():
    R = _requests()
    reqs = [replace(R["A"], name=f"A{q}", n_macro=3 + q % 3) for q in range(6)]
    one = tl.tl_workspace_bytes(reqs[0].mesh, reqs[0].options)
    budget = int(2.5 * one) + 4096
    sv = tl.Server(_pool_bytes(reqs), hbm_budget=budget, max_slots=8)
    ids = [sv.submit(w) for w in reqs]
    log = _drain(sv)
    assert max(a for a, _, _ in log) == 2           # the budget binds
    assert any(q > 0 for _, q, _ in log)            # requests had to wait
    assert sum(f for _, _, f in log) == len(reqs)
    infos = [sv.info(i) for i in ids]
    assert all(i["state"] == 2 for i in infos)
    # admitted in arrival order
    admits = [i["admit_s"] for i in infos]
    assert admits == sorted(admits)
    sv.close()


def test_failed_request_does_not_disturb_others():
    R = _requests()
    bad = replace(R["B"], name="bad", options=replace(R["B"].options, newton_max=1))
    sv = tl.Server(_pool_bytes([R["A"], bad]), max_slots=4)
    ia = sv.submit(R["A"])
    ib = sv.submit(bad)
    _drain(sv)
    with pytest.raises(tl.TLError) as e:
        sv.result(ib)
    assert e.value.status == tl.TL_ENOCONV
    assert sv.info(ib)["state"] == 3
    Cs, Fs, _, _, _ = sv.result(ia)
    s = tl.Sim(R["A"])
    s.step(R["A"].n_macro)
    Cp, _ = s.temperature(0)
    Fp, _ = s.temperature(1)
    s.close()
    assert np.array_equal(Cs, Cp) and np.array_equal(Fs, Fp)
    sv.close()


def test_request_errors():
    """Invalid requests are refused at submit (EINVAL), one larger than the
    budget with EBUSY; an unknown id gives EINVAL and an unfinished request
    EBUSY; none of them disturbs a valid request."""
    R = _requests()
    sv = tl.Server(_pool_bytes([R["A"]]), max_slots=2)
    bad_mesh = replace(R["A"], mesh=replace(R["A"].mesh, win_nx=R["A"].mesh.nx + 1))
    for wl, n in ((bad_mesh, None), (R["A"], 0)):
        with pytest.raises(tl.TLError) as e:
            sv.submit(wl, n)
        assert e.value.status == tl.TL_EINVAL
    small = tl.Server(tl.tl_workspace_bytes(R["A"].mesh, R["A"].options) // 2
                      + tl.tl_server_overhead_bytes(2) + 4096, max_slots=2)
    with pytest.raises(tl.TLError) as e:
        small.submit(R["A"])
    assert e.value.status == tl.TL_EBUSY
    small.close()
    ia = sv.submit(R["A"])
    with pytest.raises(tl.TLError) as e:
        sv.result(ia)           # nothing has run yet
    assert e.value.status == tl.TL_EBUSY
    with pytest.raises(tl.TLError) as e:
        sv.result(ia + 1000)
    assert e.value.status == tl.TL_EINVAL
    _drain(sv)
    Cs, Fs, _, _, _ = sv.result(ia)
    s = tl.Sim(R["A"])
    s.step(R["A"].n_macro)
    assert np.array_equal(Cs, s.temperature(0)[0]) and np.array_equal(Fs, s.temperature(1)[0])
    s.close()
    sv.close()
