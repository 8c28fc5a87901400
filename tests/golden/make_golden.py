"""Write oracle reference fields for the full-size parity tests.

Runs the FP64 CPU oracle (converged to 1e-10 K in Newton and in the
two-level iteration) on the first macro steps of a workload and stores, at
each requested step count, the coarse and fine temperatures, the window
origin and the energy ledger in tests/golden/<name>_n<steps>.npz.  Nothing
here touches the GPU library.

Usage:
  python tests/golden/make_golden.py single_track_2mm 20
  python tests/golden/make_golden.py raster_10mm 20 --snap 2,20
  python tests/golden/make_golden.py served_tracks 4 --requests 0,1,2
    (requests q of the served stream, each alone, after 4 macro steps:
     tests/golden/served_req<q>_n4.npz)
  python tests/golden/make_golden.py single_track_2mm 20 --snap 3,20 --coupling consistent
    (another two-level correction: tests/golden/<name>_<coupling>_n<steps>.npz)
"""
from dataclasses import replace
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def save(sim, name, steps):
    c, f = sim.coarse, sim.win.fine
    led = sim.ledger
    out = os.path.join(HERE, f"{name}_n{steps}.npz")
    np.savez_compressed(out, Tc=sim.Tc.reshape(c.shape), Tf=sim.Tf.reshape(f.shape),
                        origin=np.array(sim.fine_origin()), steps=steps,
                        stored=led["stored"], stored0=led["stored0"],
                        absorbed=led["absorbed"], bottom=led["bottom"], remap=led["remap"],
                        surface=led["surface"], dn_iters=sim.stats["dn_iters"],
                        moves=sim.stats["moves"])
    print("wrote", out, os.path.getsize(out), "bytes", flush=True)


def run(wl, name, steps, snaps):
    t0 = time.time()
    sim = oracle.TwoLevel(wl, newton_tol=1e-10, dn_tol=1e-10)
    for n in range(1, steps + 1):
        sim.step()
        print(f"{name}: macro step {n}/{steps} done after {time.time() - t0:.0f} s "
              f"(moves {sim.stats['moves']})", flush=True)
        if n in snaps:
            save(sim, name, n)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("steps", type=int)
    ap.add_argument("--snap", default=None,
                    help="comma-separated step counts to store (default: the last)")
    ap.add_argument("--requests", default="0",
                    help="served_tracks: comma-separated request numbers")
    ap.add_argument("--coupling", default=None, choices=["dn", "alternate", "consistent"],
                    help="two-level correction other than the workload's (composite)")
    a = ap.parse_args()
    snaps = {a.steps} if a.snap is None else {int(s) for s in a.snap.split(",")}
    if a.name == "served_tracks":
        stream = W.served_tracks(64, seed=0)
        for q in (int(s) for s in a.requests.split(",")):
            wl = stream[q][1]
            run(wl, wl.name, min(a.steps, wl.n_macro), snaps)
        return
    wl = W.by_name(a.name)
    name = a.name
    if a.coupling is not None:
        code = {"dn": W.DN, "alternate": W.ALTERNATE, "consistent": W.CONSISTENT}[a.coupling]
        wl = replace(wl, options=replace(wl.options, coupling=code))
        name = f"{a.name}_{a.coupling}"
    run(wl, name, a.steps, snaps)


if __name__ == "__main__":
    main()
