"""Write oracle reference fields for the full-size parity tests.

Runs the FP64 CPU oracle (converged to 1e-10 K in Newton and in the
two-level iteration) on the first macro steps of a workload and stores the
coarse and fine temperatures, the window origin and the energy ledger in
tests/golden/<name>_n<steps>.npz.  Nothing here touches the GPU library.

Usage: python tests/golden/make_golden.py single_track_2mm 3
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main(name, steps):
    wl = W.by_name(name)
    t0 = time.time()
    sim = oracle.TwoLevel(wl, newton_tol=1e-10, dn_tol=1e-10)
    for n in range(steps):
        sim.step()
        print(f"{name}: macro step {n + 1}/{steps} done after {time.time() - t0:.0f} s",
              flush=True)
    c, f = sim.coarse, sim.win.fine
    led = sim.ledger
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_n{steps}.npz")
    np.savez_compressed(out, Tc=sim.Tc.reshape(c.shape), Tf=sim.Tf.reshape(f.shape),
                        origin=np.array(sim.fine_origin()), steps=steps,
                        stored=led["stored"], stored0=led["stored0"],
                        absorbed=led["absorbed"], bottom=led["bottom"], remap=led["remap"],
                        dn_iters=sim.stats["dn_iters"])
    print("wrote", out, os.path.getsize(out), "bytes")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]))
