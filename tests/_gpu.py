"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_maxerr(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def oracle_fields(sim):
    """Oracle fields reshaped like the GPU output (nz+1, ny+1, nx+1)."""
    c, f = sim.coarse, sim.win.fine
    return sim.Tc.reshape(c.shape), sim.Tf.reshape(f.shape), sim.fine_origin()
