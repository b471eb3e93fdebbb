"""Writes ellipsoid128_oracle.npz: the FP64 oracle's Dirichlet solve of the
ellipsoid workload (semi-axes 0.9, 0.7, 0.5 in [-1.2, 1.2]^3, 128^3 grid,
u = e^(x+y+z), kappa = 0, every grid-edge crossing a control point), which takes
minutes on the host and so is stored rather than recomputed inside a GPU test.

Calls only oracle/ (and the seeded input generators in synth/).  Stored: the
trace u+ at every control point, u at a seeded sample of 20000 nodes in Omega,
the oracle's GMRES iteration count and relative residual.  Regenerate with
``python tests/golden/make_ellipsoid128.py``.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import kfbi_oracle3d as O3  # noqa: E402

N = 128
AXES = (0.9, 0.7, 0.5)
TOL = 3e-12
SAMPLE = 20000
SEED = 128


def main():
    pr = synth.ellipsoid_problem(n=N, axes=AXES)
    op = O3.build_plan(N, synth.BOX_LO, synth.BOX_HI, AXES)
    fg, g = pr.boundary_data(op.q_pos)
    ref = O3.solve_bvp(op, pr.kappa, pr.f_grid, fg, g, tol=TOL, max_iter=1500)
    inside = np.flatnonzero(np.asarray(op.inside).ravel())
    pick = np.sort(np.random.default_rng(SEED).choice(inside, size=SAMPLE, replace=False))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ellipsoid128_oracle.npz")
    np.savez_compressed(out, n=N, axes=np.asarray(AXES), tol=TOL, iters=int(ref.iters), relres=float(ref.relres),
                        u_gamma=np.asarray(ref.u_gamma), node=pick.astype(np.int64),
                        u_node=np.asarray(ref.u_grid).ravel()[pick])
    print(f"wrote {out}: {ref.iters} iterations, relres {ref.relres:.3e}")


if __name__ == "__main__":
    main()
