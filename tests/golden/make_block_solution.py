"""Writes the oracle's solution of the 64^3 jittered linear-elastic block
(tests/golden/block64_solution.npz), sampled, for the GPU parity test.

Calls only ``oracle/`` (and the seeded inputs of ``meshgen``): the 1 m cube
of 64^3 hexes with +-20% node jitter (seed 2), E = 200 GPa, nu = 0.3,
clamped bottom, 10 MPa pressure on the top face (Section 2.1 boundary
classes, dead load), linear elastic (Appendix B).  The linear solve is flexible GMRES
(Section 3.2) preconditioned by the approximate Jacobian of Section 3.1
inverted exactly (its sparse LU factors; about 13 minutes and 12 GB to
factor), run far below the GPU's tolerance (1e-12 relative).  The Jacobian
action inside GMRES is the complex-step derivative, exact up to rounding for
this law: the forward difference levels off near 1e-10 of |R| on this mesh,
where GMRES would stagnate.  R is affine in u, so one Newton step is the
solution.  Stored: every 61st cell of the solution (in input cell order) and
the norms the test needs.  About 17 minutes on 8 cores (60 GMRES iterations).

Run from the repository root:  python tests/golden/make_block_solution.py
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import meshgen as mg  # noqa: E402
from oracle.fv import prepare, residual  # noqa: E402
from oracle.newton import newton_solve  # noqa: E402

STRIDE = 61


def main():
    c = mg.config_c2()
    pr = prepare(c["mesh"], c["material"])
    t0 = time.time()
    mon = lambda k, it, rel, gm: print("  Newton %d: |R|/|R0| %.2e (%d GMRES, %.0f s)" % (it, rel, gm, time.time() - t0),
                                       flush=True)
    u, st = newton_solve(pr, n_increments=1, rtol=1e-12, max_newton_it=1, eta=1e-12, restart=60,
                         precond="lu", max_krylov_it=600, monitor=mon, jv="complex_step")
    R = np.linalg.norm(residual(u, pr, 1.0))
    R0 = np.linalg.norm(residual(np.zeros_like(u), pr, 1.0))
    print("64^3 block: %.0f s, newton %s, gmres %s, |R|/|R0| %.2e" % (time.time() - t0, st["newton_it"],
                                                                   st["gmres_it"], R / R0), flush=True)
    uc = u.reshape(-1, 3)
    idx = np.arange(0, uc.shape[0], STRIDE)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "block64_solution.npz")
    np.savez_compressed(out, cells=idx, u=uc[idx], u_norm=np.linalg.norm(u), res_rel=R / R0, res0=R0)
    print("wrote", out)


if __name__ == "__main__":
    main()
