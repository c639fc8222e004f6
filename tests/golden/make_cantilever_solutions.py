"""Writes the oracle's converged neo-Hookean cantilever solutions that the
GPU tests compare against (tests/golden/cantilever_<nx>x<ny>x<nz>.npz).

Calls only ``oracle/`` (and the seeded inputs of ``meshgen``): the 10 x 1 x 1 m
cantilever clamped at x = 0 under a dead shear traction tau = 750 Pa on
x = 10 m (E = 1 MPa, nu = 0.45, total Lagrangian neo-Hookean law of
Appendix B), applied in 10 equal increments (Section 2.2, Eq.
NewtonRaphson with the convergence test of Section 3.3).  The oracle is
solved with the exact Jacobian action (Newton rtol 1e-9 per increment, or a
Newton correction below 1e-10 |u|, the step test of Section 3.3; full Newton
steps, linear solves to 1e-3 (the forcing term of
Section 3.2) with long-basis GMRES preconditioned by the sparse LU of the
approximate Jacobian, and the complex-step Jacobian action in place of the
finite difference).  1e-9 is near the rounding floor of the oracle's
residual: its neo-Hookean law is evaluated as written, and near the
reference state its terms of size mu |Gamma| cancel, which leaves |R| about
3.5e-10 |R(u_0)| at 200 x 20 x 2, higher at larger loads; below that
Newton cannot go, and the step test ends the increment once the
displacement no longer changes at the 1e-10 level.

Run from the repository root:  python tests/golden/make_cantilever_solutions.py 200 20 2
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

N_INCREMENTS = 10
NEWTON_RTOL = 1e-9
STOL = 1e-10
ETA = 1e-3
RESTART = 250


def solve(nx, ny, nz):
    c = mg.config_c3(nx, ny, nz, n_increments=N_INCREMENTS)
    pr = prepare(c["mesh"], c["material"])
    t0 = time.time()
    mon = lambda k, it, rel, gm: print("  increment %d, Newton %d: |R|/|R0| %.2e (%d GMRES, %.0f s)"
                                       % (k, it, rel, gm, time.time() - t0), flush=True)
    u, st = newton_solve(pr, n_increments=N_INCREMENTS, rtol=NEWTON_RTOL, eta=ETA, restart=RESTART,
                         precond="lu", max_newton_it=30, max_krylov_it=20000,
                         monitor=mon, jv="complex_step", stol=STOL)
    rel = [rf / r0 for rf, r0 in zip(st["res_final"], st["res0"])]
    R = np.linalg.norm(residual(u, pr, 1.0))
    print("%dx%dx%d: %.0f s, newton %s, gmres %s, final |R|/|R0| %s, converged %s" %
          (nx, ny, nz, time.time() - t0, st["newton_it"], st["gmres_it"],
           ["%.1e" % r for r in rel], st["converged"]), flush=True)
    assert st["converged"]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cantilever_%dx%dx%d.npz" % (nx, ny, nz))
    np.savez_compressed(out, u=u.reshape(-1, 3), newton_it=np.array(st["newton_it"]),
                        gmres_it=np.array(st["gmres_it"]), res_final=np.array(st["res_final"]),
                        res0=np.array(st["res0"]), residual_norm=R,
                        settings=np.array([N_INCREMENTS, NEWTON_RTOL, ETA, RESTART, STOL]))
    print("wrote", out, "tip u_y max %.6f m" % u.reshape(-1, 3)[:, 1].max())


if __name__ == "__main__":
    solve(*(int(a) for a in sys.argv[1:4]))
