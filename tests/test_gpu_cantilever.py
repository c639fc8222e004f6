"""The neo-Hookean cantilever at reduced sizes against the oracle's
converged solutions (tests/golden/cantilever_*.npz, written by
tests/golden/make_cantilever_solutions.py, which calls only the oracle).

10 x 1 x 1 m, clamped at x = 0, dead shear tau = 750 Pa on x = 10 m in 10
equal increments, E = 1 MPa, nu = 0.45 (total Lagrangian neo-Hookean law,
Appendix B).  The GPU path runs the FP32 AMG preconditioner inside FGMRES
(forcing term 1e-3), iterating past the usual Newton tolerance (rtol 1e-10
per increment) so that the comparison measures the solver and not the
stopping rule; the stored oracle solution is converged with the exact
Jacobian action to 1e-9, near its residual's rounding floor.  Bar: relative
L2 displacement error <= 1e-8.

The solves use a restart length of 200: on this slender problem the bending
modes are poorly represented by the component-wise approximate Jacobian and
restarting discards the long recurrence GMRES needs for them (the test
below compares 50 and 200); the basis memory is small next to the GPU's
HBM.
"""

import os

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare, residual

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(shape):
    path = os.path.join(GOLDEN, "cantilever_%dx%dx%d.npz" % shape)
    if not os.path.exists(path):
        pytest.skip("oracle solution %s not generated" % os.path.basename(path))
    return np.load(path)


@pytest.mark.parametrize("shape", [(200, 20, 2), (400, 40, 4)])
def test_cantilever_vs_oracle(lib, shape):
    ref = _load(shape)
    cfg = mg.config_c3(*shape)
    m, mat = cfg["mesh"], cfg["material"]
    gm = lib.create_mesh(m, mat)
    restart = 200
    work = lib.make_workspace(gm, 1, restart=restart, precond=lib.PC_AMG32)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    opts = lib.newton_opts(n_increments=10, max_newton_it=30, rtol=1e-10, eta=1e-3, restart=restart,
                           max_it=200000, precond="amg32", cheb_degree=3, stol=1e-12)
    st, stats = lib.newton_solve(gm, opts, u, work)
    ug = gm.to_external(u).cpu().numpy().reshape(-1, 3)
    uo = ref["u"]
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    pr = prepare(m, mat)
    r_end = np.linalg.norm(residual(ug.reshape(-1), pr, 1.0))
    r_ref = np.linalg.norm(residual(uo.reshape(-1), pr, 1.0))
    print(shape, "rel L2 vs oracle %.2e" % err, "tip u_y %.4f (oracle %.4f)" % (ug[:, 1].max(), uo[:, 1].max()),
          "|R| gpu %.2e oracle %.2e" % (r_end, r_ref), stats, flush=True)
    assert st == lib.OK
    assert err <= 1e-8
    gm.close()


def test_restart_length_on_the_cantilever(lib):
    """The first linear solve of the 200x20x2 cantilever (J at rest, the
    bending response to the first load increment) to the forcing term 1e-3
    with FGMRES(50), the configured length, and FGMRES(200): both reach it;
    the longer basis needs fewer Arnoldi steps (restarting discards the
    slowly converging bending directions)."""
    cfg = mg.config_c3(200, 20, 2)
    gm = lib.create_mesh(cfg["mesh"], cfg["material"])
    res = {}
    for restart in (50, 200):
        work = lib.make_workspace(gm, 1, restart=restart, precond=lib.PC_AMG32)
        u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
        R = torch.empty_like(u)
        lib.residual(gm, 0.1, u, R, work)
        x = torch.zeros_like(u)
        opts = lib.gmres_opts(restart=restart, max_it=5000, rtol=1e-3, precond=lib.PC_AMG32)
        st, stats = lib.gmres(gm, 0.1, u, R, -R, x, opts, work)
        res[restart] = (st, stats["gmres_it"], stats["res_final"] / stats["res0"])
        del work
    print("restart 50:", res[50], " restart 200:", res[200], flush=True)
    assert res[200][0] == lib.OK and res[50][0] == lib.OK
    assert res[200][1] <= res[50][1]
    gm.close()
