"""Failure paths of the solvers, each forced from the host so that every
kernel runs to its normal end and the status travels back through the C ABI.

  E_NAN           a NaN in the initial displacement (the first residual is NaN)
  E_NOT_CONVERGED one Newton iteration allowed with a tight tolerance; a GMRES
                  run capped at two Arnoldi steps
  E_BREAKDOWN     no displacement patch: J is singular (rigid-body modes) and a
                  net applied force is outside its range, so the true residual
                  stops decreasing
  E_DIVERGED      a divergence tolerance below 1: the first residual check
                  already finds |R| > dtol |R(u_0)|
The oracle's Newton takes the same decisions on the same inputs (checked
where its cost is small).
"""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare
from oracle.newton import newton_solve as o_newton

pytestmark = pytest.mark.gpu


def _block(law="linear_elastic", clamp=True, tau=2.0e4):
    m = mg.box_mesh_3d(8, 5, 4, 1.0, 0.6, 0.5, jitter=0.1, seed=11)
    if clamp:
        mg.set_patch(m, "xmin", "displacement", (0.0, 0.0, 0.0))
    mg.set_patch(m, "xmax", "traction", (0.0, tau, 0.0))
    E = 200e9 if law == "linear_elastic" else 1.0e6
    return m, mg.Material(law, E, 0.3)


def _setup(lib, m, mat, restart=20):
    gm = lib.create_mesh(m, mat)
    work = lib.make_workspace(gm, 1, restart=restart, precond=lib.PC_JACOBI)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    return gm, work, u


def test_nan_in_state(lib):
    m, mat = _block()
    gm, work, u = _setup(lib, m, mat)
    u[5] = float("nan")
    opts = lib.newton_opts(max_newton_it=5, rtol=1e-8, eta=1e-6, restart=20, max_it=200, precond="jacobi")
    st, stats = lib.newton_solve(gm, opts, u, work, allow=(lib.E_NAN,))
    assert st == lib.E_NAN
    assert stats["newton_it"] == 0
    assert not np.isfinite(stats["res_final"])
    assert b"NaN" in lib._lib.jfnk_last_error()
    gm.close()


def test_newton_iteration_limit(lib):
    m, mat = _block("neo_hookean", tau=2.0e4)
    gm, work, u = _setup(lib, m, mat)
    opts = lib.newton_opts(max_newton_it=1, rtol=1e-12, eta=1e-3, restart=20, max_it=400, precond="jacobi")
    st, stats = lib.newton_solve(gm, opts, u, work)
    assert st == lib.E_NOT_CONVERGED
    assert stats["newton_it"] == 1
    assert np.isfinite(stats["res_final"]) and stats["res_final"] > 1e-12 * stats["res0"]
    # the output holds the last iterate: one Newton step away from zero
    assert torch.isfinite(u).all() and float(u.abs().max()) > 0
    pr = prepare(m, mat)
    _, so = o_newton(pr, rtol=1e-12, max_newton_it=1, eta=1e-3, restart=20, precond="jacobi")
    assert so["status"] == "not_converged"
    gm.close()


def test_gmres_iteration_limit(lib):
    m, mat = _block()
    gm, work, u = _setup(lib, m, mat)
    R = torch.empty_like(u)
    lib.residual(gm, 1.0, u, R, work)
    b = -R
    x = torch.zeros_like(u)
    opts = lib.gmres_opts(restart=20, max_it=2, rtol=1e-14, precond=lib.PC_JACOBI)
    st, stats = lib.gmres(gm, 1.0, u, R, b, x, opts, work)
    assert st == lib.E_NOT_CONVERGED
    assert stats["gmres_it"] == 2
    assert stats["res_final"] < stats["res0"]
    gm.close()


def test_no_displacement_patch_breaks_down(lib):
    m, mat = _block(clamp=False)
    gm, work, u = _setup(lib, m, mat, restart=10)
    R = torch.empty_like(u)
    lib.residual(gm, 1.0, u, R, work)
    x = torch.zeros_like(u)
    opts = lib.gmres_opts(restart=10, max_it=5000, rtol=1e-10, precond=lib.PC_JACOBI)
    st, stats = lib.gmres(gm, 1.0, u, R, -R, x, opts, work)
    assert st == lib.E_BREAKDOWN
    assert stats["gmres_it"] < 5000
    assert b"stagnation" in lib._lib.jfnk_last_error()
    # the net force cannot be balanced: the residual keeps at least the
    # component of b along the uniform translation
    bn = (-R).view(3, -1).sum(dim=1).norm() / np.sqrt(gm.n_cells)
    assert stats["res_final"] >= 0.99 * float(bn)
    gm.close()


def test_divergence_tolerance(lib):
    m, mat = _block("neo_hookean", tau=2.0e4)
    gm, work, u = _setup(lib, m, mat)
    opts = lib.newton_opts(max_newton_it=10, rtol=1e-10, eta=1e-8, restart=20, max_it=4000,
                           precond="jacobi", dtol=0.5)
    st, stats = lib.newton_solve(gm, opts, u, work, allow=(lib.E_DIVERGED,))
    assert st == lib.E_DIVERGED
    assert stats["newton_it"] == 0
    assert float(u.abs().max()) == 0.0   # no step was taken
    assert b"diverged" in lib._lib.jfnk_last_error()
    pr = prepare(m, mat)
    _, so = o_newton(pr, rtol=1e-10, max_newton_it=10, eta=1e-8, precond="jacobi", dtol=0.5)
    assert so["status"] == "diverged"
    gm.close()
