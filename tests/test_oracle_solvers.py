"""Pins for the oracle GMRES and Newton (Sections 2.2, 3.2, 3.3).

  * GMRES against a library dense solve; exact in n steps when n <= m;
  * CGS2 basis orthonormal to rounding;
  * Newton on the linear problem: one step solves it, and the result
    matches a dense solve with the brute-force Jacobian;
  * global equilibrium at convergence: the clamp reaction balances the
    applied traction;
  * hyperelastic path independence under dead loads: 4 and 8 equal
    increments reach the same state.
"""

import numpy as np
import pytest

import meshgen as mg
from oracle.fv import prepare, residual
from oracle.jacobian import brute_force_jacobian
from oracle.krylov import gmres
from oracle.newton import newton_solve


def test_gmres_matches_dense_solve():
    rng = np.random.default_rng(1)
    n = 60
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    x, info = gmres(lambda z: A @ z, b, restart=15, rtol=1e-13)
    assert info["converged"]
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)


def test_gmres_exact_in_n_steps_and_orthonormal_basis():
    rng = np.random.default_rng(2)
    n = 12
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    b = rng.standard_normal(n)
    x, info = gmres(lambda z: A @ z, b, restart=30, rtol=1e-14, keep_basis=True)
    assert info["iterations"] <= n
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    V = info["V"]
    assert np.linalg.norm(V @ V.T - np.eye(V.shape[0])) <= 1e-13


def test_gmres_right_preconditioned_same_solution():
    rng = np.random.default_rng(3)
    n = 80
    A = np.diag(np.linspace(1, 100, n)) + rng.standard_normal((n, n)) * 0.5
    b = rng.standard_normal(n)
    d = np.diag(A).copy()
    x1, i1 = gmres(lambda z: A @ z, b, restart=20, rtol=1e-12, max_it=5000)
    x2, i2 = gmres(lambda z: A @ z, b, M=lambda r: r / d, restart=20, rtol=1e-12)
    assert i2["iterations"] < i1["iterations"]
    assert np.linalg.norm(x1 - x2) <= 1e-9 * np.linalg.norm(x1)


@pytest.mark.parametrize("precond", ["jacobi", "lu", "none"])
def test_newton_linear_problem_one_step(precond):
    m = mg.box_mesh_2d(6, 5, 1.0, 1.0, jitter=0.2, seed=4)
    mg.set_patch(m, "xmin", "displacement", (0.0, 0.0))
    mg.set_patch(m, "xmax", "traction", (1e6, 0.0))
    pr = prepare(m, mg.Material("linear_elastic", 200e9, 0.3))
    u, st = newton_solve(pr, rtol=1e-6, max_newton_it=1, eta=1e-11, precond=precond, restart=30)
    assert st["newton_it"] == [1] and st["converged"]
    n = pr["nc"] * 2
    J = brute_force_jacobian(np.zeros(n), pr)
    ref = np.linalg.solve(J, -residual(np.zeros(n), pr).reshape(-1))
    assert np.linalg.norm(u - ref) <= 1e-8 * np.linalg.norm(ref)


def test_clamp_reaction_balances_applied_traction():
    """Square 1 x 1 (unit depth), 1 MPa on the right edge: reaction -1e6 N in x."""
    m = mg.box_mesh_2d(10, 10, 1.0, 1.0)
    mg.set_patch(m, "xmin", "displacement", (0.0, 0.0))
    mg.set_patch(m, "xmax", "traction", (1e6, 0.0))
    pr = prepare(m, mg.Material("linear_elastic", 200e9, 0.3))
    u, st = newton_solve(pr, rtol=1e-10, max_newton_it=2, eta=1e-11, precond="lu")
    parts_total = residual(u, pr).sum(axis=0)
    assert np.abs(parts_total).max() <= 1e-10 * 1e6   # converged: sum of cell residuals ~ 0 (N)
    # the displacement-face forces (traction + Rhie-Chow) = total minus interior and applied
    # equals -1e6 N: evaluate the clamp contribution alone by zeroing the applied load
    mg.set_patch(m, "xmax", "traction", (0.0, 0.0))
    pr0 = prepare(m, mg.Material("linear_elastic", 200e9, 0.3))
    reaction = residual(u, pr0).sum(axis=0)
    assert reaction[0] == pytest.approx(-1e6, rel=1e-9)
    assert abs(reaction[1]) <= 1e-6 * 1e6


def test_hyperelastic_dead_load_path_independence():
    m = mg.cantilever_mesh(10, 2, 2, L=(5.0, 1.0, 1.0), tau=400.0)
    pr = prepare(m, mg.Material("neo_hookean", 1e6, 0.45))
    # (FD J.v limits the attainable residual reduction to ~1e-11; rtol 1e-9 is safely above)
    u4, s4 = newton_solve(pr, n_increments=4, rtol=1e-9, max_newton_it=15, eta=1e-6, precond="lu",
                          max_krylov_it=300)
    u8, s8 = newton_solve(pr, n_increments=8, rtol=1e-9, max_newton_it=15, eta=1e-6, precond="lu",
                          max_krylov_it=300)
    assert s4["converged"] and s8["converged"]
    assert np.linalg.norm(u4 - u8) <= 1e-8 * np.linalg.norm(u8)
    # genuinely nonlinear: more than one Newton iteration per increment
    assert max(s4["newton_it"]) >= 2
    # and the tip moved substantially
    assert np.abs(u8.reshape(-1, 3)[:, 1]).max() > 0.03


# ---------------------------------------------------------------- line search (Section 3.2)
def _bent_strip(tau):
    m = mg.box_mesh_2d(12, 3, 4.0, 1.0, jitter=0.1, seed=5)
    mg.set_patch(m, "xmin", "displacement", (0.0, 0.0))
    mg.set_patch(m, "xmax", "traction", (0.0, tau))
    return prepare(m, mg.Material("neo_hookean", 1e6, 0.3))


def test_line_search_takes_the_first_halving_that_decreases_the_residual():
    """A neo-Hookean strip under a large tip shear in one increment: the full
    first Newton step (the linear solution) raises |R| by orders of magnitude;
    the step taken is the first of 1, 1/2, 1/4, ... below |R(0)|."""
    pr = _bent_strip(2e5)
    u1, _ = newton_solve(pr, rtol=1e-10, max_newton_it=1, eta=1e-12, precond="lu", restart=80)
    _, st = newton_solve(pr, rtol=1e-10, max_newton_it=1, eta=1e-12, precond="lu", restart=80,
                         line_search=True)
    s = st["steps"][0]
    r0 = np.linalg.norm(residual(np.zeros_like(u1), pr))
    assert s < 1.0
    with np.errstate(invalid="ignore"):
        assert np.linalg.norm(residual(s * u1, pr)) < r0
        k = 1.0
        while k > s:
            rk = np.linalg.norm(residual(k * u1, pr))
            assert not rk < r0, k
            k *= 0.5


def test_line_search_rescues_a_diverging_newton_solve():
    pr = _bent_strip(2e5)
    with np.errstate(invalid="ignore"):
        _, plain = newton_solve(pr, rtol=1e-6, max_newton_it=40, eta=1e-4, precond="lu", restart=80)
    _, ls = newton_solve(pr, rtol=1e-6, max_newton_it=40, eta=1e-4, precond="lu", restart=80,
                         line_search=True)
    assert plain["status"] in ("nan", "diverged", "not_converged")
    assert ls["status"] == "ok"
    assert ls["steps"][-1] == 1.0        # quadratic range reached: full steps again


def test_line_search_keeps_full_steps_when_they_decrease():
    pr = _bent_strip(1e2)
    u_a, a = newton_solve(pr, rtol=1e-8, max_newton_it=20, eta=1e-6, precond="lu", restart=80)
    u_b, b = newton_solve(pr, rtol=1e-8, max_newton_it=20, eta=1e-6, precond="lu", restart=80,
                          line_search=True)
    assert b["steps"] == [1.0] * len(b["steps"])
    assert np.array_equal(u_a, u_b)


def test_divergence_tolerance_stops_the_solve():
    pr = _bent_strip(2e3)
    u, st = newton_solve(pr, rtol=1e-10, max_newton_it=20, eta=1e-10, precond="lu", restart=80, dtol=0.5)
    assert st["status"] == "diverged" and st["newton_it"] == [0]
    assert not np.any(u)


# ---------------------------------------------------------------- GMRES variants
def test_left_preconditioned_and_augmented_gmres_reach_the_dense_solution():
    """Left preconditioning and LGMRES augmentation change the iterates, not
    the solution: both reach the dense solve; with the cycle length fixed,
    two augmentation vectors cut the iteration count of restarted GMRES."""
    rng = np.random.default_rng(11)
    n = 120
    A = np.diag(np.linspace(1.0, 400.0, n)) + rng.standard_normal((n, n)) * 0.8
    b = rng.standard_normal(n)
    d = np.diag(A).copy()
    x_ref = np.linalg.solve(A, b)
    xl, il = gmres(lambda z: A @ z, b, M=lambda r: r / d, restart=20, rtol=1e-12, left=True, max_it=4000)
    assert il["converged"]
    assert np.linalg.norm(xl - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    # same cycle length (10 directions), two of them augmentation vectors
    x0, i0 = gmres(lambda z: A @ z, b, restart=10, rtol=1e-10, max_it=20000)
    xa, ia = gmres(lambda z: A @ z, b, restart=10, rtol=1e-10, max_it=20000, augment=2)
    assert ia["converged"]
    assert np.linalg.norm(xa - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    assert ia["iterations"] < 0.8 * i0["iterations"]
