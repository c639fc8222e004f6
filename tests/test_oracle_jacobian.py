"""Pins for J.v, the brute-force Jacobian and the approximate Jacobian.

  * FD J.v (Eq. JF) against the exact Jacobian within the FD error budget
    (about sqrt(eps_mach) relative for a nonlinear residual);
  * the linear law gives an affine residual: R(u) = R(0) + J u exactly,
    so one Newton step solves the problem (Section 2.2);
  * null space of the linear-elastic Jacobian with traction-only
    boundaries: rigid translations and infinitesimal rotations;
  * neo-Hookean J at u = 0 equals the linear-elastic J (Appendix B);
  * J_tilde structure: symmetric, negative diagonal, diagonally dominant,
    with hand-computed values on a 2 x 2 mesh (Section 3.1).
"""

import numpy as np
import pytest

import meshgen as mg
from oracle.fv import prepare, residual
from oracle.jacobian import (jv_fd, jv_complex_step, brute_force_jacobian, eps_walker_pernice,
                             approximate_jacobian_scalar, jv_fd_central, eps_central)


def _small(dim, law, jitter=0.2, seed=3):
    if dim == 2:
        m = mg.box_mesh_2d(4, 4, 1.0, 1.0, jitter=jitter, seed=seed)
    else:
        m = mg.box_mesh_3d(3, 3, 3, jitter=jitter, seed=seed)
    mg.set_patch(m, "xmin", "displacement", (0.0,) * dim)
    mg.set_patch(m, "xmax", "traction", (1e3, 2e3, 0.0)[:dim])
    return prepare(m, mg.Material(law, 1e6, 0.45))


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("law", ["linear_elastic", "neo_hookean"])
def test_fd_jv_against_brute_force_jacobian(dim, law):
    pr = _small(dim, law)
    n = pr["nc"] * dim
    rng = np.random.default_rng(11)
    u = rng.standard_normal(n) * 0.02
    Jbf = brute_force_jacobian(u, pr, load=0.8)
    for _ in range(3):
        v = rng.standard_normal(n)
        ref = Jbf @ v
        fd, eps = jv_fd(u, v, pr, load=0.8)
        assert eps == pytest.approx(eps_walker_pernice(u, v))
        assert np.linalg.norm(fd - ref) <= 1e-6 * np.linalg.norm(ref)
        cs = jv_complex_step(u, v, pr, load=0.8)
        assert np.linalg.norm(cs - ref) <= 1e-13 * np.linalg.norm(ref)


def test_fd_jv_scales_with_eps_for_nonlinear_law():
    """The FD error of Eq. (JF) is first order in eps (truncation-dominated range)."""
    pr = _small(3, "neo_hookean")
    n = pr["nc"] * 3
    rng = np.random.default_rng(2)
    u = rng.standard_normal(n) * 0.05
    v = rng.standard_normal(n)
    exact = jv_complex_step(u, v, pr)
    e1 = np.linalg.norm(jv_fd(u, v, pr, eps=1e-3)[0] - exact)
    e2 = np.linalg.norm(jv_fd(u, v, pr, eps=5e-4)[0] - exact)
    assert 1.8 < e1 / e2 < 2.2


def test_central_difference_is_second_order():
    """The central difference: error second order in eps (a halving of eps
    quarters it), exact for the linear law, and at its automatic step far
    closer to the exact product than the forward difference."""
    pr = _small(3, "neo_hookean")
    n = pr["nc"] * 3
    rng = np.random.default_rng(2)
    u = rng.standard_normal(n) * 0.05
    v = rng.standard_normal(n)
    exact = jv_complex_step(u, v, pr)
    e1 = np.linalg.norm(jv_fd_central(u, v, pr, eps=2e-3)[0] - exact)
    e2 = np.linalg.norm(jv_fd_central(u, v, pr, eps=1e-3)[0] - exact)
    assert 3.6 < e1 / e2 < 4.4
    c, eps = jv_fd_central(u, v, pr)
    assert eps == np.cbrt(2.0 ** -52) * np.sqrt(1.0 + np.linalg.norm(u)) / np.linalg.norm(v)
    f, _ = jv_fd(u, v, pr)
    ec = np.linalg.norm(c - exact) / np.linalg.norm(exact)
    ef = np.linalg.norm(f - exact) / np.linalg.norm(exact)
    assert ec < 1e-9 and ec < 0.05 * ef, (ec, ef)
    # hand value of the step: |u| = 3, |v| = 4 -> eps_mach^(1/3) * 2 / 4
    assert eps_central(np.array([3.0, 0.0]), np.array([0.0, 4.0])) == np.cbrt(2.0 ** -52) / 2
    # the linear law is affine in u: any step gives J v to rounding
    pl = _small(3, "linear_elastic")
    el = jv_complex_step(u, v, pl)
    assert np.linalg.norm(jv_fd_central(u, v, pl, eps=0.3)[0] - el) <= 1e-12 * np.linalg.norm(el)


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_law_residual_is_affine(dim):
    pr = _small(dim, "linear_elastic")
    n = pr["nc"] * dim
    rng = np.random.default_rng(4)
    J = brute_force_jacobian(np.zeros(n), pr)
    u = rng.standard_normal(n) * 1e-3
    R0 = residual(np.zeros(n), pr).reshape(-1)
    Ru = residual(u, pr).reshape(-1)
    assert np.linalg.norm(Ru - (R0 + J @ u)) <= 1e-12 * np.linalg.norm(Ru - R0)
    # one exact Newton step solves R(u) = 0
    du = np.linalg.solve(J, -R0)
    assert np.linalg.norm(residual(du, pr)) <= 1e-9 * np.linalg.norm(R0)


def test_linear_elastic_null_space_traction_only():
    m = mg.box_mesh_3d(3, 3, 2, jitter=0.25, seed=6)
    pr = prepare(m, mg.Material("linear_elastic", 1e6, 0.3))
    xc = pr["geo"]["xc"]
    n = pr["nc"] * 3
    J = brute_force_jacobian(np.zeros(n), pr)
    scale = np.abs(J).max()
    for k in range(3):
        t = np.zeros((pr["nc"], 3))
        t[:, k] = 1.0
        assert np.abs(J @ t.reshape(-1)).max() <= 1e-12 * scale
    W = np.array([[0.0, 1.0, -2.0], [-1.0, 0.0, 0.5], [2.0, -0.5, 0.0]])
    rot = (xc @ W.T).reshape(-1)
    assert np.abs(J @ rot).max() <= 1e-12 * scale
    # a stretch is not in the null space (control)
    st = (xc * np.array([1.0, 0.0, 0.0])).reshape(-1)
    assert np.abs(J @ st).max() > 1e-3 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_neo_hookean_jacobian_at_rest_equals_linear(dim):
    prn = _small(dim, "neo_hookean", seed=8)
    prl = _small(dim, "linear_elastic", seed=8)
    n = prn["nc"] * dim
    v = np.random.default_rng(9).standard_normal(n)
    a = jv_complex_step(np.zeros(n), v, prn)
    b = jv_complex_step(np.zeros(n), v, prl)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


def test_approximate_jacobian_structure():
    pr = _small(3, "linear_elastic", jitter=0.3)
    A = approximate_jacobian_scalar(pr).toarray()
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    d = np.diag(A)
    off = np.abs(A).sum(axis=1) - np.abs(d)
    assert np.all(d < 0)
    assert np.all(-d >= off * (1 - 1e-14))
    # strictly dominant on cells touching the clamped face
    clamp_cells = np.unique(pr["Pb"][pr["btype"] == 1])
    assert np.all(-d[clamp_cells] > off[clamp_cells] * (1 + 1e-6))


def test_approximate_jacobian_by_hand():
    """2 x 2 unit squares, left edge clamped: each internal face gives
    alpha Kbar |Delta||Gamma|/|d| = alpha Kbar off the diagonal, each clamp
    face adds alpha Kbar * 1 * 1 / 0.5 to its cell's diagonal (Section 3.1)."""
    m = mg.box_mesh_2d(2, 2, 2.0, 2.0)
    mg.set_patch(m, "xmin", "displacement", (0.0, 0.0))
    mat = mg.Material("linear_elastic", 1e6, 0.3, alpha_rc=0.3, alpha_pc=1.0)
    pr = prepare(m, mat)
    K = pr["mat"]["Kbar"]
    A = approximate_jacobian_scalar(pr).toarray()
    expect = K * np.array([[-4, 1, 1, 0], [1, -2, 0, 1], [1, 0, -4, 1], [0, 1, 1, -2]])
    assert np.allclose(A, expect, rtol=1e-14)


def test_eps_rule_hand_values():
    """Reading A1, eps = sqrt(eps_mach) sqrt(1 + |u|_2) / |v|_2, at hand-worked
    points: sqrt(eps_mach) = 2^-26 in FP64, so |u| = 3, |v| = 4 gives
    2^-26 * 2 / 4 = 2^-27 exactly; |u| = 0, |v| = 1 gives 2^-26; |u| = 8,
    |v| = 1/2 gives 6 * 2^-26.  A missing square root or another constant
    fails every one of them."""
    assert eps_walker_pernice(np.array([3.0, 0.0]), np.array([0.0, 4.0])) == 2.0 ** -27
    assert eps_walker_pernice(np.array([3.0, 0.0]), np.array([0.0, 4.0])) == 7.450580596923828e-09
    assert eps_walker_pernice(np.zeros(5), np.array([0.6, 0.8, 0.0, 0.0, 0.0])) == pytest.approx(
        2.0 ** -26, rel=1e-15)
    assert eps_walker_pernice(np.array([0.0, 8.0, 0.0]), np.array([0.3, 0.0, 0.4])) == pytest.approx(
        6.0 * 2.0 ** -26, rel=1e-15)
    assert eps_walker_pernice(np.ones(4), np.zeros(4)) == 0.0
