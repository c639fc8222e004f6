"""Pins of the oracle's volume terms (Section 2.3.1): body force and BDF2
inertia (Eq. inertia2) with the Taylor predictor (Section 3.2, Eq.
predictor).

  * the manufactured-solution body force of Appendix E, derived here
    symbolically as f_b = -div sigma(u_mms) (the balance R = surface terms
    + int f_b = 0 of Section 2.2), equals the negative of the printed
    expression with its "mu_" read as mu (the printed form is +div sigma);
  * with such a body force and the manufactured displacement on the whole
    boundary, the displacement error falls at second order on regular hex
    meshes (Section 4.1, case 1 reports about 2.3);
  * a clamped block under a uniform body force: the clamp reaction
    balances the total body force (the face sums telescope);
  * a free block under a uniform body force moves rigidly, every cell
    following the scalar BDF2 recurrence worked out independently here.
"""

import numpy as np
import pytest

import meshgen as mg
from oracle.fv import prepare, residual, face_forces, with_source
from oracle.geometry import mesh_geometry
from oracle.newton import newton_solve, dynamic_solve

sp = pytest.importorskip("sympy")

AX, AY, AZ = 0.1, 0.1, 0.1
E, NU = 200e9, 0.3


def _lame():
    mu = E / (2 * (1 + NU))
    lam = E * NU / ((1 + NU) * (1 - 2 * NU))
    return mu, lam


def _mms_symbolic(k=(4, 2, 1)):
    """u_mms = a sin(k_x pi x) sin(k_y pi y) sin(k_z pi z) per component (the
    manufactured displacement whose body force Appendix E prints, for the
    default wave numbers) and f_b = -div sigma(u_mms) for the linear law."""
    x, y, z = sp.symbols("x y z")
    X = (x, y, z)
    S = sp.sin(k[0] * sp.pi * x) * sp.sin(k[1] * sp.pi * y) * sp.sin(k[2] * sp.pi * z)
    u = [AX * S, AY * S, AZ * S]
    mu, lam = _lame()
    grad = [[sp.diff(u[j], X[i]) for j in range(3)] for i in range(3)]      # grad[i][j] = d_i u_j
    div = sum(grad[i][i] for i in range(3))
    sig = [[lam * div * (1 if i == j else 0) + mu * (grad[i][j] + grad[j][i]) for j in range(3)]
           for i in range(3)]
    fb = [-sum(sp.diff(sig[i][j], X[i]) for i in range(3)) for j in range(3)]
    fu = sp.lambdify(X, u, "numpy")
    ff = sp.lambdify(X, fb, "numpy")
    return fu, ff


def _printed_appendix_e(x, y, z):
    """The body force as printed in Appendix E ("mu_" read as mu)."""
    mu, lam = _lame()
    p2 = np.pi ** 2
    s4x, c4x = np.sin(4 * np.pi * x), np.cos(4 * np.pi * x)
    s2y, c2y = np.sin(2 * np.pi * y), np.cos(2 * np.pi * y)
    s1z, c1z = np.sin(np.pi * z), np.cos(np.pi * z)
    fx = (lam * (8 * AY * p2 * c4x * c2y * s1z + 4 * AZ * p2 * c4x * c1z * s2y - 16 * AX * p2 * s4x * s2y * s1z)
          + mu * (8 * AY * p2 * c4x * c2y * s1z + 4 * AZ * p2 * c4x * c1z * s2y - 5 * AX * p2 * s4x * s2y * s1z)
          - 32 * AX * mu * p2 * s4x * s2y * s1z)
    fy = (lam * (8 * AX * p2 * c4x * c2y * s1z + 2 * AZ * p2 * c2y * c1z * s4x - 4 * AY * p2 * s4x * s2y * s1z)
          + mu * (8 * AX * p2 * c4x * c2y * s1z + 2 * AZ * p2 * c2y * c1z * s4x - 17 * AY * p2 * s4x * s2y * s1z)
          - 8 * AY * mu * p2 * s4x * s2y * s1z)
    fz = (lam * (4 * AX * p2 * c4x * c1z * s2y + 2 * AY * p2 * c2y * c1z * s4x - AZ * p2 * s4x * s2y * s1z)
          + mu * (4 * AX * p2 * c4x * c1z * s2y + 2 * AY * p2 * c2y * c1z * s4x - 20 * AZ * p2 * s4x * s2y * s1z)
          - 2 * AZ * mu * p2 * s4x * s2y * s1z)
    return np.stack([fx, fy, fz])


def test_mms_body_force_is_minus_the_printed_expression():
    _, ff = _mms_symbolic()
    rng = np.random.default_rng(3)
    pts = rng.uniform(0, 1, size=(3, 50))
    ours = np.array(ff(*pts))
    printed = _printed_appendix_e(*pts)
    assert np.allclose(ours, -printed, rtol=1e-12, atol=1e-12 * np.abs(printed).max())


def mms_problem(n, k=(4, 2, 1)):
    fu, ff = _mms_symbolic(k)
    m = mg.box_mesh_3d(n, n, n, 1.0, 1.0, 1.0)
    geo = mesh_geometry(m)
    for name in ("xmin", "xmax", "ymin", "ymax", "zmin", "zmax"):
        p = [q for q in m["patches"] if q["name"] == name][0]
        xf = geo["xf"][p["start"]:p["start"] + p["size"]]
        mg.set_patch(m, name, "displacement", per_face=np.stack(fu(*xf.T), axis=1))
    xc = geo["xc"]
    body = np.stack(ff(*xc.T), axis=1)
    exact = np.stack(fu(*xc.T), axis=1)
    return m, body, exact


def test_mms_second_order():
    """Lower wave numbers than Appendix E's (one half-period per axis) so
    that meshes the oracle solves in seconds are in the asymptotic range;
    the GPU tests run Appendix E's own field on finer meshes."""
    errs, hs = [], []
    for n in (6, 12, 24):
        m, body, exact = mms_problem(n, k=(1, 1, 1))
        pr = with_source(prepare(m, mg.Material("linear_elastic", E, NU)), body=body)
        u, st = newton_solve(pr, rtol=1e-6, atol=0.0, max_newton_it=3, eta=1e-7, precond="lu", restart=100,
                             max_krylov_it=1000)
        err = np.sqrt(np.mean(np.sum((u.reshape(-1, 3) - exact) ** 2, axis=1)))
        errs.append(err)
        hs.append(1.0 / n)
    orders = [np.log(errs[k] / errs[k + 1]) / np.log(hs[k] / hs[k + 1]) for k in range(2)]
    print("MMS L2 errors", errs, "orders", orders)
    assert orders[-1] > 1.8 and orders[-1] < 2.6


def test_body_force_reaction_balances_total_load():
    m = mg.box_mesh_3d(6, 5, 4, 1.0, 0.8, 0.6, jitter=0.15, seed=8)
    mg.set_patch(m, "zmin", "displacement", (0.0, 0.0, 0.0))
    b = np.array([1.0e5, -2.0e5, -7.8e4])
    pr0 = prepare(m, mg.Material("linear_elastic", E, NU))
    body = np.tile(b, (pr0["nc"], 1))
    pr = with_source(pr0, body=body)
    u, st = newton_solve(pr, rtol=1e-13, atol=0.0, max_newton_it=2, eta=1e-13, precond="lu", restart=200)
    ff = face_forces(u, pr)
    disp = pr["btype"] == 1
    reaction = (ff["T_b"] + ff["RC_b"])[disp].sum(axis=0)
    total = b * pr["geo"]["V"].sum()
    assert np.allclose(reaction, -total, rtol=1e-9, atol=1e-9 * np.abs(total).max())


def test_free_block_translates_with_the_bdf2_recurrence():
    m = mg.box_mesh_3d(4, 3, 3, 1.0, 0.8, 0.6, jitter=0.1, seed=9)
    b = np.array([3.0e4, 0.0, -1.0e4])
    rho, dt = 7800.0, 1e-3
    pr = prepare(m, mg.Material("linear_elastic", E, NU))
    body = np.tile(b, (pr["nc"], 1))
    us, _ = dynamic_solve(pr, rho, dt, 5, body=body, rtol=1e-12, atol=1e-30, max_newton_it=3, eta=1e-12,
                          precond="lu", restart=50)
    # scalar recurrence of Eq. (inertia2) for a = b / rho, from rest
    acc = b / rho
    un, unm1, vn, vnm1 = np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3)
    for step in range(5):
        # [3 (3u - 4un + unm1)/(2 dt) - 4 vn + vnm1] / (2 dt) = acc, solved for u
        u = ((2 * dt * acc + 4 * vn - vnm1) * 2 * dt / 3 + 4 * un - unm1) / 3
        v = (3 * u - 4 * un + unm1) / (2 * dt)
        unm1, un, vnm1, vn = un, u, vn, v
        got = us[step].reshape(-1, 3)
        assert np.allclose(got, u[None, :], rtol=1e-10, atol=1e-14), (step, got[:2], u)
