"""Pins for the oracle residual R(u) (Section 2.3, Appendices A-D).

  * linear patch test on distorted meshes (exactness for linear fields,
    Section 2.3.2; the Rhie-Chow term vanishes for linear fields, App. D);
  * homogeneous finite deformation patch test (total Lagrangian, App. A);
  * the printed 1-D Rhie-Chow stencil (App. C) on a uniform hex mesh;
  * the jump form of the Rhie-Chow term (App. D);
  * telescoping: with traction boundaries only, sum_P R_P equals the applied
    force for any u (each internal face enters two cells with opposite sign);
  * objectivity of the neo-Hookean residual under a rigid rotation;
  * invariance under cell renumbering;
  * second-order convergence on the thick-walled cylinder (Lame) problem.
"""

import json
import os

import numpy as np
import pytest

import meshgen as mg
from oracle.fv import prepare, residual, material_constants, neo_hookean
from oracle.newton import newton_solve

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NORMALS = {"xmin": (0, -1), "xmax": (0, 1), "ymin": (1, -1), "ymax": (1, 1), "zmin": (2, -1), "zmax": (2, 1)}


def _normal(name, dim):
    ax, s = NORMALS[name]
    n = np.zeros(dim)
    n[ax] = s
    return n


def _mesh(dim, jitter=0.25, seed=1):
    if dim == 2:
        return mg.box_mesh_2d(6, 5, 1.3, 0.9, jitter=jitter, seed=seed)
    return mg.box_mesh_3d(5, 4, 3, 1.0, 0.8, 0.6, jitter=jitter, seed=seed)


def _face_centres(m):
    return prepare(m, mg.Material())["geo"]["xf"]


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_patch_test(dim):
    m = _mesh(dim)
    mat = mg.Material("linear_elastic", 200e9, 0.3)
    c = material_constants(mat)
    A = np.random.default_rng(0).standard_normal((dim, dim)) * 1e-4
    g = A.T
    sig = c["mu"] * (g + g.T) + c["lam"] * np.trace(g) * np.eye(dim)
    xf = _face_centres(m)
    for p in m["patches"]:
        s = slice(p["start"], p["start"] + p["size"])
        if p["name"] in ("xmin", "ymin"):
            mg.set_patch(m, p["name"], "displacement", per_face=xf[s] @ A.T)
        else:
            mg.set_patch(m, p["name"], "traction", _normal(p["name"], dim) @ sig)
    pr = prepare(m, mat)
    u = pr["geo"]["xc"] @ A.T
    R = residual(u, pr)
    scale = pr["magG"].max() * np.abs(sig).max()
    assert np.abs(R).max() <= 1e-13 * scale
    # and the Rhie-Chow part alone vanishes
    assert np.abs(residual(u, pr, parts=True)["rc"]).max() <= 1e-13 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_homogeneous_finite_deformation_patch_test(dim):
    m = _mesh(dim, seed=2)
    mat = mg.Material("neo_hookean", 1e6, 0.45)
    c = material_constants(mat)
    A = np.random.default_rng(1).standard_normal((dim, dim)) * 0.15
    g3 = np.zeros((3, 3))
    g3[:dim, :dim] = A.T
    sig, cof = neo_hookean(g3[None], c)
    xf = _face_centres(m)
    for p in m["patches"]:
        s = slice(p["start"], p["start"] + p["size"])
        if p["name"] == "xmin":
            mg.set_patch(m, "xmin", "displacement", per_face=xf[s] @ A.T)
        else:
            N3 = np.zeros(3)
            N3[:dim] = _normal(p["name"], dim)
            # dead-load traction per undeformed area: (cof F N) . sigma
            mg.set_patch(m, p["name"], "traction", ((cof[0] @ N3) @ sig[0])[:dim])
    pr = prepare(m, mat)
    R = residual(pr["geo"]["xc"] @ A.T, pr)
    assert np.abs(R).max() <= 1e-12 * np.abs(sig).max() * pr["magG"].max()


def test_rhie_chow_stencil_appendix_c():
    st = json.load(open(os.path.join(GOLDEN, "rc_stencil_1d.json")))
    coef = np.array(st["coefficients"], dtype=float)
    dx = 0.1
    m = mg.box_mesh_3d(9, 3, 3, 9 * dx, 0.3, 0.3)
    mat = mg.Material("linear_elastic", 200e9, 0.3, alpha_rc=0.7)
    pr = prepare(m, mat)
    aK = 0.7 * pr["mat"]["Kbar"]
    area = 0.1 * 0.1
    x = pr["geo"]["xc"][:, 0]
    for f in (lambda t: t ** 2, lambda t: t ** 3, lambda t: t ** 4, lambda t: np.sin(3 * t)):
        u = np.zeros((pr["nc"], 3))
        u[:, 2] = f(x)
        rc = residual(u, pr, parts=True)["rc"]
        for i in range(2, 7):      # cells with WW..EE present
            cell = i + 9 * (1 + 3 * 1)
            xs = (np.arange(i - 2, i + 3) + 0.5) * dx
            expect = aK * area / (4 * dx) * np.dot(coef, f(xs))
            scale = aK * area / dx * np.abs(f(xs)).max()
            assert abs(rc[cell, 2] - expect) <= 1e-13 * scale
            assert abs(rc[cell, 0]) <= 1e-13 * scale and abs(rc[cell, 1]) <= 1e-13 * scale
    # closed forms of the stencil: zero on cubics, -6 aK |Gamma| dx^3 on x^4
    u = np.zeros((pr["nc"], 3))
    u[:, 0] = x ** 4
    cell = 4 + 9 * 4
    assert np.isclose(residual(u, pr, parts=True)["rc"][cell, 0], -6 * aK * area * dx ** 3, rtol=1e-10)


def test_rhie_chow_jump_form_appendix_d():
    """RC_f = alpha Kbar |Gamma| / (d.n) (u*_N - u*_P), u*_P = u_P + (d/2).grad u_P,
    u*_N = u_N - (d/2).grad u_N, on an orthogonal uniform mesh (w_f = 1/2)."""
    m = mg.box_mesh_3d(5, 4, 4, 1.0, 0.7, 0.9)      # all-traction boundaries: no boundary RC
    pr = prepare(m, mg.Material("linear_elastic", 1e9, 0.25))
    xc = pr["geo"]["xc"]
    u = np.stack([np.sin(2 * xc[:, 0]) * xc[:, 1], np.cos(xc[:, 2]) * xc[:, 0] ** 2, np.exp(xc[:, 1])], 1)
    parts = residual(u, pr, parts=True)
    g = parts["grad"]
    P, N, d = pr["P"], pr["N"], pr["d"]
    dn = np.einsum("fi,fi->f", d, pr["n"])
    us_P = u[P] + 0.5 * np.einsum("fi,fij->fj", d, g[P])
    us_N = u[N] - 0.5 * np.einsum("fi,fij->fj", d, g[N])
    flux = pr["mat"]["Kbar"] * (pr["magG"] / dn)[:, None] * (us_N - us_P)
    rc = np.zeros_like(u)
    np.add.at(rc, P, flux)
    np.add.at(rc, N, -flux)
    assert np.abs(rc - parts["rc"]).max() <= 1e-12 * np.abs(parts["rc"]).max()


@pytest.mark.parametrize("law", ["linear_elastic", "neo_hookean"])
def test_total_force_equals_applied_traction(law):
    m = mg.box_mesh_3d(4, 3, 5, 1.0, 0.6, 1.2, jitter=0.25, seed=9)
    rng = np.random.default_rng(2)
    applied = np.zeros(3)
    pr0 = prepare(m, mg.Material())
    for p in m["patches"]:
        t = rng.standard_normal(3) * 1e3
        mg.set_patch(m, p["name"], "traction", t)
        applied += t * pr0["magGb"][p["start"] - m["n_internal"]: p["start"] - m["n_internal"] + p["size"]].sum()
    pr = prepare(m, mg.Material(law, 1e6, 0.3))
    u = rng.standard_normal((pr["nc"], 3)) * 0.02
    R = residual(u, pr, load=1.0)
    scale = np.abs(residual(u, pr, parts=True)["traction"]).max()
    assert np.allclose(R.sum(axis=0), applied, rtol=0, atol=1e-11 * max(scale, 1.0) * pr["nc"])


def test_neo_hookean_residual_objective():
    m = mg.box_mesh_3d(4, 4, 3, jitter=0.2, seed=3)
    rng = np.random.default_rng(8)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    A = Q - np.eye(3)
    xf = _face_centres(m)
    p = [q for q in m["patches"] if q["name"] == "xmin"][0]
    mg.set_patch(m, "xmin", "displacement", per_face=xf[p["start"]:p["start"] + p["size"]] @ A.T)
    for nm in ("xmax", "ymin", "ymax", "zmin", "zmax"):
        mg.set_patch(m, nm, "traction", (0, 0, 0))
    prn = prepare(m, mg.Material("neo_hookean", 1e6, 0.3))
    prl = prepare(m, mg.Material("linear_elastic", 1e6, 0.3))
    u = prn["geo"]["xc"] @ A.T
    scale = prn["mat"]["Kbar"] * prn["magG"].max()
    assert np.abs(residual(u, prn)).max() <= 1e-12 * scale
    assert np.abs(residual(u, prl)).max() >= 1e-3 * scale     # control: linear law is not objective


def test_residual_invariant_under_renumbering():
    m = mg.box_mesh_3d(4, 3, 3, jitter=0.2, seed=21)
    mg.set_patch(m, "xmin", "displacement", (0.01, 0.0, -0.02))
    mg.set_patch(m, "ymax", "pressure", (2e4, 0, 0))
    mg.set_patch(m, "xmax", "traction", (0.0, 1e4, 0.0))
    mat = mg.Material("neo_hookean", 1e6, 0.4)
    rng = np.random.default_rng(3)
    perm = rng.permutation(m["n_cells"])
    m2 = mg.renumber_cells(m, perm)
    pr1, pr2 = prepare(m, mat), prepare(m2, mat)
    u = rng.standard_normal((m["n_cells"], 3)) * 0.03
    u2 = np.zeros_like(u)
    u2[perm] = u
    R1 = residual(u, pr1, load=0.6)
    R2 = residual(u2, pr2, load=0.6)
    assert np.allclose(R2[perm], R1, rtol=0, atol=1e-11 * np.abs(R1).max())


def _lame_problem(nr, nt, E=200e9, nu=0.3, p=1e6, a=0.5, b=1.0):
    A = p * a * a / (b * b - a * a)
    B = p * a * a * b * b / (b * b - a * a)

    def ur(r):   # plane-strain thick cylinder, internal pressure p, free outer surface
        return (1 + nu) / E * ((1 - 2 * nu) * A * r + B / r)

    m = mg.annulus_mesh_2d(nr, nt, a, b)
    po = [q for q in m["patches"] if q["name"] == "outer"][0]
    fp, fv, pts = m["face_ptr"], m["face_pts"], m["points"]
    idx = np.arange(po["start"], po["start"] + po["size"])
    mid = 0.5 * (pts[fv[fp[idx]]] + pts[fv[fp[idx] + 1]])
    rr = np.linalg.norm(mid, axis=1)
    mg.set_patch(m, "outer", "displacement", per_face=(ur(rr) / rr)[:, None] * mid)
    mg.set_patch(m, "inner", "pressure", (p, 0, 0))
    return m, mg.Material("linear_elastic", E, nu), ur


def test_lame_cylinder_second_order():
    spec = json.load(open(os.path.join(GOLDEN, "orders_of_accuracy.json")))
    errs = []
    for nr, nt in [(8, 32), (16, 64), (32, 128)]:
        m, mat, ur = _lame_problem(nr, nt)
        pr = prepare(m, mat)
        u, st = newton_solve(pr, rtol=1e-9, max_newton_it=3, eta=1e-10, precond="lu")
        assert st["converged"]
        xc = pr["geo"]["xc"]
        r = np.linalg.norm(xc, axis=1)
        e = u.reshape(-1, 2) - (ur(r) / r)[:, None] * xc
        errs.append(np.sqrt(np.mean(np.sum(e * e, axis=1))))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - spec["displacement_order"]) <= spec["tolerance"]), orders


def _sheared_quads(s=0.5):
    """4 x 3 unit quads sheared into parallelograms: node (i, j) at (i + s j, j)."""
    m = mg.box_mesh_2d(4, 3, 4.0, 3.0)
    m["points"] = m["points"].copy()
    m["points"][:, 0] += s * m["points"][:, 1]
    return m


def test_rhie_chow_skewed_face_worked_by_hand():
    """Eq. (RhieChow) on a non-orthogonal face: Delta = d/(d.n), worked by hand
    (tests/golden/rc_skewed_face.md).  The cubic field makes the jump differ
    from d . grad u_f, so the magnitude of Delta decides the value: a unit
    Delta = d/|d| would give -6.708 instead of -7.5."""
    from oracle.fv import face_forces
    gold = json.load(open(os.path.join(GOLDEN, "rc_skewed_face.json")))
    m = _sheared_quads()
    mat = mg.Material("linear_elastic", 8.0 / 3.0, 1.0 / 3.0)
    pr = prepare(m, mat)
    assert pr["mat"]["mu"] == pytest.approx(gold["material"]["mu"], rel=1e-14)
    assert pr["mat"]["lam"] == pytest.approx(gold["material"]["lambda"], rel=1e-14)
    xc = pr["geo"]["xc"]
    u = np.zeros((pr["nc"], 2))
    u[:, 0] = xc[:, 0] ** 3
    P, N = 1 + 4 * 1, 2 + 4 * 1
    f = int(np.nonzero((pr["P"] == P) & (pr["N"] == N))[0][0])
    np.testing.assert_allclose(xc[P], gold["owner_centroid"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(xc[N], gold["neighbour_centroid"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(pr["Gam"][f], gold["face_Gamma"], rtol=0, atol=1e-14)
    assert pr["w"][f] == pytest.approx(gold["face_weight"], abs=1e-14)
    ff = face_forces(u.reshape(-1), pr)
    g = ff["grad"]
    np.testing.assert_allclose(g[P], gold["grad_owner"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(g[N], gold["grad_neighbour"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(ff["RC_int"][f], gold["rhie_chow_force"], rtol=0, atol=1e-11)
    np.testing.assert_allclose(ff["T_int"][f], gold["traction_force"], rtol=0, atol=1e-11)
    wrong = np.array(gold["rhie_chow_force_if_Delta_were_d_over_abs_d"])
    assert np.abs(ff["RC_int"][f] - wrong).max() > 0.5
