"""Spherical cavity under remote uniaxial tension (Section 4.1, case 2;
Appendix G), one-eighth model with three symmetry planes.

  * the closed forms as printed are one solution: the stress equals the
    linear-elastic stress of the displacement (checked by central
    differences), it is divergence-free, the cavity surface is
    traction-free, and far away the stress tends to T e_z e_z;
  * the oracle's solution on the octant mesh (symmetry planes x, y, z = 0,
    the exact traction on the cube faces, a free cavity) converges to the
    closed-form displacement at about second order, as the paper reports.
"""

import numpy as np
import pytest

import meshgen as mg
from meshgen.cavity import cavity_octant_mesh
from oracle.fv import prepare
from oracle.newton import newton_solve

import cavity_solution as cs

T, E, NU, A = 1e6, 200e9, 0.3, 0.2


def cavity_problem(nr, nt, grade=1.5):
    """The octant mesh with the case's boundary conditions (per-face exact
    tractions on the cube faces)."""
    m = cavity_octant_mesh(nr, nt, a=A, L=1.0, grade=grade)
    for name in ("xsym", "ysym", "zsym"):
        mg.set_patch(m, name, "symmetry")
    fp, fpts, pts = m["face_ptr"], m["face_pts"], m["points"]
    for ax, name in enumerate(("xmax", "ymax", "zmax")):
        p = next(q for q in m["patches"] if q["name"] == name)
        f = np.arange(p["start"], p["start"] + p["size"])
        xf = pts[fpts[fp[f][:, None] + np.arange(4)]].mean(axis=1)
        n = np.zeros(3)
        n[ax] = 1.0
        mg.set_patch(m, name, "traction", per_face=cs.stress(xf, T, NU, A) @ n)
    mg.set_patch(m, "cavity", "traction", (0.0, 0.0, 0.0))
    return m, mg.Material("linear_elastic", E, NU)


def displacement_errors(u, pr):
    """Mean (L2 over cells) and max displacement error against the closed form."""
    xc = pr["geo"]["xc"]
    ue = cs.displacement(xc, T, E, NU, A)
    d = np.linalg.norm(u.reshape(-1, 3) - ue, axis=1)
    return float(np.sqrt(np.mean(d * d))), float(d.max())


def test_closed_forms_are_consistent():
    mu = E / (2 * (1 + NU))
    lam = E * NU / ((1 + NU) * (1 - 2 * NU))
    rng = np.random.default_rng(0)
    x = rng.uniform(0.05, 1.0, size=(40, 3))
    x = x[np.linalg.norm(x, axis=1) > 0.3]
    h = 1e-6
    G = np.zeros((x.shape[0], 3, 3))
    div = np.zeros((x.shape[0], 3))
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        G[:, i, :] = (cs.displacement(x + e, T, E, NU, A) - cs.displacement(x - e, T, E, NU, A)) / (2 * h)
        div += (cs.stress(x + e, T, NU, A)[:, i, :] - cs.stress(x - e, T, NU, A)[:, i, :]) / (2 * h)
    eps = 0.5 * (G + np.swapaxes(G, 1, 2))
    sig_u = 2 * mu * eps + lam * np.trace(eps, axis1=1, axis2=2)[:, None, None] * np.eye(3)
    assert np.abs(cs.stress(x, T, NU, A) - sig_u).max() < 1e-8 * T
    assert np.abs(div).max() < 1e-8 * T
    n = np.abs(rng.standard_normal((20, 3)))
    n /= np.linalg.norm(n, axis=1)[:, None]
    assert np.abs(np.einsum("nij,nj->ni", cs.stress(A * n, T, NU, A), n)).max() < 1e-12 * T
    far = cs.stress(np.array([[300.0, 200.0, 400.0]]), T, NU, A)[0]
    assert np.abs(far - np.diag([0.0, 0.0, T])).max() < 1e-6 * T
    # the stress concentration at the equator: sigma_zz(a, 0, 0) = T (27 - 15 nu) / (14 - 10 nu)
    assert cs.stress(np.array([[A, 0.0, 0.0]]), T, NU, A)[0, 2, 2] == pytest.approx(
        T * (27 - 15 * NU) / (14 - 10 * NU), rel=1e-12)


def test_oracle_cavity_second_order():
    errs = []
    for nr, nt in [(4, 3), (8, 6), (16, 12)]:
        m, mat = cavity_problem(nr, nt)
        pr = prepare(m, mat)
        u, info = newton_solve(pr, rtol=1e-10, max_newton_it=3, eta=1e-12, precond="lu", restart=100,
                               max_krylov_it=3000)
        assert info["converged"]
        errs.append(displacement_errors(u, pr))
    l2 = [e[0] for e in errs]
    orders = [np.log2(l2[i] / l2[i + 1]) for i in range(len(l2) - 1)]
    print("cavity L2 errors", l2, "orders", orders)
    assert orders[-1] > 1.6
