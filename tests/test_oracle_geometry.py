"""Pins for the oracle's mesh geometry (Section 2.3 notation).

Pinned against exact invariants: a jittered box keeps planar boundary
faces, so the cell volumes must sum to the box volume and the first
moments to volume x box centre; every closed cell has zero net outward
area vector; a regular grid has known centroids, areas and w_f = 1/2.
"""

import numpy as np
import pytest

import meshgen as mg
from oracle.geometry import mesh_geometry
from oracle.fv import prepare, gradient


def _outward_sum(mesh, Gamma):
    nc = mesh["n_cells"]
    s = np.zeros((nc, mesh["dim"]))
    np.add.at(s, mesh["owner"], Gamma)
    np.add.at(s, mesh["neighbour"], -Gamma[: mesh["n_internal"]])
    return s


@pytest.mark.parametrize("dim", [2, 3])
def test_jittered_box_volume_and_moment(dim):
    if dim == 2:
        m = mg.box_mesh_2d(7, 5, 1.4, 0.9, jitter=0.3, seed=11)
        vol, centre = 1.4 * 0.9, np.array([0.7, 0.45])
    else:
        m = mg.box_mesh_3d(5, 4, 6, 1.0, 0.8, 1.2, jitter=0.3, seed=12)
        vol, centre = 1.0 * 0.8 * 1.2, np.array([0.5, 0.4, 0.6])
    g = mesh_geometry(m)
    assert np.all(g["V"] > 0)
    assert abs(g["V"].sum() - vol) <= 1e-13 * vol
    if dim == 2:
        # polygons are exact, so the first moment telescopes too (in 3-D the
        # pyramid centroid of a non-planar face is an approximation)
        moment = (g["V"][:, None] * g["xc"]).sum(axis=0)
        assert np.allclose(moment, vol * centre, rtol=0, atol=1e-13)
    s = _outward_sum(m, g["Gamma"])
    assert np.abs(s).max() <= 1e-15 * max(1.0, np.abs(g["Gamma"]).max())


def test_planar_faces_first_moment_3d():
    m = mg.box_mesh_3d(3, 4, 2, 0.9, 1.2, 0.5)
    g = mesh_geometry(m)
    moment = (g["V"][:, None] * g["xc"]).sum(axis=0)
    assert np.allclose(moment, 0.9 * 1.2 * 0.5 * np.array([0.45, 0.6, 0.25]), rtol=0, atol=1e-14)


def test_regular_grid_values():
    m = mg.box_mesh_3d(4, 3, 2, 0.8, 0.6, 0.2)
    g = mesh_geometry(m)
    hx, hy, hz = 0.2, 0.2, 0.1
    # cell (i,j,k) -> i + 4*(j + 3*k)
    idx = np.arange(24)
    i, j, k = idx % 4, (idx // 4) % 3, idx // 12
    nominal = np.stack([(i + 0.5) * hx, (j + 0.5) * hy, (k + 0.5) * hz], axis=1)
    assert np.allclose(g["xc"], nominal, atol=1e-15)
    assert np.allclose(g["V"], hx * hy * hz, rtol=1e-14)
    pr = prepare(m, mg.Material())
    assert np.allclose(pr["w"], 0.5, atol=1e-14)
    # face areas: x-faces hy*hz, y-faces hx*hz, z-faces hx*hy
    n = pr["n"]
    ax = np.argmax(np.abs(n), axis=1)
    expect = np.array([hy * hz, hx * hz, hx * hy])[ax]
    assert np.allclose(pr["magG"], expect, rtol=1e-14)


def test_nonplanar_face_area_is_loop_area():
    """The fan area vector equals 1/2 sum p_i x p_{i+1} (independent of the fan centre)."""
    m = mg.box_mesh_3d(3, 3, 3, jitter=0.3, seed=5)
    g = mesh_geometry(m)
    fp, fv, P = m["face_ptr"], m["face_pts"], m["points"]
    for f in range(0, m["n_faces"], 7):
        pts = P[fv[fp[f]:fp[f + 1]]]
        loop = 0.5 * sum(np.cross(pts[i], pts[(i + 1) % len(pts)]) for i in range(len(pts)))
        assert np.allclose(g["Gamma"][f], loop, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_least_squares_gradient_exact_for_linear_fields(dim):
    """Eq. (leastSquaresGrad) is exact for linear functions (stated below it)."""
    if dim == 2:
        m = mg.box_mesh_2d(6, 7, 1.0, 1.2, jitter=0.25, seed=3)
    else:
        m = mg.box_mesh_3d(4, 5, 3, 1.0, 1.1, 0.7, jitter=0.25, seed=4)
    pr = prepare(m, mg.Material())
    rng = np.random.default_rng(7)
    A = rng.standard_normal((dim, dim))
    u = pr["geo"]["xc"] @ A.T + rng.standard_normal(dim)
    g = gradient(u, pr)
    assert np.abs(g - A.T[None]).max() <= 1e-12 * np.abs(A).max()


def test_annulus_geometry():
    m = mg.annulus_mesh_2d(4, 24, 0.5, 1.0)
    g = mesh_geometry(m)
    # polygon area between the two inscribed 24-gons
    area = 0.5 * 24 * np.sin(2 * np.pi / 24) * (1.0 - 0.25)
    assert abs(g["V"].sum() - area) < 1e-13
    s = _outward_sum(m, g["Gamma"])
    assert np.abs(s).max() < 1e-15
