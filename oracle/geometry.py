"""Mesh geometry for the cell-centred finite-volume discretisation.

Paper: Section 2.3 (cell-centred finite volume discretisation) defines
cells P, faces f, area vectors Gamma_f, the centroids x_P and x_f and the
vectors d between them; it does not fix how they are computed.  The
definition used here (the usual polyhedral-mesh construction):

* face with vertices p_0..p_{k-1}: x_bar = mean vertex; fan triangles
  a_i = 1/2 (p_i - x_bar) x (p_{i+1} - x_bar) with centroids
  c_i = (p_i + p_{i+1} + x_bar)/3; Gamma_f = sum a_i;
  x_f = sum (a_i . n) c_i / sum (a_i . n),  n = Gamma_f/|Gamma_f|.
  2-D (plane strain, unit depth): a face is an edge p0 -> p1 with
  Gamma = (y1 - y0, -(x1 - x0)) and x_f its midpoint.
* cell: x_bar_c = mean of its face centroids; each face closes a pyramid
  (3-D: volume Gamma_out.(x_f - x_bar_c)/3, centroid x_bar_c + 3/4 (x_f -
  x_bar_c); 2-D: area Gamma_out.(x_f - x_bar_c)/2, centroid x_bar_c +
  2/3 (x_f - x_bar_c)); Omega_P = sum of pyramid volumes, x_P the
  volume-weighted mean of the pyramid centroids.
"""

import numpy as np


def _face_geometry(mesh):
    dim = mesh["dim"]
    pts = mesh["points"]
    fp = mesh["face_ptr"]
    fv = mesh["face_pts"]
    nf = mesh["n_faces"]
    Gamma = np.zeros((nf, dim))
    xf = np.zeros((nf, dim))
    counts = np.diff(fp)
    if dim == 2:
        if not np.all(counts == 2):
            raise ValueError("2-D faces must be edges with two points")
        p0 = pts[fv[fp[:-1]]]
        p1 = pts[fv[fp[:-1] + 1]]
        Gamma[:, 0] = p1[:, 1] - p0[:, 1]
        Gamma[:, 1] = -(p1[:, 0] - p0[:, 0])
        xf[:] = 0.5 * (p0 + p1)
        return Gamma, xf
    for k in np.unique(counts):
        sel = np.nonzero(counts == k)[0]
        idx = fp[sel][:, None] + np.arange(k)[None, :]
        P = pts[fv[idx]]                       # [m, k, 3]
        xbar = P.mean(axis=1)                  # [m, 3]
        a = np.zeros((sel.size, k, 3))
        c = np.zeros((sel.size, k, 3))
        for i in range(k):
            pi = P[:, i, :]
            pj = P[:, (i + 1) % k, :]
            a[:, i, :] = 0.5 * np.cross(pi - xbar, pj - xbar)
            c[:, i, :] = (pi + pj + xbar) / 3.0
        G = a.sum(axis=1)
        n = G / np.linalg.norm(G, axis=1)[:, None]
        wgt = np.einsum("mkd,md->mk", a, n)
        Gamma[sel] = G
        xf[sel] = np.einsum("mk,mkd->md", wgt, c) / wgt.sum(axis=1)[:, None]
    return Gamma, xf


def _scatter(idx, vals, n):
    """out[idx[i]] += vals[i] (rows), in index order."""
    if vals.ndim == 1:
        return np.bincount(idx, weights=vals, minlength=n)
    return np.stack([np.bincount(idx, weights=vals[:, d], minlength=n)
                     for d in range(vals.shape[1])], axis=1)


def _cell_geometry(mesh, Gamma, xf):
    dim = mesh["dim"]
    nc = mesh["n_cells"]
    n_int = mesh["n_internal"]
    own = mesh["owner"].astype(np.int64)
    nb = mesh["neighbour"].astype(np.int64)
    # cell-face incidence with outward area vectors
    cells = np.concatenate([own, nb])
    faces = np.concatenate([np.arange(mesh["n_faces"]), np.arange(n_int)])
    sgn = np.concatenate([np.ones(mesh["n_faces"]), -np.ones(n_int)])
    nface = np.bincount(cells, minlength=nc).astype(np.float64)
    xbar = _scatter(cells, xf[faces], nc) / nface[:, None]
    r = xf[faces] - xbar[cells]
    Gout = Gamma[faces] * sgn[:, None]
    if dim == 3:
        vol = np.einsum("md,md->m", Gout, r) / 3.0
        cen = xbar[cells] + 0.75 * r
    else:
        vol = np.einsum("md,md->m", Gout, r) / 2.0
        cen = xbar[cells] + (2.0 / 3.0) * r
    V = _scatter(cells, vol, nc)
    xc = _scatter(cells, vol[:, None] * cen, nc) / V[:, None]
    return V, xc


def mesh_geometry(mesh):
    """Return dict(Gamma, xf, V, xc) for a mesh dictionary (see meshgen)."""
    Gamma, xf = _face_geometry(mesh)
    V, xc = _cell_geometry(mesh, Gamma, xf)
    if np.any(V <= 0.0):
        bad = int(np.argmin(V))
        raise ValueError("non-positive cell volume at cell %d" % bad)
    return dict(Gamma=Gamma, xf=xf, V=V, xc=xc)
