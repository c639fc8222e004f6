"""Octant of a cube with a spherical cavity, as a conforming hex mesh.

The domain is [0, L]^3 minus the ball of radius a about the origin (the
one-eighth model of the spherical-cavity case).  Three structured blocks
fill it, one per outer face of the cube: the block facing x = L joins the
sphere point a (1, s, t) / |(1, s, t)| to the cube point L (1, s, t) for
s, t in [0, 1] (and likewise for y = L and z = L), so that neighbouring
blocks share their nodes on the planes x = y, x = z and y = z.  Radial node
spacing is graded towards the cavity by the exponent `grade` (1: uniform).

Patches: "xsym", "ysym", "zsym" (the planes x, y, z = 0), "xmax", "ymax",
"zmax" (the cube faces) and "cavity" (the sphere), all traction-free until
set_patch assigns them.  Faces follow the OpenFOAM conventions of the box
generators: internal faces sorted by (owner, neighbour), owner < neighbour,
vertex order with the right-hand normal out of the owner.
"""

import numpy as np

# faces of a hex (v0..v7: v0-v3 the bottom quad counter-clockwise seen from
# above, v4-v7 above them), each with its outward vertex order
_HEX_FACES = np.array([[0, 3, 2, 1], [4, 5, 6, 7], [0, 1, 5, 4],
                       [3, 7, 6, 2], [0, 4, 7, 3], [1, 2, 6, 5]])


def _block_points(axis, nr, nt, a, L, grade):
    s = np.linspace(0.0, 1.0, nt + 1)
    r = np.linspace(0.0, 1.0, nr + 1) ** grade
    S, T = np.meshgrid(s, s, indexing="ij")              # [nt+1, nt+1]
    d = np.zeros(S.shape + (3,))
    others = [k for k in range(3) if k != axis]
    d[..., axis] = 1.0
    d[..., others[0]] = S
    d[..., others[1]] = T
    inner = a * d / np.linalg.norm(d, axis=-1, keepdims=True)
    outer = L * d
    # node (i, j, k): radial i, angular j, k
    return inner[None] + r[:, None, None, None] * (outer - inner)[None]


def cavity_octant_mesh(nr, nt, a=0.2, L=1.0, grade=1.0):
    """nr cells radially and nt x nt across each of the three blocks."""
    pts, cells = [], []
    base = 0
    for axis in range(3):
        P = _block_points(axis, nr, nt, a, L, grade)
        pts.append(P.reshape(-1, 3))

        def nid(i, j, k):
            return base + (i * (nt + 1) + j) * (nt + 1) + k

        I, J, K = np.meshgrid(np.arange(nr), np.arange(nt), np.arange(nt), indexing="ij")
        I, J, K = I.ravel(), J.ravel(), K.ravel()
        hexes = np.stack([nid(I, J, K), nid(I + 1, J, K), nid(I + 1, J + 1, K), nid(I, J + 1, K),
                          nid(I, J, K + 1), nid(I + 1, J, K + 1), nid(I + 1, J + 1, K + 1),
                          nid(I, J + 1, K + 1)], axis=1)
        cells.append(hexes)
        base += P.shape[0] * P.shape[1] * P.shape[2]
    pts = np.concatenate(pts)
    cells = np.concatenate(cells)
    # merge the nodes the blocks share (identical coordinates by construction)
    key = np.round(pts / (L * 1e-9)).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.ravel()
    order = np.argsort(first)
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    pts = pts[first[order]]
    cells = rank[inv[cells]]
    # right-handed vertex order: flip hexes whose corner triple product is negative
    e1 = pts[cells[:, 1]] - pts[cells[:, 0]]
    e2 = pts[cells[:, 3]] - pts[cells[:, 0]]
    e3 = pts[cells[:, 4]] - pts[cells[:, 0]]
    neg = np.einsum("ci,ci->c", np.cross(e1, e2), e3) < 0
    cells[neg] = cells[neg][:, [0, 3, 2, 1, 4, 7, 6, 5]]
    nc = cells.shape[0]
    # faces: each hex face once per side, matched by its sorted vertex set
    fv = cells[:, _HEX_FACES].reshape(-1, 4)             # [6 nc, 4], outward from its cell
    fc = np.repeat(np.arange(nc), 6)
    skey = np.sort(fv, axis=1)
    _, grp, cnt = np.unique(skey, axis=0, return_inverse=True, return_counts=True)
    grp = grp.ravel()
    if cnt.max() > 2:
        raise ValueError("cavity mesh: a face shared by more than two cells")
    order = np.lexsort((fc, grp))
    g_sorted = grp[order]
    start = np.searchsorted(g_sorted, np.arange(cnt.size))
    first_of = order[start]
    shared = cnt == 2
    A = first_of[shared]                                  # the lower cell's copy (fc ascending)
    B = order[start[shared] + 1]
    own_int, nb_int, pts_int = fc[A], fc[B], fv[A]
    srt = np.lexsort((nb_int, own_int))
    own_int, nb_int, pts_int = own_int[srt], nb_int[srt], pts_int[srt]
    bnd = first_of[~shared]
    xf = pts[fv[bnd]].mean(axis=1)
    tol = 1e-9 * L
    names = ["xsym", "ysym", "zsym", "xmax", "ymax", "zmax", "cavity"]
    label = np.full(bnd.size, 6)
    for ax in range(3):
        label[np.all(np.abs(pts[fv[bnd]][:, :, ax]) < tol, axis=1)] = ax
        label[np.all(np.abs(pts[fv[bnd]][:, :, ax] - L) < tol, axis=1)] = 3 + ax
    rad = np.linalg.norm(pts[fv[bnd]], axis=2)
    on_sphere = np.all(np.abs(rad - a) < 1e-9 * a, axis=1)
    if np.any((label == 6) & ~on_sphere):
        raise ValueError("cavity mesh: unclassified boundary face")
    n_int = own_int.size
    owner = [own_int]
    fpl = [pts_int]
    patches = []
    s0 = n_int
    for k, name in enumerate(names):
        sel = np.nonzero(label == k)[0]
        sel = sel[np.argsort(fc[bnd[sel]], kind="stable")]
        owner.append(fc[bnd[sel]])
        fpl.append(fv[bnd[sel]])
        patches.append(dict(name=name, start=int(s0), size=int(sel.size), type="traction",
                            value=(0.0, 0.0, 0.0), per_face=None))
        s0 += sel.size
    face_pts = np.concatenate(fpl).astype(np.int32)
    return dict(dim=3, points=np.ascontiguousarray(pts, dtype=np.float64),
                face_ptr=np.arange(0, 4 * face_pts.shape[0] + 1, 4, dtype=np.int64),
                face_pts=face_pts.reshape(-1), owner=np.concatenate(owner).astype(np.int32),
                neighbour=nb_int.astype(np.int32), n_cells=int(nc), n_internal=int(n_int),
                n_faces=int(face_pts.shape[0]), patches=patches,
                meta=dict(kind="cavity_octant", n=(nr, nt), L=(a, L), jitter=0.0, seed=None))
