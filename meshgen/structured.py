"""Structured quad / hex / annulus mesh generators with seeded node jitter.

All generators follow the OpenFOAM face conventions: internal faces first,
sorted by (owner, neighbour) with owner < neighbour; boundary faces
grouped by patch; face vertices ordered so that the right-hand normal
points out of the owner cell (2-D: an edge p0 -> p1 has its outward side
on the right).

Jitter (used for the distorted-hex meshes): every node coordinate gets an
independent U(-j*h, +j*h) displacement, h the cell size in that
direction, drawn from ``numpy.random.Generator(PCG64(seed))``.  Nodes on
the box boundary keep the coordinate normal to that boundary, so the box
stays exact and boundary faces stay planar.
"""

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _csr(face_pt_lists):
    """Stack equal-length vertex lists [n_faces, k] into CSR arrays."""
    n, k = face_pt_lists.shape
    ptr = np.arange(0, (n + 1) * k, k, dtype=np.int64)
    return ptr, face_pt_lists.reshape(-1).astype(np.int32)


def box_mesh_2d(nx, ny, Lx=1.0, Ly=1.0, jitter=0.0, seed=None):
    """nx*ny quads on [0,Lx]x[0,Ly]; patches xmin, xmax, ymin, ymax."""
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = np.linspace(0.0, Ly, ny + 1)
    # node (i, j) -> i + (nx+1)*j ; np.indices order is (j, i) for C layout
    X, Y = np.meshgrid(xs, ys, indexing="xy")  # shape (ny+1, nx+1)
    pts = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
    if jitter > 0.0:
        rng = _rng(seed)
        h = np.array([Lx / nx, Ly / ny])
        delta = rng.uniform(-1.0, 1.0, size=pts.shape) * (jitter * h)[None, :]
        jj, ii = np.divmod(np.arange(pts.shape[0]), nx + 1)
        delta[(ii == 0) | (ii == nx), 0] = 0.0
        delta[(jj == 0) | (jj == ny), 1] = 0.0
        pts = pts + delta

    def P(i, j):
        return i + (nx + 1) * j

    def C(i, j):
        return i + nx * j

    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")  # cell order c = i + nx*j
    I = I.reshape(-1)
    J = J.reshape(-1)
    cells = C(I, J)
    # candidate internal faces per owner: +x then +y (neighbour c+1 < c+nx)
    fx_ok = I < nx - 1
    fy_ok = J < ny - 1
    fx_pts = np.stack([P(I + 1, J), P(I + 1, J + 1)], axis=1)
    fy_pts = np.stack([P(I + 1, J + 1), P(I, J + 1)], axis=1)
    cand_pts = np.stack([fx_pts, fy_pts], axis=1)           # [nc, 2, 2]
    cand_nb = np.stack([cells + 1, cells + nx], axis=1)
    cand_ok = np.stack([fx_ok, fy_ok], axis=1)
    own_int = np.repeat(cells[:, None], 2, axis=1)[cand_ok]
    nb_int = cand_nb[cand_ok]
    pts_int = cand_pts[cand_ok]

    jr = np.arange(ny)
    ir = np.arange(nx)
    bnd = [
        ("xmin", C(0, jr), np.stack([P(0, jr + 1), P(0, jr)], 1)),
        ("xmax", C(nx - 1, jr), np.stack([P(nx, jr), P(nx, jr + 1)], 1)),
        ("ymin", C(ir, 0), np.stack([P(ir, 0), P(ir + 1, 0)], 1)),
        ("ymax", C(ir, ny - 1), np.stack([P(ir + 1, ny), P(ir, ny)], 1)),
    ]
    return _assemble(2, pts, nx * ny, own_int, nb_int, pts_int, bnd,
                     dict(kind="box2d", n=(nx, ny), L=(Lx, Ly), jitter=jitter, seed=seed))


def box_mesh_3d(nx, ny, nz, Lx=1.0, Ly=1.0, Lz=1.0, jitter=0.0, seed=None):
    """nx*ny*nz hexes on a box; patches xmin, xmax, ymin, ymax, zmin, zmax."""
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = np.linspace(0.0, Ly, ny + 1)
    zs = np.linspace(0.0, Lz, nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")  # node i + (nx+1)*(j + (ny+1)*k)
    pts = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
    if jitter > 0.0:
        rng = _rng(seed)
        h = np.array([Lx / nx, Ly / ny, Lz / nz])
        delta = rng.uniform(-1.0, 1.0, size=pts.shape) * (jitter * h)[None, :]
        n = np.arange(pts.shape[0])
        ii = n % (nx + 1)
        jj = (n // (nx + 1)) % (ny + 1)
        kk = n // ((nx + 1) * (ny + 1))
        delta[(ii == 0) | (ii == nx), 0] = 0.0
        delta[(jj == 0) | (jj == ny), 1] = 0.0
        delta[(kk == 0) | (kk == nz), 2] = 0.0
        pts = pts + delta

    def P(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    def C(i, j, k):
        return i + nx * (j + ny * k)

    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    I = I.reshape(-1)
    J = J.reshape(-1)
    K = K.reshape(-1)
    cells = C(I, J, K)
    fx = np.stack([P(I + 1, J, K), P(I + 1, J + 1, K), P(I + 1, J + 1, K + 1), P(I + 1, J, K + 1)], 1)
    fy = np.stack([P(I, J + 1, K), P(I, J + 1, K + 1), P(I + 1, J + 1, K + 1), P(I + 1, J + 1, K)], 1)
    fz = np.stack([P(I, J, K + 1), P(I + 1, J, K + 1), P(I + 1, J + 1, K + 1), P(I, J + 1, K + 1)], 1)
    cand_pts = np.stack([fx, fy, fz], axis=1)                 # [nc, 3, 4]
    cand_nb = np.stack([cells + 1, cells + nx, cells + nx * ny], axis=1)
    cand_ok = np.stack([I < nx - 1, J < ny - 1, K < nz - 1], axis=1)
    own_int = np.repeat(cells[:, None], 3, axis=1)[cand_ok]
    nb_int = cand_nb[cand_ok]
    pts_int = cand_pts[cand_ok]

    # boundary faces, each patch ordered by owner index
    Kx, Jx = np.meshgrid(np.arange(nz), np.arange(ny), indexing="ij")
    Jx = Jx.reshape(-1)
    Kx = Kx.reshape(-1)
    Ky, Iy = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    Iy = Iy.reshape(-1)
    Ky = Ky.reshape(-1)
    Jz, Iz = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    Iz = Iz.reshape(-1)
    Jz = Jz.reshape(-1)
    i0 = np.zeros_like(Jx)
    bnd = [
        ("xmin", C(i0, Jx, Kx),
         np.stack([P(i0, Jx, Kx), P(i0, Jx, Kx + 1), P(i0, Jx + 1, Kx + 1), P(i0, Jx + 1, Kx)], 1)),
        ("xmax", C(i0 + nx - 1, Jx, Kx),
         np.stack([P(i0 + nx, Jx, Kx), P(i0 + nx, Jx + 1, Kx), P(i0 + nx, Jx + 1, Kx + 1), P(i0 + nx, Jx, Kx + 1)], 1)),
    ]
    j0 = np.zeros_like(Iy)
    bnd += [
        ("ymin", C(Iy, j0, Ky),
         np.stack([P(Iy, j0, Ky), P(Iy + 1, j0, Ky), P(Iy + 1, j0, Ky + 1), P(Iy, j0, Ky + 1)], 1)),
        ("ymax", C(Iy, j0 + ny - 1, Ky),
         np.stack([P(Iy, j0 + ny, Ky), P(Iy, j0 + ny, Ky + 1), P(Iy + 1, j0 + ny, Ky + 1), P(Iy + 1, j0 + ny, Ky)], 1)),
    ]
    k0 = np.zeros_like(Iz)
    bnd += [
        ("zmin", C(Iz, Jz, k0),
         np.stack([P(Iz, Jz, k0), P(Iz, Jz + 1, k0), P(Iz + 1, Jz + 1, k0), P(Iz + 1, Jz, k0)], 1)),
        ("zmax", C(Iz, Jz, k0 + nz - 1),
         np.stack([P(Iz, Jz, k0 + nz), P(Iz + 1, Jz, k0 + nz), P(Iz + 1, Jz + 1, k0 + nz), P(Iz, Jz + 1, k0 + nz)], 1)),
    ]
    return _assemble(3, pts, nx * ny * nz, own_int, nb_int, pts_int, bnd,
                     dict(kind="box3d", n=(nx, ny, nz), L=(Lx, Ly, Lz), jitter=jitter, seed=seed))


def annulus_mesh_2d(nr, nt, a, b):
    """Full annulus a < r < b, nr radial x nt angular quads (periodic in theta).

    Patches: ``inner`` (r = a) and ``outer`` (r = b).  Edges are straight
    chords between nodes placed exactly on the circles.
    """
    r = np.linspace(a, b, nr + 1)
    th = 2.0 * np.pi * np.arange(nt) / nt
    R, T = np.meshgrid(r, th, indexing="xy")  # node (i, j) -> i + (nr+1)*j
    pts = np.stack([(R * np.cos(T)).reshape(-1), (R * np.sin(T)).reshape(-1)], axis=1)

    def P(i, j):
        return i + (nr + 1) * (j % nt)

    def C(i, j):
        return i + nr * (j % nt)

    owners, nbs, fpts = [], [], []
    J, I = np.meshgrid(np.arange(nt), np.arange(nr), indexing="ij")
    I = I.reshape(-1)
    J = J.reshape(-1)
    # radial faces (between (i,j) and (i+1,j)); edge p(i+1,j) -> p(i+1,j+1)
    m = I < nr - 1
    owners.append(C(I[m], J[m]))
    nbs.append(C(I[m] + 1, J[m]))
    fpts.append(np.stack([P(I[m] + 1, J[m]), P(I[m] + 1, J[m] + 1)], 1))
    # angular faces (between (i,j) and (i,j+1)); edge p(i+1,j+1) -> p(i,j+1)
    m = J < nt - 1
    owners.append(C(I[m], J[m]))
    nbs.append(C(I[m], J[m] + 1))
    fpts.append(np.stack([P(I[m] + 1, J[m] + 1), P(I[m], J[m] + 1)], 1))
    # wrap faces: owner (i,0), neighbour (i,nt-1); edge p(i,0) -> p(i+1,0)
    ir = np.arange(nr)
    owners.append(C(ir, 0))
    nbs.append(C(ir, nt - 1))
    fpts.append(np.stack([P(ir, 0), P(ir + 1, 0)], 1))
    own = np.concatenate(owners)
    nb = np.concatenate(nbs)
    fp = np.concatenate(fpts)
    order = np.lexsort((nb, own))
    jr = np.arange(nt)
    bnd = [
        ("inner", C(0, jr), np.stack([P(0, jr + 1), P(0, jr)], 1)),
        ("outer", C(nr - 1, jr), np.stack([P(nr, jr), P(nr, jr + 1)], 1)),
    ]
    return _assemble(2, pts, nr * nt, own[order], nb[order], fp[order], bnd,
                     dict(kind="annulus", n=(nr, nt), L=(a, b), jitter=0.0, seed=None))


def _assemble(dim, pts, n_cells, own_int, nb_int, pts_int, bnd, meta):
    n_int = own_int.shape[0]
    owner = [own_int]
    fpl = [pts_int]
    patches = []
    start = n_int
    for name, own_b, pts_b in bnd:
        owner.append(own_b)
        fpl.append(pts_b)
        patches.append(dict(name=name, start=int(start), size=int(own_b.shape[0]),
                            type="traction", value=(0.0, 0.0, 0.0), per_face=None))
        start += own_b.shape[0]
    owner = np.concatenate(owner).astype(np.int32)
    face_ptr, face_pts = _csr(np.concatenate(fpl, axis=0))
    return dict(dim=dim, points=np.ascontiguousarray(pts, dtype=np.float64),
                face_ptr=face_ptr, face_pts=face_pts, owner=owner,
                neighbour=nb_int.astype(np.int32), n_cells=int(n_cells),
                n_internal=int(n_int), n_faces=int(owner.shape[0]),
                patches=patches, meta=meta)


def set_patch(mesh, name, type, value=(0.0, 0.0, 0.0), per_face=None):
    """Set the boundary condition of one patch (in place); returns the mesh.

    type: "displacement" (value = prescribed u), "traction" (value = T),
    "pressure" (value[0] = p, traction = -p n on the undeformed face), or
    "symmetry" (a mirror plane; the value is unused).
    per_face, if given, overrides value with one vector per patch face.
    """
    if type not in ("displacement", "traction", "pressure", "symmetry"):
        raise ValueError("unknown patch type %r" % (type,))
    for p in mesh["patches"]:
        if p["name"] == name:
            v = tuple(float(x) for x in value) + (0.0,) * (3 - len(value))
            p["type"] = type
            p["value"] = v[:3]
            if per_face is not None:
                pf = np.ascontiguousarray(per_face, dtype=np.float64)
                if pf.shape != (p["size"], mesh["dim"]):
                    raise ValueError("per_face must be [%d, %d]" % (p["size"], mesh["dim"]))
                p["per_face"] = pf
            else:
                p["per_face"] = None
            return mesh
    raise KeyError(name)


def mirrored_box_pair(dim, m, ny, nz=1, L=1.0, Ly=1.0, Lz=1.0, jitter=0.0, seed=None):
    """A box mesh on [0, 2L] whose nodes are mirror images across x = L,
    and the mesh of its left half [0, L] with the same nodes.

    The full mesh has 2m cells along x; its node jitter is drawn for the
    left half (plus the plane) and mirrored to the right half, nodes on the
    plane keeping x = L.  Returns (half, full, left, mirror): full-mesh cell
    numbers of the half mesh's cells (half cell k is full cell left[k]) and
    of their mirror images (mirror[k]).  Patches of the half mesh keep the
    box names; its plane x = L is the patch "xmax".
    """
    if dim == 2:
        full = box_mesh_2d(2 * m, ny, 2 * L, Ly, jitter=jitter, seed=seed)
        half = box_mesh_2d(m, ny, L, Ly)
        nyz = ny + 1
    else:
        full = box_mesh_3d(2 * m, ny, nz, 2 * L, Ly, Lz, jitter=jitter, seed=seed)
        half = box_mesh_3d(m, ny, nz, L, Ly, Lz)
        nyz = (ny + 1) * (nz + 1)
    nxf = 2 * m + 1
    pts = full["points"].reshape(nyz, nxf, dim).copy()
    # right half (i > m) = mirror of left (2m - i); the plane i = m at x = L
    pts[:, m + 1:, :] = pts[:, m - 1::-1, :]
    pts[:, m + 1:, 0] = 2.0 * L - pts[:, m + 1:, 0]
    pts[:, m, 0] = L
    full["points"] = np.ascontiguousarray(pts.reshape(-1, dim))
    half["points"] = np.ascontiguousarray(pts[:, :m + 1, :].reshape(-1, dim))
    ncyz = ny * (nz if dim == 3 else 1)
    k = np.arange(m * ncyz)
    i, rest = k % m, k // m
    left = rest * (2 * m) + i
    mirror = rest * (2 * m) + (2 * m - 1 - i)
    return half, full, left, mirror


def mesh_summary(mesh):
    return dict(dim=mesh["dim"], n_cells=mesh["n_cells"], n_faces=mesh["n_faces"],
                n_internal=mesh["n_internal"], n_boundary=mesh["n_faces"] - mesh["n_internal"],
                n_points=int(mesh["points"].shape[0]))


def renumber_cells(mesh, new_of_old):
    """Return a copy of the mesh with cells renumbered: cell c -> new_of_old[c].

    Internal faces whose owner would exceed the neighbour are flipped
    (vertex order reversed) and faces are re-sorted by (owner, neighbour).
    Boundary faces keep their patch grouping.
    """
    new_of_old = np.asarray(new_of_old, dtype=np.int64)
    n_int = mesh["n_internal"]
    fp, fpts = mesh["face_ptr"], mesh["face_pts"]
    lists = [fpts[fp[f]:fp[f + 1]] for f in range(mesh["n_faces"])]
    own = new_of_old[mesh["owner"]]
    nb = new_of_old[mesh["neighbour"]]
    flip = own[:n_int] > nb
    o_int = np.where(flip, nb, own[:n_int])
    n_new = np.where(flip, own[:n_int], nb)
    for f in np.nonzero(flip)[0]:
        lists[f] = lists[f][::-1].copy()
    order = np.lexsort((n_new, o_int))
    new_lists = [lists[f] for f in order] + lists[n_int:]
    ptr = np.zeros(len(new_lists) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(x) for x in new_lists])
    out = dict(mesh)
    out["face_ptr"] = ptr
    out["face_pts"] = np.concatenate(new_lists).astype(np.int32)
    out["owner"] = np.concatenate([o_int[order], own[n_int:]]).astype(np.int32)
    out["neighbour"] = n_new[order].astype(np.int32)
    out["patches"] = [dict(p) for p in mesh["patches"]]
    return out
