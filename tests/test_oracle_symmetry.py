"""Pins for symmetry planes in the oracle (Section 2.3.2, Eq. symm; the
symmetry sums of Eq. leastSquaresGrad and Eq. RhieChow; the symmetry
block of the approximate Jacobian, Section 3.1).

  * mirror pin: on a mesh that is mirror-symmetric across x = L, with
    mirror-symmetric loads and a mirror-symmetric displacement field, the
    residual of the full mesh restricted to its left half equals the
    residual of the half mesh with a symmetry plane at x = L, for every
    law, in 2-D and 3-D (the symmetry face sees the mirror cell exactly as
    the internal face on the plane sees its neighbour);
  * no shear on a symmetry plane (the remark after Eq. symm): for the
    linear law the face force is |Gamma| (n.sigma_P.n) n;
  * patch test: a linear field that is symmetric about the plane, with
    the matching tractions elsewhere, has zero residual on a jittered mesh;
  * J_tilde of the half mesh equals the full mesh's J_tilde folded across
    the plane (the reading of the symmetry block's coefficient);
  * the half-mesh Newton solution equals the left half of the full-mesh
    solution.
"""

import numpy as np
import pytest

import meshgen as mg
from oracle.fv import prepare, residual, face_forces, material_constants, SYMM
from oracle.jacobian import approximate_jacobian
from oracle.newton import newton_solve

LAWS = ["linear_elastic", "neo_hookean", "st_venant_kirchhoff"]


def _material(law):
    if law == "linear_elastic":
        return mg.Material(law, 200e9, 0.3)
    return mg.Material(law, 1e6, 0.35)


def _pair(dim, jitter=0.2, seed=3):
    if dim == 2:
        return mg.mirrored_box_pair(2, 4, 5, L=0.8, Ly=1.1, jitter=jitter, seed=seed)
    return mg.mirrored_box_pair(3, 3, 4, 3, L=0.7, Ly=1.0, Lz=0.8, jitter=jitter, seed=seed)


def _loads(half, full, dim, scale):
    """Mirror-consistent loads: prescribed u on x = 0 (and its mirror on
    x = 2L), a traction with no x part on ymin, pressures, and (3-D) a
    prescribed u with no x part on zmax."""
    ub = np.array([0.3, -0.2, 0.1][:dim]) * scale
    ub_m = ub.copy()
    ub_m[0] = -ub_m[0]
    t = np.array([0.0, 0.4, -0.3][:dim])
    for m in (half, full):
        mg.set_patch(m, "xmin", "displacement", tuple(ub))
        mg.set_patch(m, "ymin", "traction", tuple(t))
        mg.set_patch(m, "ymax", "pressure", (0.7,))
        if dim == 3:
            mg.set_patch(m, "zmin", "pressure", (-0.2,))
            mg.set_patch(m, "zmax", "displacement", (0.0, 0.5 * ub[1], 0.5 * ub[2]))
    mg.set_patch(full, "xmax", "displacement", tuple(ub_m))
    mg.set_patch(half, "xmax", "symmetry")


def _mirror_field(u_half, left, mirror, n_full):
    u = np.zeros((n_full, u_half.shape[1]))
    u[left] = u_half
    um = u_half.copy()
    um[:, 0] = -um[:, 0]
    u[mirror] = um
    return u


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("law", LAWS)
def test_half_mesh_equals_mirrored_full_mesh(dim, law):
    half, full, left, mirror = _pair(dim)
    mat = _material(law)
    scale = 1e-4 if law == "linear_elastic" else 0.02
    _loads(half, full, dim, scale)
    # loads in the units of the law's modulus
    ph, pf = prepare(half, mat), prepare(full, mat)
    assert np.count_nonzero(ph["btype"] == SYMM) == (half["n_cells"] // 4 if dim == 2 else 12)
    rng = np.random.default_rng(7)
    uh = rng.standard_normal((half["n_cells"], dim)) * scale
    uf = _mirror_field(uh, left, mirror, full["n_cells"])
    Rh = residual(uh, ph, load=0.8)
    Rf = residual(uf, pf, load=0.8)
    ref = np.abs(Rf).max()
    assert ref > 0
    err = np.abs(Rh - Rf[left]).max() / ref
    assert err < 1e-12, err
    # the mirror half of the full residual is the mirror image
    Rm = Rf[mirror].copy()
    Rm[:, 0] = -Rm[:, 0]
    assert np.abs(Rm - Rf[left]).max() / ref < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_no_shear_on_symmetry_plane_linear_law(dim):
    half, full, left, mirror = _pair(dim)
    mat = _material("linear_elastic")
    _loads(half, full, dim, 1e-4)
    pr = prepare(half, mat)
    u = np.random.default_rng(2).standard_normal((half["n_cells"], dim)) * 1e-4
    ff = face_forces(u, pr)
    c = material_constants(mat)
    sym = pr["sym"]
    g = ff["grad"][pr["Ps"]]
    sig = c["mu"] * (g + np.swapaxes(g, 1, 2)) + c["lam"] * np.trace(g, axis1=1, axis2=2)[:, None, None] * np.eye(dim)
    n = pr["ns"]
    nsn = np.einsum("fi,fij,fj->f", n, sig, n)
    expect = pr["magGb"][sym][:, None] * nsn[:, None] * n
    T = ff["T_b"][sym]
    assert np.abs(T - expect).max() <= 1e-12 * np.abs(expect).max()
    # and the traction has no tangential part although sigma_P has shear
    assert np.abs(np.einsum("fij,fj->fi", sig, n) - nsn[:, None] * n).max() > 1e-3 * np.abs(nsn).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_symmetric_linear_patch_test(dim):
    half, _, _, _ = _pair(dim)
    L = half["points"][:, 0].max()            # the plane
    mat = _material("linear_elastic")
    c = material_constants(mat)
    a = np.array([2.0, -1.0, 0.5][:dim]) * 1e-4
    eps = np.diag(a)
    sig = 2 * c["mu"] * eps + c["lam"] * np.trace(eps) * np.eye(dim)
    normals = {"xmin": 0, "ymin": 1, "ymax": 1, "zmin": 2, "zmax": 2}
    for p in half["patches"]:
        if p["name"] == "xmax":
            mg.set_patch(half, "xmax", "symmetry")
            continue
        ax = normals[p["name"]]
        n = np.zeros(dim)
        n[ax] = -1.0 if p["name"].endswith("min") else 1.0
        mg.set_patch(half, p["name"], "traction", tuple(sig @ n))
    pr = prepare(half, mat)
    x = pr["geo"]["xc"]
    u = x * a[None, :]
    u[:, 0] = a[0] * (x[:, 0] - L)            # u_x odd about the plane x = L
    R = residual(u, pr)
    scale = np.abs(sig).max() * pr["magGb"].max()
    assert np.abs(R).max() < 1e-10 * scale
    # the gradient is the exact one
    g = face_forces(u, pr)["grad"]
    assert np.abs(g - np.diag(a)[None]).max() < 1e-11 * np.abs(a).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_half_mesh_jtilde_is_folded_full_jtilde(dim):
    half, full, left, mirror = _pair(dim)
    mat = _material("linear_elastic")
    _loads(half, full, dim, 1e-4)
    Jh = approximate_jacobian(prepare(half, mat)).toarray()
    Jf = approximate_jacobian(prepare(full, mat)).toarray()
    nh = half["n_cells"]
    Rm = np.eye(dim)
    Rm[0, 0] = -1.0
    fold = np.zeros_like(Jh)
    for P in range(nh):
        for Q in range(nh):
            rp, rq = slice(P * dim, (P + 1) * dim), slice(Q * dim, (Q + 1) * dim)
            a = Jf[left[P] * dim:(left[P] + 1) * dim, left[Q] * dim:(left[Q] + 1) * dim]
            b = Jf[left[P] * dim:(left[P] + 1) * dim, mirror[Q] * dim:(mirror[Q] + 1) * dim]
            fold[rp, rq] = a + b @ Rm
    assert np.abs(Jh - fold).max() <= 1e-12 * np.abs(Jh).max()
    # the symmetry block is not scalar x I
    sym_cells = np.unique(prepare(half, mat)["Ps"])
    P = sym_cells[0]
    blk = Jh[P * dim:(P + 1) * dim, P * dim:(P + 1) * dim]
    assert abs(blk[0, 0] - blk[1, 1]) > 1e-3 * abs(blk[1, 1])


@pytest.mark.parametrize("law", ["linear_elastic", "neo_hookean"])
def test_half_solution_is_left_half_of_full_solution(law):
    half, full, left, mirror = _pair(2)
    mat = _material(law)
    scale = 1e-4 if law == "linear_elastic" else 0.02
    _loads(half, full, 2, scale)
    E = mat.E
    for m in (half, full):
        for p in m["patches"]:
            if p["type"] in ("traction", "pressure"):
                p["value"] = tuple(v * E * scale for v in p["value"])
    kw = dict(n_increments=2 if law == "neo_hookean" else 1, rtol=1e-11, eta=1e-12, restart=60,
              precond="lu", max_newton_it=15, jv="complex_step")
    uh, ih = newton_solve(prepare(half, mat), **kw)
    uf, jf = newton_solve(prepare(full, mat), **kw)
    assert ih["converged"] and jf["converged"]
    uh = uh.reshape(-1, 2)
    uf = uf.reshape(-1, 2)
    err = np.linalg.norm(uh - uf[left]) / np.linalg.norm(uf[left])
    assert err < 1e-9, err
