"""Symmetry planes on the GPU against the oracle (Section 2.3.2, Eq. symm;
the symmetry sums of Eq. leastSquaresGrad and Eq. RhieChow; the symmetry
block of the approximate Jacobian, Section 3.1).

  * residual and J.v parity on half meshes with a symmetry plane, for the
    three laws, 2-D and 3-D, jittered nodes, on every cell-pass launch
    shape (which agree bit for bit);
  * a tilted symmetry plane (normal not along an axis), where the mirror
    image mixes the components;
  * Newton solves with the Jacobi, FP32-AMG and FP64-AMG preconditioners
    (per-component diagonal of the symmetry blocks) reach the oracle
    solution;
  * a batch that mixes a mesh with symmetry planes and one without.
Tolerances as in the other kernel parity tests: residual 1e-11 of the
largest face force, J.v with the oracle's eps 1e-6 relative, solves 1e-8.
"""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare, residual as o_residual
from oracle.jacobian import jv_fd, eps_walker_pernice
from oracle.newton import newton_solve as o_newton

from gpu_common import Pair

pytestmark = pytest.mark.gpu

LAWS = ["linear_elastic", "neo_hookean", "st_venant_kirchhoff"]


def _half_mesh(dim, shape, seed=5):
    """Box with jittered nodes, symmetry planes on xmax and ymin."""
    if dim == 2:
        m = mg.box_mesh_2d(shape[0], shape[1], 1.0, 0.8, jitter=0.2, seed=seed)
    else:
        m = mg.box_mesh_3d(shape[0], shape[1], shape[2], 1.0, 0.8, 0.6, jitter=0.2, seed=seed)
    mg.set_patch(m, "xmin", "displacement", (0.001, -0.002, 0.0005)[:dim])
    mg.set_patch(m, "xmax", "symmetry")
    mg.set_patch(m, "ymin", "symmetry")
    mg.set_patch(m, "ymax", "traction", (2e4, 1e4, -5e3)[:dim])
    if dim == 3:
        mg.set_patch(m, "zmax", "pressure", (3e4, 0, 0))
    return m


def _tilted_mesh():
    """A 3-D block sheared so that its xmax face is the plane x + y/2 = 1
    (normal not along an axis), with that face a symmetry plane."""
    m = mg.box_mesh_3d(11, 9, 6, 1.0, 0.8, 0.6, jitter=0.15, seed=9)
    p = m["points"].copy()
    p[:, 0] = p[:, 0] - 0.5 * p[:, 1] * p[:, 0]
    m["points"] = p
    mg.set_patch(m, "xmin", "displacement", (0.0, 0.0, 0.0))
    mg.set_patch(m, "xmax", "symmetry")
    mg.set_patch(m, "ymax", "traction", (1e4, 2e4, 0.0))
    mg.set_patch(m, "zmax", "pressure", (-2e4, 0, 0))
    return m


def _state(pr, seed, amp):
    rng = np.random.default_rng(seed)
    xc = pr["geo"]["xc"]
    dim = xc.shape[1]
    A = rng.uniform(-0.1, 0.1, size=(dim, dim)) * amp
    u = xc @ A.T + 0.002 * amp * rng.standard_normal(xc.shape)
    return u.reshape(-1)


def _shapes(info):
    out = [(0, 0)]
    if info["tiled"]:
        out += [(1, 0), (1, 16)]
    if info["fused"]:
        out += [(2, 0), (2, 8)]
    return out


CASES = [(2, (37, 29)), (3, (13, 11, 7)), (3, (41, 29, 9))]


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dd-%s" % (c[0], "x".join(map(str, c[1]))))
def test_symmetry_residual_and_jv_parity(lib, case, law):
    dim, shape = case
    m = _half_mesh(dim, shape)
    p = Pair(lib, m, mg.Material(law, 1e6, 0.3, alpha_rc=0.8))
    try:
        assert np.count_nonzero(p.pr["btype"] == 4) > 0
        u = _state(p.pr, 3, 1.0)
        v = np.random.default_rng(4).standard_normal(p.n)
        load = 0.9
        Ro = o_residual(u, p.pr, load).reshape(-1)
        parts = o_residual(u, p.pr, load, parts=True)
        scale = max(np.abs(parts["traction"]).max(), np.abs(parts["rc"]).max(), 1.0)
        eps = eps_walker_pernice(u, v)
        Jo, _ = jv_fd(u, v, p.pr, load, eps=eps, Ru=Ro)
        ud, vd = p.internal(u), p.internal(v)
        ref = None
        for passes, persist in _shapes(p.gm.info):
            lib.set_cell_passes(p.gm, passes, persist)
            R = p.residual(ud, load)
            J = torch.empty_like(ud)
            lib.jv(p.gm, load, ud, R, vd, eps, J, p.work)
            if ref is None:
                ref = (R.clone(), J.clone())
                err = np.abs(p.external(R) - Ro).max()
                rel = np.linalg.norm(p.external(J) - Jo) / np.linalg.norm(Jo)
                print(dim, shape, law, "residual err / scale", err / scale, "J.v rel", rel, flush=True)
                assert err <= 1e-11 * scale
                assert rel <= 1e-6
            else:
                assert torch.equal(R, ref[0]), (passes, persist)
                assert torch.equal(J, ref[1]), (passes, persist)
    finally:
        p.close()


def test_tilted_symmetry_plane_parity(lib):
    m = _tilted_mesh()
    p = Pair(lib, m, mg.Material("neo_hookean", 1e6, 0.3))
    try:
        ns = p.pr["ns"]
        assert np.abs(ns[:, 1]).min() > 0.1          # the plane's normal mixes x and y
        u = _state(p.pr, 8, 0.3)
        Ro = o_residual(u, p.pr, 1.0).reshape(-1)
        assert np.isfinite(Ro).all()
        parts = o_residual(u, p.pr, 1.0, parts=True)
        scale = max(np.abs(parts["traction"]).max(), np.abs(parts["rc"]).max(), 1.0)
        R = p.residual(p.internal(u), 1.0)
        err = np.abs(p.external(R) - Ro).max()
        print("tilted plane residual err / scale", err / scale)
        assert err <= 1e-11 * scale
    finally:
        p.close()


@pytest.mark.parametrize("precond", ["jacobi", "amg32", "amg64"])
@pytest.mark.parametrize("law", ["linear_elastic", "neo_hookean"])
def test_symmetry_solve_matches_oracle(lib, law, precond):
    m = _half_mesh(3, (13, 11, 7))
    mat = mg.Material(law, 1e6, 0.3)
    n_inc = 2 if law == "neo_hookean" else 1
    pr = prepare(m, mat)
    uo, io = o_newton(pr, n_increments=n_inc, rtol=1e-10, max_newton_it=20, eta=1e-11, precond="lu",
                      max_krylov_it=4000, jv="complex_step")
    assert io["converged"]
    gm = lib.create_mesh(m, mat)
    pc = lib.PRECOND[precond]
    work = lib.make_workspace(gm, 1, restart=60, precond=pc)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    opts = lib.newton_opts(n_increments=n_inc, max_newton_it=30, rtol=1e-10, eta=1e-6, restart=60,
                           max_it=40000, precond=precond, cheb_degree=3, stol=1e-13)
    st, stats = lib.newton_solve(gm, opts, u, work, allow=(lib.E_NOT_CONVERGED, lib.E_BREAKDOWN))
    ug = gm.to_external(u).cpu().numpy()
    gm.close()
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    print(law, precond, "status", st, "rel L2", err, stats["newton_it"], stats["gmres_it"])
    assert st == lib.OK
    assert err <= 1e-8


def test_batch_with_and_without_symmetry(lib):
    a = _half_mesh(3, (13, 11, 7), seed=5)
    b = mg.box_mesh_3d(9, 8, 7, 1.0, 0.8, 0.6, jitter=0.2, seed=6)
    mg.set_patch(b, "xmin", "displacement", (0.0, 0.0, 0.0))
    mg.set_patch(b, "xmax", "traction", (1e4, 0.0, 2e4))
    mats = [mg.Material("neo_hookean", 1e6, 0.3), mg.Material("linear_elastic", 1e6, 0.3)]
    gm = lib.create_batch([a, b], mats)
    work = lib.make_workspace(gm, 1, restart=60, precond=lib.PC_AMG32)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    opts = lib.newton_opts(max_newton_it=30, rtol=1e-10, eta=1e-6, restart=60, max_it=40000,
                           precond="amg32", cheb_degree=3, stol=1e-13)
    st, stats, seg = lib.newton_solve_batch(gm, opts, u, work, n_increments=[2, 1])
    assert st == lib.OK and all(x == lib.OK for x in seg), (st, seg)
    ue = gm.to_external(u).cpu().numpy()
    for s, (m, mat, ninc) in enumerate(zip([a, b], mats, [2, 1])):
        uo, _ = o_newton(prepare(m, mat), n_increments=ninc, rtol=1e-10, max_newton_it=20, eta=1e-11,
                         precond="lu", max_krylov_it=4000, jv="complex_step")
        err = np.linalg.norm(ue[gm.segment_slice_external(s)] - uo) / np.linalg.norm(uo)
        print("segment", s, "rel L2", err)
        assert err <= 1e-8
    gm.close()
