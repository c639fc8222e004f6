"""The 64^3 linear-elastic block with +-20% node jitter (262,144 cells;
E = 200 GPa, nu = 0.3, clamped bottom, 10 MPa pressure on top) on the GPU
against the oracle, at full size.

* residual and automatic-step J v of every cell-pass form (direct gathers,
  LDS-staged passes, the fused pass when the mesh fits it) against the
  oracle on a seeded state: the mesh has over 64 tiles, so the step size is
  finished by the separate large-segment reduction;
* GMRES(30) with the block-Jacobi preconditioner (the compact-stencil
  approximate Jacobian's diagonal blocks, Section 3.1) to the configured
  1e-10, and asked for 1e-12: the oracle's residual at the GPU solution
  meets 2e-10 (the difference quotient's rounding floor on this mesh is
  about 1e-10), and, when tests/golden/block64_solution.npz exists
  (written by tests/golden/make_block_solution.py from the oracle alone),
  the solution matches the oracle's on every 61st cell.
"""

import os

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare, residual
from oracle.jacobian import jv_fd

from gpu_common import to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "block64_solution.npz")


@pytest.fixture(scope="module")
def block(lib):
    cfg = mg.config_c2()
    m, mat = cfg["mesh"], cfg["material"]
    pr = prepare(m, mat)
    gm = lib.create_mesh(m, mat)
    yield m, mat, pr, gm
    gm.close()


def test_block64_residual_and_jv_every_pass(lib, block):
    m, mat, pr, gm = block
    rng = np.random.default_rng(64)
    u = 1e-4 * rng.standard_normal(gm.n_dof)
    v = rng.standard_normal(gm.n_dof)
    v /= np.linalg.norm(v)
    Ro = residual(u, pr, 1.0).reshape(-1)
    eps_ref = None
    work = lib.make_workspace(gm, 0)
    ud, vd = gm.to_internal(to_dev(u)), gm.to_internal(to_dev(v))
    passes = [0, 1] + ([2] if gm.info["fused"] else [])
    outs = {}
    for p in passes:
        lib.set_cell_passes(gm, p, 0)
        R = torch.empty_like(ud)
        lib.residual(gm, 1.0, ud, R, work)
        Jv, eps = lib.jv(gm, 1.0, ud, R, vd, 0.0, torch.empty_like(ud), work, return_eps=True)
        Rg = gm.to_external(R).cpu().numpy()
        err_r = np.abs(Rg - Ro).max() / np.abs(Ro).max()
        if eps_ref is None:
            eps_ref = eps
            Jo, eps_o = jv_fd(u, v, pr, 1.0, eps=None, Ru=Ro)
            print("eps gpu %.17g oracle %.17g" % (eps, eps_o))
            assert abs(eps - eps_o) <= 1e-13 * eps_o
        assert eps == eps_ref
        err_j = np.linalg.norm(gm.to_external(Jv).cpu().numpy() - Jo) / np.linalg.norm(Jo)
        print("passes", p, "residual rel inf %.2e" % err_r, "J.v rel L2 %.2e" % err_j, flush=True)
        assert err_r <= 1e-12
        assert err_j <= 1e-6
        outs[p] = (R.clone(), Jv.clone())
    for p in passes[1:]:
        assert torch.equal(outs[p][0], outs[0][0]) and torch.equal(outs[p][1], outs[0][1]), p
    lib.set_cell_passes(gm, 1, 0)


@pytest.mark.parametrize("rtol", [1e-10, 1e-12])
def test_block64_gmres_block_jacobi_vs_oracle(lib, block, rtol):
    """The GPU solution satisfies the oracle's residual equation to 2e-10 of
    |R_oracle(0)|; when the stored oracle solution exists, the sampled cells
    also match it.  On this mesh GMRES(30) with block Jacobi and the
    forward-difference J v levels off at about 1e-10 of |b| (the rounding
    floor of the difference quotient: asked for 1e-12 it stops by the
    stagnation test at 8e-11), so the configured 1e-10 is met up to that
    floor and the solve may end by the stagnation test."""
    m, mat, pr, gm = block
    work = lib.make_workspace(gm, 1, restart=30, precond=lib.PC_JACOBI)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    R = torch.empty_like(u)
    lib.residual(gm, 1.0, u, R, work)
    x = torch.zeros_like(u)
    opts = lib.gmres_opts(restart=30, max_it=200000, rtol=rtol, precond=lib.PC_JACOBI)
    st, stats = lib.gmres(gm, 1.0, u, R, -R, x, opts, work)
    ug = gm.to_external(x).cpu().numpy()
    r0 = np.linalg.norm(residual(np.zeros_like(ug), pr, 1.0))
    rel = np.linalg.norm(residual(ug, pr, 1.0)) / r0
    print("rtol %g: %s, %d GMRES, oracle |R(u_gpu)|/|R0| %.2e" % (rtol, lib.STATUS_NAMES[st], stats["gmres_it"], rel),
          flush=True)
    assert st in (lib.OK, lib.E_BREAKDOWN)
    assert rel <= 2e-10
    if os.path.exists(GOLDEN):
        ref = np.load(GOLDEN)
        uc = ug.reshape(-1, 3)[ref["cells"]]
        err = np.linalg.norm(uc - ref["u"]) / np.linalg.norm(ref["u"])
        print("  sampled rel L2 vs the stored oracle solution %.2e" % err, flush=True)
        assert abs(float(ref["res0"]) - r0) <= 1e-12 * r0
        assert err <= 1e-8
