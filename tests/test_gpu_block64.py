"""The 64^3 linear-elastic block with +-20% node jitter (262,144 cells;
E = 200 GPa, nu = 0.3, clamped bottom, 10 MPa pressure on top) on the GPU
against the oracle, at full size.

* residual and automatic-step J v of every cell-pass form (direct gathers,
  LDS-staged passes, the fused pass when the mesh fits it) against the
  oracle on a seeded state: the mesh has over 64 tiles, so the step size is
  finished by the separate large-segment reduction;
* GMRES(30) with the block-Jacobi preconditioner (the compact-stencil
  approximate Jacobian's diagonal blocks, Section 3.1) to the configured
  1e-10, and further to 1e-12, against the oracle's solution sampled on
  every 61st cell (tests/golden/block64_solution.npz, written by
  tests/golden/make_block_solution.py from the oracle alone), and the
  oracle's residual at the GPU solution.
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
    if not os.path.exists(GOLDEN):
        pytest.skip("oracle solution not generated")
    ref = np.load(GOLDEN)
    m, mat, pr, gm = block
    work = lib.make_workspace(gm, 1, restart=30, precond=lib.PC_JACOBI)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    R = torch.empty_like(u)
    lib.residual(gm, 1.0, u, R, work)
    x = torch.zeros_like(u)
    opts = lib.gmres_opts(restart=30, max_it=200000, rtol=rtol, precond=lib.PC_JACOBI)
    st, stats = lib.gmres(gm, 1.0, u, R, -R, x, opts, work)
    ug = gm.to_external(x).cpu().numpy()
    uc = ug.reshape(-1, 3)[ref["cells"]]
    err = np.linalg.norm(uc - ref["u"]) / np.linalg.norm(ref["u"])
    rel = np.linalg.norm(residual(ug, pr, 1.0)) / float(ref["res0"])
    print("rtol %g: %s, %d GMRES, sampled rel L2 vs oracle %.2e, oracle |R(u_gpu)|/|R0| %.2e"
          % (rtol, lib.STATUS_NAMES[st], stats["gmres_it"], err, rel), flush=True)
    assert st == lib.OK
    assert rel <= 2 * rtol
    assert err <= (1e-8 if rtol >= 1e-10 else 1e-10)
