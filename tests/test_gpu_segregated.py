"""The segregated solution procedure (Section 3.1, Eq. SegSys and
Eq. SegSysX-Z; inner tolerance 0.9 of Section 3.2) on the GPU.

It iterates on the same discrete equations R(u) = 0 as the Newton path, so
at a tight outer tolerance its solution is the oracle's Newton solution
(relative L2 <= 1e-8): a linear-elastic jittered block with each
preconditioner, a neo-Hookean block in two load increments, and a mesh
with symmetry planes (per-component J_tilde diagonal).  The option checks
return JFNK_E_ARG without device work."""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare
from oracle.newton import newton_solve as o_newton

pytestmark = pytest.mark.gpu


def _block(law_scale=1.0, sym=False, seed=12):
    m = mg.box_mesh_3d(9, 8, 7, 1.0, 0.8, 0.6, jitter=0.2, seed=seed)
    mg.set_patch(m, "ymin", "displacement", (0.0, 0.0, 0.0))
    mg.set_patch(m, "ymax", "pressure", (5e4 * law_scale, 0, 0))
    mg.set_patch(m, "xmax", "symmetry" if sym else "traction", (1e4 * law_scale, 0.0, 2e4 * law_scale))
    return m


def _segregated(lib, m, mat, **kw):
    gm = lib.create_mesh(m, mat)
    pc = lib.PRECOND[kw.get("precond", "amg32")]
    work = lib.make_workspace(gm, 1, restart=4, precond=pc)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    st, stats = lib.segregated_solve(gm, lib.segregated_opts(**kw), u, work)
    out = gm.to_external(u).cpu().numpy()
    gm.close()
    return out, st, stats


@pytest.mark.parametrize("precond", ["jacobi", "amg32", "amg64"])
def test_segregated_linear_block_matches_oracle(lib, precond):
    m = _block()
    mat = mg.Material("linear_elastic", 1e6, 0.3)
    uo, io = o_newton(prepare(m, mat), rtol=1e-10, max_newton_it=3, eta=1e-12, precond="lu",
                      max_krylov_it=400)
    ug, st, stats = _segregated(lib, m, mat, rtol=1e-11, max_outer_it=50000, inner_rtol=0.9,
                                precond=precond)
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    print(precond, "segregated outer", stats["newton_it"], "CG", stats["gmres_it"], "rel L2", err,
          "ms", stats["t_ms"][0])
    assert st == lib.OK
    assert stats["newton_it"] > 5          # a fixed-point iteration, not one Newton step
    assert err <= 1e-8


def test_segregated_neo_hookean_increments(lib):
    m = _block(law_scale=1.0)
    mat = mg.Material("neo_hookean", 1e6, 0.3)
    uo, io = o_newton(prepare(m, mat), n_increments=2, rtol=1e-11, max_newton_it=20, eta=1e-12,
                      precond="lu", max_krylov_it=400, jv="complex_step")
    ug, st, stats = _segregated(lib, m, mat, n_increments=2, rtol=1e-11, max_outer_it=50000,
                                inner_rtol=0.9, precond="amg32")
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    print("NH segregated outer", stats["newton_it"], "CG", stats["gmres_it"], "rel L2", err)
    assert st == lib.OK
    assert err <= 1e-8


def test_segregated_with_symmetry_plane(lib):
    m = _block(sym=True)
    mat = mg.Material("linear_elastic", 1e6, 0.3)
    uo, _ = o_newton(prepare(m, mat), rtol=1e-10, max_newton_it=3, eta=1e-12, precond="lu",
                     max_krylov_it=400)
    ug, st, stats = _segregated(lib, m, mat, rtol=1e-11, max_outer_it=50000, precond="amg32")
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    print("symmetry segregated outer", stats["newton_it"], "rel L2", err)
    assert st == lib.OK and err <= 1e-8


def test_segregated_option_errors(lib):
    m = _block()
    mat = mg.Material("linear_elastic", 1e6, 0.3)
    gm = lib.create_mesh(m, mat)
    work = lib.make_workspace(gm, 1, restart=4, precond=lib.PC_AMG32)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    for kw in (dict(inner_rtol=1.0), dict(inner_rtol=0.0), dict(max_outer_it=0), dict(precond="none")):
        with pytest.raises(lib.JfnkError) as e:
            lib.segregated_solve(gm, lib.segregated_opts(**kw), u, work)
        assert e.value.status == lib.E_ARG
    assert torch.count_nonzero(u).item() == 0
    gm.close()
    gb = lib.create_batch([m, m], [mat, mat])
    wb = lib.make_workspace(gb, 1, restart=4, precond=lib.PC_AMG32)
    ub = torch.zeros(gb.n_dof, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.JfnkError) as e:
        lib.segregated_solve(gb, lib.segregated_opts(), ub, wb)
    assert e.value.status == lib.E_ARG
    gb.close()
