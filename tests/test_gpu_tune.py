"""The launch-shape and schedule tuner: every candidate it times computes
the same bits (fused, LDS-staged or gathered cell passes, one workgroup per tile
or a persistent grid, any run length of Arnoldi steps, graphs or not), so
tuning changes time only.  Checked on a mesh large enough for persistent
grids (more tiles than 512 workgroups).  The orthogonalisation it also
times (Gram-Schmidt twice or delayed) changes rounding, not the method: a
solve that leaves it to the handle gets the tuner's choice."""

import numpy as np
import pytest
import torch

import meshgen as mg

from gpu_common import to_dev

pytestmark = pytest.mark.gpu


def _mesh():
    m = mg.box_mesh_3d(72, 48, 44, 1.5, 1.0, 0.9, jitter=0.15, seed=77)
    mg.set_patch(m, "zmin", "displacement", (0.0, 0.0, 0.0))
    mg.set_patch(m, "zmax", "traction", (2e3, -1e3, 4e3))
    return m, mg.Material("neo_hookean", 5e5, 0.35)


def test_tuner_choices_keep_results(lib):
    m, mat = _mesh()
    gm = lib.create_mesh(m, mat)
    assert gm.info["tiled"] == 1 and gm.n_cells // 256 > 512
    rng = np.random.default_rng(5)
    u_ext = rng.uniform(-1e-3, 1e-3, size=gm.n_dof_external)
    v_ext = rng.standard_normal(gm.n_dof_external)
    u = gm.to_internal(torch.tensor(u_ext, device="cuda"))
    v = gm.to_internal(torch.tensor(v_ext, device="cuda"))
    gopts = lib.gmres_opts(restart=20, max_it=400, rtol=1e-6, precond="amg32", cheb_degree=3)
    work = lib.make_workspace(gm, 1, restart=20, precond=lib.PC_AMG32)
    Ru = torch.empty_like(u)
    Jv0 = torch.empty_like(u)
    lib.residual(gm, 1.0, u, Ru, work)
    lib.jv(gm, 1.0, u, Ru, v, 0.0, Jv0, work)
    # a Newton solve with the default launch shapes
    nopts = lib.newton_opts(n_increments=1, max_newton_it=6, rtol=1e-6, eta=1e-4, restart=20, max_it=400,
                            precond="amg32", cheb_degree=3)
    u0 = torch.zeros_like(u)
    st0, s0 = lib.newton_solve(gm, nopts, u0, work)
    rep = lib.autotune(gm, gopts, u, work)
    print(rep)
    assert len(rep["jv"]) >= 4 and len(rep["solve"]) >= 4
    assert {c["persist"] for c in rep["jv"]} >= {0, 512}
    assert {c["lds"] for c in rep["jv"]} == ({0, 1, 2} if gm.info["fused"] else {0, 1})
    assert all(c["ms"] > 0 for c in rep["jv"] + rep["solve"])
    # same bits after tuning
    Jv1 = torch.empty_like(u)
    lib.jv(gm, 1.0, u, Ru, v, 0.0, Jv1, work)
    assert torch.equal(Jv0, Jv1)
    u1 = torch.zeros_like(u)
    st1, s1 = lib.newton_solve(gm, nopts, u1, work)
    assert st0 == st1 and s0["gmres_it"] == s1["gmres_it"]
    assert torch.equal(u0, u1)
    # the orthogonalisation left to the handle is the one the tuner chose
    assert rep["orth"] in (0, 1) and all(t > 0 for t in rep["orth_ms"])
    out = []
    for orth in ("auto", rep["orth"]):
        ua = torch.zeros_like(u)
        oa = lib.newton_opts(n_increments=1, max_newton_it=6, rtol=1e-6, eta=1e-4, restart=20, max_it=400,
                             precond="amg32", cheb_degree=3, orth=orth)
        sta, sa = lib.newton_solve(gm, oa, ua, work)
        out.append((ua, sa["gmres_it"], sta))
    assert out[0][2] == out[1][2] and out[0][1] == out[1][1] and torch.equal(out[0][0], out[1][0])
    gm.close()
