"""The AMG hierarchy description (jfnk_amg_info_get): refused before the
hierarchy exists and for non-AMG preconditioners; after an AMG32 solve the
finest level has the mesh's cells as rows, every level is smaller than the
one above it, the row kernels' lane counts are powers of two, and the
operator complexity is at least one.  On a large single mesh the coarsest
level is a dense inverse formed on the device, and the solve still meets
the oracle's residual equation."""

import pytest
import torch

import meshgen as mg

pytestmark = pytest.mark.gpu


def test_amg_info(lib):
    m = mg.box_mesh_3d(30, 24, 20, 1.0, 0.8, 0.7, jitter=0.15, seed=3)
    mg.set_patch(m, "xmin", "displacement", (0.0, 0.0, 0.0))
    mg.set_patch(m, "xmax", "traction", (1e6, -3e5, 2e5))
    gm = lib.create_mesh(m, mg.Material("linear_elastic", 200e9, 0.3))
    for pc in (lib.PC_AMG32, lib.PC_JACOBI):
        with pytest.raises(lib.JfnkError) as e:
            lib.amg_info(gm, pc)
        assert e.value.status == lib.E_ARG
    work = lib.make_workspace(gm, 1, restart=30, precond=lib.PC_AMG32)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    st, _ = lib.newton_solve(gm, lib.newton_opts(rtol=1e-8, eta=1e-6, restart=30, max_it=2000, precond="amg32"),
                             u, work)
    assert st == lib.OK
    info = lib.amg_info(gm, lib.PC_AMG32)
    print(info)
    n = info["levels"]
    assert n >= 2
    assert info["rows"][0] == m["n_cells"]
    assert all(info["rows"][l + 1] < info["rows"][l] for l in range(n - 1))
    assert all(x > 0 for x in info["nnz"][:-1]) and info["nnz"][-1] == 0
    assert all(g in (1, 2, 4, 8, 16, 32, 64) for g in info["lanes"][:-1]) and info["lanes"][-1] == 0
    assert info["operator_complexity"] >= 1.0 and info["device_bytes"] > 0
    with pytest.raises(lib.JfnkError):
        lib.amg_info(gm, lib.PC_AMG64)   # not built by the AMG32 solve
    gm.close()


@pytest.mark.parametrize("precond", ["amg32", "amg64"])
def test_large_mesh_dense_coarse_level(lib, precond):
    """A single mesh of 64^3 cells stops coarsening at a level of up to 5000
    rows whose dense inverse is formed on the device; the FGMRES solution
    satisfies the oracle's residual equation to the solve tolerance."""
    import numpy as np
    from oracle.fv import prepare, residual
    c = mg.config_c2()
    m, mat = c["mesh"], c["material"]
    gm = lib.create_mesh(m, mat)
    work = lib.make_workspace(gm, 1, restart=30, precond=precond)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    R = torch.empty_like(u)
    lib.residual(gm, 1.0, u, R, work)
    x = torch.zeros_like(u)
    rtol = 1e-10
    st, stats = lib.gmres(gm, 1.0, u, R, -R, x, lib.gmres_opts(restart=30, max_it=5000, rtol=rtol, precond=precond),
                          work)
    info = lib.amg_info(gm, precond)
    print(precond, stats["gmres_it"], "GMRES;", info)
    assert st == lib.OK
    assert info["coarse"] == "dense" and 200 < info["rows"][-1] <= 5000
    pr = prepare(m, mat)
    ug = gm.to_external(x).cpu().numpy()
    r0 = np.linalg.norm(residual(np.zeros_like(ug), pr, 1.0))
    rel = np.linalg.norm(residual(ug, pr, 1.0)) / r0
    print("oracle |R(u_gpu)| / |R(0)| %.2e" % rel)
    assert rel <= 2 * rtol
    gm.close()


def test_served_pool_mesh_coarse_level(lib):
    """The 1,081,472-cell block of the serving stream's request pool (seeded
    generator, 24 requests of up to 2M cells): its 5000-row coarse operator
    was found not positive definite by the device Cholesky in two serving
    runs (among concurrent requests), which failed the request; run alone its
    1,924-row coarse operator factorises.  A hierarchy whose factorisation
    fails coarsens on to the 200-row host limit; either way the
    preconditioned GMRES solve of J x = -R(0) converges."""
    pool = mg.config_c5_stream(rate=200.0, duration=1e9, hi=2e6, max_requests=24)
    hit = [r for r in pool if r["mesh"]["n_cells"] == 1081472]
    assert hit, sorted(r["mesh"]["n_cells"] for r in pool)
    r = hit[0]
    print("pool mesh: %d cells, %s" % (r["mesh"]["n_cells"], r["material"].law), flush=True)
    gm = lib.create_mesh(r["mesh"], r["material"])
    work = lib.make_workspace(gm, 1, restart=30, precond=lib.PC_AMG32)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    R = torch.empty_like(u)
    lib.residual(gm, 1.0, u, R, work)
    x = torch.zeros_like(u)
    st, stats = lib.gmres(gm, 1.0, u, R, -R, x, lib.gmres_opts(restart=30, max_it=5000, rtol=1e-8, precond="amg32"),
                          work)
    info = lib.amg_info(gm, lib.PC_AMG32)
    print(stats["gmres_it"], "GMRES;", info, flush=True)
    assert st == lib.OK
    assert info["coarse"] == "dense" and info["rows"][-1] <= 5000
    gm.close()
