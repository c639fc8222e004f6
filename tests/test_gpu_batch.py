"""Batched meshes: many independent problems in one handle, one launch per
kernel, per-mesh material, J v step, GMRES and Newton convergence.

Parity per mesh against the oracle (residual 1e-11 of the face forces, J v
1e-6 relative with the same step, solutions 1e-8 relative), and the same
mesh alone (a batch of one) versus inside the mix: residual and J v are
bitwise identical (per-mesh arithmetic does not see the other meshes); the
solutions agree within the stated solve tolerance (the union
preconditioner's smoother interval depends on the mix, which changes the
Krylov path but not the converged answer).
"""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare, residual as o_residual
from oracle.jacobian import jv_fd, eps_walker_pernice
from oracle.newton import newton_solve as o_newton

from gpu_common import to_dev

pytestmark = pytest.mark.gpu


def _problems(dim):
    rng = np.random.default_rng(40 + dim)
    out = []
    shapes = [(9, 7), (23, 11), (5, 31), (17, 17)] if dim == 2 else [(5, 4, 6), (9, 7, 5), (4, 11, 3)]
    for i, sh in enumerate(shapes):
        m = (mg.box_mesh_2d(*sh, 1.0 + 0.2 * i, 0.8, jitter=0.15, seed=100 + i) if dim == 2
             else mg.box_mesh_3d(*sh, 1.0, 0.7 + 0.1 * i, 0.9, jitter=0.15, seed=200 + i))
        mg.set_patch(m, "xmin", "displacement", (0.0,) * dim)
        mg.set_patch(m, "xmax", "traction", tuple(rng.uniform(-1, 1, dim) * 2e3))
        law = "neo_hookean" if (dim == 3 and i == 1) else "linear_elastic"
        out.append((m, mg.Material(law, float(rng.uniform(1e5, 1e6)), float(rng.uniform(0.2, 0.4)))))
    return out


def _ext_state(gm, probs, seed, amp):
    rng = np.random.default_rng(seed)
    parts = []
    for m, _ in probs:
        xc = prepare(m, mg.Material())["geo"]["xc"]
        A = rng.uniform(-0.05, 0.05, size=(m["dim"], m["dim"])) * amp
        parts.append((xc @ A.T).reshape(-1))
    return np.concatenate(parts)


@pytest.mark.parametrize("dim", [2, 3])
def test_batch_residual_and_jv_parity(lib, dim):
    probs = _problems(dim)
    gm = lib.create_batch([p[0] for p in probs], [p[1] for p in probs])
    assert gm.n_segments == len(probs)
    work = lib.make_workspace(gm, 0)
    u = _ext_state(gm, probs, 1, 1.0)
    v = np.random.default_rng(2).standard_normal(gm.n_dof_external)
    ud, vd = gm.to_internal(to_dev(u)), gm.to_internal(to_dev(v))
    R = torch.empty_like(ud)
    lib.residual(gm, 0.8, ud, R, work)
    Jv = torch.empty_like(ud)
    _, eps = lib.jv(gm, 0.8, ud, R, vd, 0.0, Jv, work, return_eps=True)
    Rg, Jg = gm.to_external(R).cpu().numpy(), gm.to_external(Jv).cpu().numpy()
    for s, (m, mat) in enumerate(probs):
        sl = gm.segment_slice_external(s)
        pr = prepare(m, mat)
        Ro = o_residual(u[sl], pr, 0.8).reshape(-1)
        parts = o_residual(u[sl], pr, 0.8, parts=True)
        scale = max(np.abs(parts["traction"]).max(), np.abs(parts["rc"]).max())
        assert np.abs(Rg[sl] - Ro).max() <= 1e-11 * scale, s
        eo = eps_walker_pernice(u[sl], v[sl])
        assert eps[s] == pytest.approx(eo, rel=1e-13)
        Jo, _ = jv_fd(u[sl], v[sl], pr, 0.8, eps=eo, Ru=Ro)
        assert np.linalg.norm(Jg[sl] - Jo) <= 1e-6 * np.linalg.norm(Jo), s
    # padding between meshes stays zero
    assert torch.isfinite(R).all() and torch.isfinite(Jv).all()
    # alone (batch of one) vs in the mix: bitwise identical per mesh
    for s, (m, mat) in enumerate(probs):
        g1 = lib.create_batch([m], [mat])
        w1 = lib.make_workspace(g1, 0)
        sl = gm.segment_slice_external(s)
        u1 = g1.to_internal(to_dev(u[sl]))
        v1 = g1.to_internal(to_dev(v[sl]))
        R1 = torch.empty_like(u1)
        lib.residual(g1, 0.8, u1, R1, w1)
        J1 = torch.empty_like(u1)
        lib.jv(g1, 0.8, u1, R1, v1, 0.0, J1, w1)
        assert np.array_equal(g1.to_external(R1).cpu().numpy(), Rg[sl])
        assert np.array_equal(g1.to_external(J1).cpu().numpy(), Jg[sl])
        g1.close()
    gm.close()


@pytest.mark.parametrize("precond", ["jacobi", "amg32"])
def test_batch_newton_parity_and_alone_vs_mixed(lib, precond):
    probs = _problems(3)
    n_inc = [1, 3, 2]
    gm = lib.create_batch([p[0] for p in probs], [p[1] for p in probs])
    pc = lib.PRECOND[precond]
    work = lib.make_workspace(gm, 1, restart=40, precond=pc)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    opts = lib.newton_opts(max_newton_it=20, rtol=1e-10, eta=1e-8, restart=40, max_it=20000,
                           precond=precond, cheb_degree=3)
    st, stats, seg = lib.newton_solve_batch(gm, opts, u, work, n_increments=n_inc)
    assert st == lib.OK and all(x == lib.OK for x in seg), (st, seg)
    ue = gm.to_external(u).cpu().numpy()
    for s, (m, mat) in enumerate(probs):
        sl = gm.segment_slice_external(s)
        pr = prepare(m, mat)
        uo, _ = o_newton(pr, n_increments=n_inc[s], rtol=1e-10, max_newton_it=20, eta=1e-9, precond="lu",
                         max_krylov_it=4000)
        err = np.linalg.norm(ue[sl] - uo) / np.linalg.norm(uo)
        print(precond, "mesh", s, "err", err, stats[s]["newton_it"], stats[s]["gmres_it"])
        assert err <= 1e-8
        # alone
        g1 = lib.create_batch([m], [mat])
        w1 = lib.make_workspace(g1, 1, restart=40, precond=pc)
        u1 = torch.zeros(g1.n_dof, dtype=torch.float64, device="cuda")
        o1 = lib.newton_opts(n_increments=n_inc[s], max_newton_it=20, rtol=1e-10, eta=1e-8, restart=40,
                             max_it=20000, precond=precond, cheb_degree=3)
        lib.newton_solve(g1, o1, u1, w1)
        ua = g1.to_external(u1).cpu().numpy()
        diff = np.linalg.norm(ua - ue[sl]) / np.linalg.norm(ua)
        print("  alone vs mixed", diff)
        assert diff <= 1e-8
        g1.close()
    gm.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_batch_many_meshes_amg32(lib, dim):
    """Two dozen meshes in one AMG32 hierarchy: every mesh coarsens to a
    single unknown long before the union does, and the padding rows of the
    256-cell alignment never couple to anything."""
    probs = [p for p in mg.config_c4(64, seed=11, lo=60, hi=900)["problems"] if p["mesh"]["dim"] == dim][:24]
    assert len(probs) >= 20
    gm = lib.create_batch([p["mesh"] for p in probs], [p["material"] for p in probs])
    work = lib.make_workspace(gm, 1, restart=40, precond=lib.PC_AMG32)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    opts = lib.newton_opts(max_newton_it=20, rtol=1e-10, eta=1e-10, restart=40, max_it=20000,
                           precond="amg32", cheb_degree=3)
    st, stats, seg = lib.newton_solve_batch(gm, opts, u, work)
    assert st == lib.OK and all(x == lib.OK for x in seg), (st, seg)
    ue = gm.to_external(u).cpu().numpy()
    for s in (0, len(probs) // 2, len(probs) - 1):
        m, mat = probs[s]["mesh"], probs[s]["material"]
        uo, _ = o_newton(prepare(m, mat), n_increments=1, rtol=1e-10, max_newton_it=20, eta=1e-11,
                         precond="lu", max_krylov_it=4000)
        err = np.linalg.norm(ue[gm.segment_slice_external(s)] - uo) / np.linalg.norm(uo)
        print("mesh", s, m["n_cells"], "err", err, stats[s]["gmres_it"])
        assert err <= 1e-8
    gm.close()
