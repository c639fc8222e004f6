"""Volume terms on the GPU (Section 2.3.1) against the oracle: the body
force of the momentum balance, the BDF2 inertia of Eq. (inertia2), transient
steps from the Taylor predictor of Eq. (predictor), and the manufactured
solution of Appendix E (body force from the symbolic divergence of the
stress), whose error must fall at second order."""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare, residual, with_source
from oracle.jacobian import jv_fd
from oracle.newton import dynamic_solve, newton_solve

from gpu_common import to_dev

pytestmark = pytest.mark.gpu


def _mesh(law, seed=31):
    m = mg.box_mesh_3d(11, 7, 5, 1.0, 0.6, 0.5, jitter=0.15, seed=seed)
    mg.set_patch(m, "xmin", "displacement", (0.0, 0.0, 0.0))
    mg.set_patch(m, "xmax", "traction", (0.0, 2e4, 0.0))
    E = 200e9 if law == "linear_elastic" else 1e6
    return m, mg.Material(law, E, 0.35, rho=7800.0 if law == "linear_elastic" else 1000.0)


@pytest.mark.parametrize("law", ["linear_elastic", "neo_hookean"])
def test_volume_terms_residual_and_jv_parity(lib, law):
    m, mat = _mesh(law)
    pr0 = prepare(m, mat)
    nc = pr0["nc"]
    rng = np.random.default_rng(5)
    scale = 1e-6 if law == "linear_elastic" else 1e-2
    body = rng.standard_normal((nc, 3)) * (1e5 if law == "linear_elastic" else 1e3)
    hist = [rng.standard_normal((nc, 3)) * scale for _ in range(2)] + \
           [rng.standard_normal((nc, 3)) * scale * 100 for _ in range(2)]
    dt = 1e-3 if law == "linear_elastic" else 2e-2
    pr = with_source(pr0, body=body, rho=mat.rho, dt=dt, u_n=hist[0], u_nm1=hist[1], v_n=hist[2], v_nm1=hist[3])
    gm = lib.create_mesh(m, mat)
    work = lib.make_workspace(gm, 0)
    lib.set_body_force(gm, body)
    hd = [gm.to_internal(to_dev(h)) for h in hist]
    lib.set_inertia(gm, dt, *hd)
    u = rng.standard_normal(nc * 3) * scale
    v = rng.standard_normal(nc * 3)
    ud, vd = gm.to_internal(to_dev(u)), gm.to_internal(to_dev(v))
    R = torch.empty_like(ud)
    lib.residual(gm, 0.8, ud, R, work)
    Ro = residual(u, pr, 0.8).reshape(-1)
    err_r = np.abs(gm.to_external(R).cpu().numpy() - Ro).max() / np.abs(Ro).max()
    Jv, eps = lib.jv(gm, 0.8, ud, R, vd, 0.0, torch.empty_like(ud), work, return_eps=True)
    Jo, _ = jv_fd(u, v, pr, 0.8, eps=eps, Ru=Ro)
    err_j = np.linalg.norm(gm.to_external(Jv).cpu().numpy() - Jo) / np.linalg.norm(Jo)
    print(law, "residual rel inf %.2e" % err_r, "J.v rel L2 %.2e" % err_j)
    assert err_r <= 1e-12 and err_j <= 1e-6
    # removing the terms gives back the static residual
    lib.set_body_force(gm, None)
    lib.set_inertia(gm, 0.0)
    lib.residual(gm, 0.8, ud, R, work)
    Rs = residual(u, pr0, 0.8).reshape(-1)
    assert np.abs(gm.to_external(R).cpu().numpy() - Rs).max() <= 1e-12 * np.abs(Rs).max()
    gm.close()


@pytest.mark.parametrize("law", ["linear_elastic", "neo_hookean"])
def test_dynamic_steps_match_oracle(lib, law):
    """A few BDF2 steps of a cantilever from rest under a suddenly applied
    tip load and gravity-like body force, GPU against the oracle's
    transient solve (Newton with the exact Jacobian action on the oracle
    side, past the tolerance the comparison needs)."""
    m = mg.cantilever_mesh(12, 3, 3, L=(2.0, 0.3, 0.3), tau=5e3 if law == "neo_hookean" else 5e6)
    mat = mg.Material(law, 1e6 if law == "neo_hookean" else 200e9, 0.3, rho=1000.0)
    pr = prepare(m, mat)
    body = np.tile([0.0, -9.81 * mat.rho, 0.0], (pr["nc"], 1))
    dt = 0.05 if law == "neo_hookean" else 2e-4
    steps = 4
    uo, so = dynamic_solve(pr, mat.rho, dt, steps, body=body, rtol=1e-11, atol=0.0, max_newton_it=20,
                           eta=1e-10, precond="lu", restart=100, max_krylov_it=2000, jv="complex_step", stol=1e-13)
    gm = lib.create_mesh(m, mat)
    lib.set_body_force(gm, body)
    work = lib.make_workspace(gm, 2, restart=60, precond=lib.PC_AMG32)
    z = lambda: torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    u, up, v, vp, a = z(), z(), z(), z(), z()
    opts = lib.newton_opts(max_newton_it=20, rtol=1e-10, eta=1e-8, restart=60, max_it=20000,
                           precond="amg32", stol=1e-13)
    for k in range(steps):
        st, stats = lib.dynamic_step(gm, dt, opts, u, up, v, vp, a, work)
        ug = gm.to_external(u).cpu().numpy()
        err = np.linalg.norm(ug - uo[k]) / np.linalg.norm(uo[k])
        print(law, "step", k + 1, lib.STATUS_NAMES[st], "newton", stats["newton_it"], "rel L2 %.2e" % err,
              flush=True)
        assert st == lib.OK
        assert err <= 1e-8
    gm.close()


def test_manufactured_solution_second_order(lib):
    """Appendix E's manufactured displacement on the unit cube (regular
    hexes), displacement prescribed on the whole boundary, the body force of
    -div sigma(u_mms): the GPU solution's error falls at second order, and at
    16^3 the GPU solution equals the oracle's."""
    sp = pytest.importorskip("sympy")
    from test_oracle_volume_terms import mms_problem, E, NU
    errs, hs = [], []
    for n in (16, 32, 64):
        m, body, exact = mms_problem(n)
        mat = mg.Material("linear_elastic", E, NU)
        gm = lib.create_mesh(m, mat)
        lib.set_body_force(gm, body)
        work = lib.make_workspace(gm, 1, restart=50, precond=lib.PC_AMG32)
        u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
        opts = lib.newton_opts(max_newton_it=3, rtol=1e-8, eta=1e-9, restart=50, max_it=20000, precond="amg32")
        st, stats = lib.newton_solve(gm, opts, u, work)
        ug = gm.to_external(u).cpu().numpy().reshape(-1, 3)
        errs.append(np.sqrt(np.mean(np.sum((ug - exact) ** 2, axis=1))))
        hs.append(1.0 / n)
        if n == 16:
            pr = with_source(prepare(m, mat), body=body)
            uo, _ = newton_solve(pr, rtol=1e-7, atol=0.0, max_newton_it=3, eta=1e-8, precond="lu", restart=100)
            par = np.linalg.norm(ug.reshape(-1) - uo) / np.linalg.norm(uo)
            print("MMS 16^3 GPU vs oracle rel L2 %.2e" % par)
            assert par <= 1e-6
        gm.close()
    orders = [np.log(errs[k] / errs[k + 1]) / np.log(hs[k] / hs[k + 1]) for k in range(len(errs) - 1)]
    print("MMS L2 errors", errs, "orders", orders, flush=True)
    assert 1.8 < orders[-1] < 2.6
