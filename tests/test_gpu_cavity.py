"""Spherical cavity (Section 4.1, case 2; Appendix G) on the GPU: the
one-eighth model with three symmetry planes, exact tractions on the cube
faces and a free cavity.  The GPU solution equals the oracle's on the same
mesh (relative L2 <= 1e-8) and converges to the closed-form displacement
over four meshes (864 to 442k cells) at an L2 order above 1.5."""

import numpy as np
import pytest
import torch

from oracle.fv import prepare
from oracle.newton import newton_solve as o_newton

from test_oracle_cavity import cavity_problem, displacement_errors

pytestmark = pytest.mark.gpu


def _solve(lib, m, mat):
    gm = lib.create_mesh(m, mat)
    work = lib.make_workspace(gm, 1, restart=60, precond=lib.PC_AMG32)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    opts = lib.newton_opts(max_newton_it=3, rtol=1e-11, eta=1e-11, restart=60, max_it=20000, precond="amg32",
                           cheb_degree=3)
    st, stats = lib.newton_solve(gm, opts, u, work)
    out = gm.to_external(u).cpu().numpy()
    gm.close()
    return out, st, stats


def test_cavity_matches_oracle_and_converges(lib):
    m, mat = cavity_problem(8, 6)
    pr = prepare(m, mat)
    uo, info = o_newton(pr, rtol=1e-11, max_newton_it=3, eta=1e-12, precond="lu", restart=100,
                        max_krylov_it=3000)
    ug, st, stats = _solve(lib, m, mat)
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    print("cavity 8x6: GPU vs oracle rel L2", err, stats["gmres_it"], flush=True)
    assert st == lib.OK and err <= 1e-8
    l2 = []
    for nr, nt in [(8, 6), (16, 12), (32, 24), (64, 48)]:
        m, mat = cavity_problem(nr, nt)
        ug, st, stats = _solve(lib, m, mat)
        assert st == lib.OK
        e = displacement_errors(ug, prepare(m, mat))
        print("cavity", nr, nt, m["n_cells"], "cells: L2 / max displacement error", e, "GMRES", stats["gmres_it"],
              flush=True)
        l2.append(e[0])
    orders = [np.log2(l2[i] / l2[i + 1]) for i in range(len(l2) - 1)]
    print("orders", orders)
    # the paper reports about second order on its polyhedral meshes; on these
    # block meshes the L2 order settles near 1.6 (the largest errors sit at
    # the cavity's pole, the cells bounded by two symmetry planes and the sphere)
    assert min(orders) > 1.5
