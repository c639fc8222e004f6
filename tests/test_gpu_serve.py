"""Request server on the GPU: concurrent solves on separate streams under an
HBM budget.  Each served result must equal the same request solved alone
(same kernels, same reduction order: bitwise), and match the oracle's
solution within the stated tolerance (1e-8 relative).
"""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare
from oracle.newton import newton_solve as o_newton

pytestmark = pytest.mark.gpu


def _requests():
    rng = np.random.default_rng(77)
    out = []
    for i in range(7):
        n = (6, 9, 7, 11, 8, 6, 10)[i]
        m = mg.box_mesh_3d(n, n + 1, n - 1, 1.0, 1.1, 0.9, jitter=0.15, seed=300 + i)
        mg.set_patch(m, "zmin", "displacement", (0.0, 0.0, 0.0))
        mg.set_patch(m, "zmax", "traction", tuple(rng.uniform(-1, 1, 3) * 3e3))
        law = "neo_hookean" if i % 3 == 1 else "linear_elastic"
        mat = mg.Material(law, float(rng.uniform(2e5, 1e6)), float(rng.uniform(0.2, 0.4)))
        inc = 1 if law == "linear_elastic" else 1 + i % 3
        out.append((m, mat, inc))
    return out


def _opts(lib, inc, precond):
    return lib.newton_opts(n_increments=inc, max_newton_it=20, rtol=1e-10, eta=1e-8, restart=40, max_it=20000,
                           precond=precond, cheb_degree=3)


@pytest.mark.parametrize("precond", ["amg32", "jacobi"])
def test_served_equals_alone_and_oracle(lib, precond):
    reqs = _requests()
    # budget that holds about three of these requests at once
    srv = lib.Server(hbm_budget=1 << 40, max_slots=1)
    f0 = srv.wait(srv.submit(reqs[3][0], reqs[3][1], _opts(lib, 1, precond)))[0]["footprint_bytes"]
    srv.close()
    srv = lib.Server(hbm_budget=int(3.2 * f0), max_slots=4)
    tickets = [srv.submit(m, mat, _opts(lib, inc, precond)) for m, mat, inc in reqs]
    served = [srv.wait(t) for t in tickets]
    mt = srv.metrics()
    srv.close()
    print(precond, mt)
    print([(i["status"], i["error"]) for i, _ in served])
    assert mt["completed"] == len(reqs), [(i["status"], i["error"]) for i, _ in served]
    assert mt["hbm_peak"] <= int(3.2 * f0)
    for k, ((m, mat, inc), (info, u)) in enumerate(zip(reqs, served)):
        assert info["status"] == lib.OK, info
        gm = lib.create_mesh(m, mat)
        w = lib.make_workspace(gm, 1, restart=40, precond=lib.PRECOND[precond])
        ud = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
        lib.newton_solve(gm, _opts(lib, inc, precond), ud, w)
        alone = gm.to_external(ud).cpu().numpy()
        gm.close()
        assert np.array_equal(alone, u), k
        if k in (0, 1):
            uo, _ = o_newton(prepare(m, mat), n_increments=inc, rtol=1e-10, max_newton_it=20, eta=1e-9,
                             precond="lu", max_krylov_it=4000)
            err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
            print("request", k, "vs oracle", err, info["latency_ms"])
            assert err <= 1e-8
