"""The FP32 Z basis of flexible GMRES (precond | PC_Z32) on the GPU.

* AMG32: the V-cycle's output is an FP32 value already, so the solve with
  the FP32 basis gives the same bits as with the FP64 one: GMRES alone,
  Newton over load increments, and a batch of meshes in one handle;
* JACOBI and AMG64, whose directions are rounded to FP32 before their J v:
  the solve converges to the same tolerance in nearly the same number of
  steps and matches the oracle's solution to 1e-8;
* the workspace of the flag is smaller by restart * n_dof * 4 bytes less
  one FP64 vector;
* left preconditioning, augmentation and the segregated solver refuse it.
"""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare
from oracle.newton import newton_solve as o_newton

pytestmark = pytest.mark.gpu


def _block():
    m = mg.box_mesh_3d(17, 15, 13, 1.0, 0.9, 0.8, jitter=0.15, seed=22)
    mg.set_patch(m, "xmin", "displacement", (0.0, 0.0, 0.0))
    mg.set_patch(m, "xmax", "traction", (1e6, -3e5, 2e5))
    return m, mg.Material("linear_elastic", 200e9, 0.3)


def _gmres(lib, gm, precond, rtol, restart=30, graphs=2):
    work = lib.make_workspace(gm, 1, restart=restart, precond=precond)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    R = torch.empty_like(u)
    lib.residual(gm, 1.0, u, R, work)
    x = torch.zeros_like(u)
    opts = lib.gmres_opts(restart=restart, max_it=20000, rtol=rtol, precond=precond, graphs=graphs)
    st, stats = lib.gmres(gm, 1.0, u, R, -R, x, opts, work)
    return st, stats, x


@pytest.mark.parametrize("graphs", [0, 1])
def test_amg32_z32_gmres_same_bits(lib, graphs):
    m, mat = _block()
    gm = lib.create_mesh(m, mat)
    s64, st64, x64 = _gmres(lib, gm, "amg32", 1e-10, graphs=graphs)
    s32, st32, x32 = _gmres(lib, gm, "amg32+z32", 1e-10, graphs=graphs)
    print("graphs", graphs, "FP64 Z:", st64["gmres_it"], "FP32 Z:", st32["gmres_it"])
    assert s64 == s32 == lib.OK
    assert st64["gmres_it"] == st32["gmres_it"]
    assert torch.equal(x64, x32)
    gm.close()


def test_amg32_z32_newton_same_bits(lib):
    m = mg.cantilever_mesh(20, 4, 2, L=(5.0, 1.0, 1.0), tau=600.0)
    mat = mg.Material("neo_hookean", 1e6, 0.45)
    gm = lib.create_mesh(m, mat)
    out = []
    for pc in ("amg32", "amg32+z32"):
        work = lib.make_workspace(gm, 1, restart=30, precond=pc)
        u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
        opts = lib.newton_opts(n_increments=3, max_newton_it=15, rtol=1e-10, eta=1e-8, restart=30,
                               max_it=20000, precond=pc, cheb_degree=3)
        st, stats = lib.newton_solve(gm, opts, u, work)
        assert st == lib.OK
        out.append((u, stats))
    print("newton", out[0][1]["newton_it"], "gmres", out[0][1]["gmres_it"], out[1][1]["gmres_it"])
    assert out[0][1]["gmres_it"] == out[1][1]["gmres_it"]
    assert torch.equal(out[0][0], out[1][0])
    gm.close()


def test_amg32_z32_batch_same_bits(lib):
    rng = np.random.default_rng(77)
    probs = []
    for i, sh in enumerate([(5, 4, 6), (9, 7, 5), (4, 11, 3)]):
        m = mg.box_mesh_3d(*sh, 1.0, 0.7 + 0.1 * i, 0.9, jitter=0.15, seed=300 + i)
        mg.set_patch(m, "xmin", "displacement", (0.0, 0.0, 0.0))
        mg.set_patch(m, "xmax", "traction", tuple(rng.uniform(-1, 1, 3) * 2e3))
        law = "neo_hookean" if i == 1 else "linear_elastic"
        probs.append((m, mg.Material(law, float(rng.uniform(1e5, 1e6)), float(rng.uniform(0.2, 0.4)))))
    gm = lib.create_batch([p[0] for p in probs], [p[1] for p in probs])
    out = []
    for pc in ("amg32", "amg32+z32"):
        work = lib.make_workspace(gm, 1, restart=40, precond=pc)
        u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
        opts = lib.newton_opts(max_newton_it=20, rtol=1e-10, eta=1e-8, restart=40, max_it=20000, precond=pc,
                               cheb_degree=3)
        st, stats, seg = lib.newton_solve_batch(gm, opts, u, work, n_increments=[1, 3, 2])
        assert st == lib.OK and all(x == lib.OK for x in seg), (st, seg)
        out.append((u, [s["gmres_it"] for s in stats]))
    print("batch gmres", out[0][1], out[1][1])
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][0], out[1][0])
    gm.close()


@pytest.mark.parametrize("precond", ["jacobi", "amg64", "amg32"])
def test_z32_solution_vs_oracle(lib, precond):
    """GMRES to 1e-10 with both bases: both converge, in nearly the same
    number of steps (the same with AMG32), to the oracle's solution."""
    m, mat = _block()
    pr = prepare(m, mat)
    uo, _ = o_newton(pr, n_increments=1, rtol=1e-6, max_newton_it=3, eta=1e-12, precond="lu",
                     max_krylov_it=600)
    gm = lib.create_mesh(m, mat)
    its = []
    for z in ("", "+z32"):
        s, st, x = _gmres(lib, gm, precond + z, 1e-10, restart=50)
        ug = gm.to_external(x).cpu().numpy()
        err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
        print(precond + z, lib.STATUS_NAMES.get(s, s), st["gmres_it"], "GMRES, rel L2 vs oracle %.2e" % err)
        assert s == lib.OK
        assert err <= 1e-8
        its.append(st["gmres_it"])
    if precond == "amg32":
        assert its[1] == its[0]
    else:
        assert its[1] <= 1.1 * its[0] + 5
    gm.close()


def test_z32_workspace_size(lib):
    m, mat = _block()
    gm = lib.create_mesh(m, mat)

    def a256(b):
        return (b + 255) // 256 * 256

    n = gm.n_dof
    for restart in (1, 30, 50):
        for pc in ("jacobi", "amg32", "amg64"):
            full = lib.workspace_size(gm, 1, restart, pc)
            half = lib.workspace_size(gm, 1, restart, pc + "+z32")
            assert full - half == a256(restart * n * 8) - a256(restart * n * 4) - a256(n * 8), (restart, pc)
            assert lib.workspace_size(gm, 2, restart, pc) - lib.workspace_size(gm, 2, restart, pc + "+z32") \
                == full - half
    gm.close()


def test_z32_option_errors(lib):
    m, mat = _block()
    gm = lib.create_mesh(m, mat)
    pc = lib.PC_AMG32 | lib.PC_Z32
    work = lib.make_workspace(gm, 1, restart=10, precond=pc)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    R = torch.empty_like(u)
    lib.residual(gm, 1.0, u, R, work)
    x = torch.zeros_like(u)
    for kw in (dict(left=1), dict(augment=2), dict(precond=pc | 32)):
        o = lib.gmres_opts(restart=10, max_it=10, rtol=1e-6, **{"precond": pc, **kw})
        with pytest.raises(lib.JfnkError) as e:
            lib.gmres(gm, 1.0, u, R, -R, x, o, work)
        assert e.value.status == lib.E_ARG, kw
    assert torch.count_nonzero(x).item() == 0
    with pytest.raises(lib.JfnkError) as e:
        lib.segregated_solve(gm, lib.segregated_opts(precond=pc), u, work)
    assert e.value.status == lib.E_ARG
    gm.close()
