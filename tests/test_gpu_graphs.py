"""Arnoldi steps replayed from captured HIP graphs, and enqueued in runs of
different lengths, give the same solutions, bit for bit, as direct
launches: the device-side Givens update stops every mesh at the same step
whatever the host does between runs.  Each Newton solve replays the step
graphs many times (every GMRES cycle of every Newton iteration), with the
host's own synchronisations and eager launches in between; both the null
stream (the library forks onto its own stream) and a caller stream (captured
directly) are covered, and every replayed result is checked against the
direct-launch one and the oracle.
"""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare
from oracle.newton import newton_solve as o_newton

pytestmark = pytest.mark.gpu


def _problems():
    rng = np.random.default_rng(91)
    out = []
    for i, sh in enumerate([(7, 5, 6), (10, 6, 4), (5, 9, 5)]):
        m = mg.box_mesh_3d(*sh, 1.0, 0.8 + 0.1 * i, 0.9, jitter=0.15, seed=400 + i)
        mg.set_patch(m, "xmin", "displacement", (0.0, 0.0, 0.0))
        mg.set_patch(m, "xmax", "traction", tuple(rng.uniform(-1, 1, 3) * 2e3))
        law = "neo_hookean" if i == 1 else "linear_elastic"
        out.append((m, mg.Material(law, float(rng.uniform(1e5, 1e6)), float(rng.uniform(0.2, 0.4)))))
    return out


def _solve(lib, probs, precond, graphs, chunk, stream):
    gm = lib.create_batch([p[0] for p in probs], [p[1] for p in probs])
    work = lib.make_workspace(gm, 1, restart=12, precond=lib.PRECOND[precond])
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    opts = lib.newton_opts(max_newton_it=20, rtol=1e-10, eta=1e-8, restart=12, max_it=20000,
                           precond=precond, cheb_degree=3, step_chunk=chunk, graphs=graphs)
    st, stats, seg = lib.newton_solve_batch(gm, opts, u, work, n_increments=[1, 2, 1], stream=stream)
    torch.cuda.synchronize()
    assert st == lib.OK and all(x == lib.OK for x in seg), (st, seg)
    out = gm.to_external(u).cpu().numpy()
    slices = [gm.segment_slice_external(k) for k in range(len(probs))]
    gm.close()
    return out, [s["gmres_it"] for s in stats], slices


@pytest.mark.parametrize("precond", ["jacobi", "amg32"])
def test_graph_replay_matches_direct_launches(lib, precond):
    probs = _problems()
    side = torch.cuda.Stream()
    ref, its_ref, slices = _solve(lib, probs, precond, graphs=0, chunk=1, stream=None)
    for graphs, chunk, stream in [(1, 4, None), (1, 1, side), (1, 5, side), (0, 12, side)]:
        u, its, _ = _solve(lib, probs, precond, graphs, chunk, stream)
        print(precond, graphs, chunk, "its", its, its_ref)
        assert its == its_ref
        assert np.array_equal(u, ref), (graphs, chunk)
    # restarted cycles were exercised (restart 12)
    assert max(its_ref) > 12
    for k in (0, 1):
        m, mat = probs[k]
        uo, _ = o_newton(prepare(m, mat), n_increments=[1, 2, 1][k], rtol=1e-10, max_newton_it=20, eta=1e-9,
                         precond="lu", max_krylov_it=4000)
        err = np.linalg.norm(ref[slices[k]] - uo) / np.linalg.norm(uo)
        print("mesh", k, "vs oracle", err)
        assert err <= 1e-8
