"""The cell-pass launch shapes give the same bits.

Direct gathers (0), LDS-staged gradient and flux passes (1) and the fused
single pass (2, the tile's halo gradients recomputed from a two-ring copy in
LDS), each with one workgroup per tile or a persistent grid, run the same
sequence of floating-point operations for every cell gradient and every
face force, so R(u) and J v agree bit for bit, on single meshes (both laws,
2-D and 3-D, ragged last tile, tiny meshes), on a mixed-law batch, and
through whole Newton solves (the solver's segment masks included).  The
fused pass is also checked against the oracle directly, to the residual
tolerance of the kernel parity tests: 1e-11 of the largest face force.
"""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import residual as o_residual

from gpu_common import Pair, jittered, with_bcs, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    (2, (37, 29), "neo_hookean"),
    (3, (13, 11, 7), "linear_elastic"),
    (3, (13, 11, 7), "neo_hookean"),
    (3, (3, 3, 3), "neo_hookean"),       # one partial tile
    (3, (41, 29, 19), "neo_hookean"),    # 89 tiles, ragged tail
    (3, (13, 11, 7), "st_venant_kirchhoff"),
]


def _shapes(info):
    out = [(0, 0), (0, 16)]
    if info["tiled"]:
        out += [(1, 0), (1, 16)]
    if info["fused"]:
        out += [(2, 0), (2, 16), (2, 8)]
    return out


def _state(p, seed, amp):
    rng = np.random.default_rng(seed)
    xc = p.pr["geo"]["xc"]
    dim = xc.shape[1]
    A = rng.uniform(-0.1, 0.1, size=(dim, dim)) * amp
    u = xc @ A.T + 0.002 * amp * rng.standard_normal(xc.shape)
    return u.reshape(-1)


@pytest.fixture(params=CASES, ids=lambda c: "%dd-%s-%s" % (c[0], "x".join(map(str, c[1])), c[2]))
def pair(request, lib):
    dim, shape, law = request.param
    m = with_bcs(jittered(dim, shape, seed=11), dim)
    p = Pair(lib, m, mg.Material(law, 1e6, 0.3, alpha_rc=0.8))
    yield p
    p.close()


def test_cell_pass_shapes_bitwise(lib, pair):
    info = pair.gm.info
    print("shapes", info["n_cells"], info["tiled"], info["fused"], info["tile_ring2_max"], flush=True)
    if pair.gm.n_cells >= 1000:
        assert info["tiled"] == 1 and info["fused"] == 1
    u = pair.internal(_state(pair, 3, 1.0))
    v = pair.internal(np.random.default_rng(4).standard_normal(pair.n))
    res = {}
    for passes, persist in _shapes(info):
        lib.set_cell_passes(pair.gm, passes, persist)
        R = pair.residual(u, 0.9)
        J1 = torch.empty_like(u)
        lib.jv(pair.gm, 0.9, u, R, v, 0.0, J1, pair.work)
        J2 = torch.empty_like(u)
        lib.jv(pair.gm, 0.9, u, R, v, 1e-7, J2, pair.work)
        res[(passes, persist)] = (R, J1, J2)
    R0, J10, J20 = res[(0, 0)]
    assert torch.isfinite(R0).all() and torch.isfinite(J10).all()
    for key, (R, J1, J2) in res.items():
        assert torch.equal(R, R0), key
        assert torch.equal(J1, J10), key
        assert torch.equal(J2, J20), key


def test_fused_residual_matches_oracle(lib, pair):
    if not pair.gm.info["fused"]:
        pytest.skip("mesh too small to be tile-ordered")
    lib.set_cell_passes(pair.gm, 2, 0)
    for seed, amp, load in [(1, 0.0, 1.0), (2, 1.0, 0.6)]:
        u = _state(pair, seed, amp)
        Ro = o_residual(u, pair.pr, load).reshape(-1)
        Rg = pair.external(pair.residual(pair.internal(u), load))
        parts = o_residual(u, pair.pr, load, parts=True)
        scale = max(np.abs(parts["traction"]).max(), np.abs(parts["rc"]).max(), 1.0)
        assert np.abs(Rg - Ro).max() <= 1e-11 * scale


def test_unsupported_shape_rejected(lib):
    m = with_bcs(jittered(3, (3, 3, 3), seed=1), 3)
    gm = lib.create_mesh(m, mg.Material())
    with pytest.raises(lib.JfnkError):
        lib.set_cell_passes(gm, 3, 0)
    with pytest.raises(lib.JfnkError):
        lib.set_cell_passes(gm, 0, -1)
    gm.close()


def _batch():
    rng = np.random.default_rng(17)
    probs = []
    for i, sh in enumerate([(5, 4, 6), (21, 13, 9), (4, 11, 3), (17, 9, 12)]):
        m = mg.box_mesh_3d(*sh, 1.0, 0.7 + 0.1 * i, 0.9, jitter=0.15, seed=300 + i)
        mg.set_patch(m, "xmin", "displacement", (0.0, 0.0, 0.0))
        mg.set_patch(m, "xmax", "traction", tuple(rng.uniform(-1, 1, 3) * 2e3))
        law = ["linear_elastic", "neo_hookean", "st_venant_kirchhoff", "neo_hookean"][i]
        probs.append((m, mg.Material(law, float(rng.uniform(1e5, 1e6)), float(rng.uniform(0.2, 0.4)))))
    return probs


def test_batch_and_newton_bitwise(lib):
    probs = _batch()
    gm = lib.create_batch([p[0] for p in probs], [p[1] for p in probs])
    assert gm.info["fused"] == 1
    rng = np.random.default_rng(9)
    u = gm.to_internal(to_dev(rng.uniform(-1e-3, 1e-3, gm.n_dof_external)))
    v = gm.to_internal(to_dev(rng.standard_normal(gm.n_dof_external)))
    work = lib.make_workspace(gm, 0)
    out = {}
    for passes, persist in [(0, 0), (1, 0), (2, 0), (2, 8)]:
        lib.set_cell_passes(gm, passes, persist)
        R = torch.empty_like(u)
        lib.residual(gm, 0.8, u, R, work)
        J = torch.empty_like(u)
        lib.jv(gm, 0.8, u, R, v, 0.0, J, work)
        out[(passes, persist)] = (R, J)
    for key, (R, J) in out.items():
        assert torch.equal(R, out[(0, 0)][0]), key
        assert torch.equal(J, out[(0, 0)][1]), key
    # whole Newton solves: segments converge at different times, so the
    # passes run under the solver's segment masks
    opts = lib.newton_opts(n_increments=2, max_newton_it=8, rtol=1e-8, eta=1e-3, restart=30, max_it=300,
                           precond="jacobi")
    wk = lib.make_workspace(gm, 1, restart=30, precond=lib.PC_JACOBI)
    sols = {}
    for passes in (0, 2):
        lib.set_cell_passes(gm, passes, 0)
        x = torch.zeros_like(u)
        st, stats, seg = lib.newton_solve_batch(gm, opts, x, wk)
        sols[passes] = (st, [s["gmres_it"] for s in stats], seg, x)
    assert sols[0][:3] == sols[2][:3]
    assert torch.equal(sols[0][3], sols[2][3])
    gm.close()
