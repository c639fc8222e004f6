"""GPU parity of the residual and J.v kernels against the oracle.

Element-by-element comparison on the same seeded inputs, at sizes that span
several 256-cell workgroups with a ragged tail, for the three laws, 2-D and 3-D,
distorted meshes, all boundary types, and degenerate cases (one partial
slice, zero direction vector).  Tolerances:
  * residual: |R_gpu - R_oracle|_inf <= 1e-11 * (largest face force), i.e.
    FP64 rounding of a sum of O(10) face terms with different association;
  * J.v with the same eps on both sides: relative L2 <= 1e-6 (the stated
    bound; the observed error is ~1e-9, the FD rounding amplification
    1e-16 / eps);
  * run-to-run: bitwise identical.
"""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import residual as o_residual
from oracle.jacobian import jv_fd, eps_walker_pernice, jv_complex_step, jv_fd_central, eps_central

from gpu_common import Pair, jittered, with_bcs, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    (2, (37, 29), "linear_elastic"),
    (2, (37, 29), "neo_hookean"),
    (3, (13, 11, 7), "linear_elastic"),
    (3, (13, 11, 7), "neo_hookean"),
    (3, (3, 3, 3), "neo_hookean"),      # one partial 64-cell slice
    (2, (37, 29), "st_venant_kirchhoff"),
    (3, (13, 11, 7), "st_venant_kirchhoff"),
]


def _scale(pr, u, load):
    parts = o_residual(u, pr, load, parts=True)
    return max(np.abs(parts["traction"]).max(), np.abs(parts["rc"]).max(), 1.0)


@pytest.fixture(params=CASES, ids=lambda c: "%dd-%s-%s" % (c[0], "x".join(map(str, c[1])), c[2]))
def pair(request, lib):
    dim, shape, law = request.param
    m = with_bcs(jittered(dim, shape, seed=7), dim)
    mat = mg.Material(law, 1e6, 0.35, alpha_rc=0.8)
    p = Pair(lib, m, mat)
    yield p
    p.close()


def _state(p, seed, scale):
    """Physically admissible state (J > 0): `scale` in [0, 1] sets a homogeneous
    strain of up to 15%, a smooth field of amplitude 0.3 h and noise 0.02 h."""
    rng = np.random.default_rng(seed)
    xc = p.pr["geo"]["xc"]
    dim = xc.shape[1]
    h = np.sqrt(p.pr["magG"].mean()) if dim == 3 else p.pr["magG"].mean()
    A = rng.uniform(-0.15, 0.15, size=(dim, dim)) * scale
    u = xc @ A.T
    u += 0.3 * h * scale * np.sin(3.0 * xc[:, :1] + 2.0 * xc[:, 1:2] + rng.uniform(0, 6, size=(1, dim)))
    u += 0.02 * h * scale * rng.standard_normal(xc.shape)
    return u.reshape(-1)


def test_residual_parity(pair):
    print("residual parity", pair.gm.info, flush=True)
    for seed, amp, load in [(1, 0.0, 1.0), (2, 0.1, 0.7), (3, 1.0, 1.0)]:
        u = _state(pair, seed, amp)
        Ro = o_residual(u, pair.pr, load).reshape(-1)
        Rg = pair.external(pair.residual(pair.internal(u), load))
        err = np.abs(Rg - Ro).max()
        assert err <= 1e-11 * _scale(pair.pr, u, load), (seed, err)


def test_residual_deterministic(pair):
    u = pair.internal(_state(pair, 4, 1.0))
    a = pair.residual(u, 0.9)
    assert torch.isfinite(a).all()
    b = pair.residual(u, 0.9)
    assert torch.equal(a, b)


def test_jv_parity_and_eps(pair):
    jfnk = pair.jfnk
    u = _state(pair, 5, 1.0)
    v = np.random.default_rng(6).standard_normal(pair.n)
    load = 0.8
    Ru_o = o_residual(u, pair.pr, load).reshape(-1)
    eps_o = eps_walker_pernice(u, v)
    Jv_o, _ = jv_fd(u, v, pair.pr, load, eps=eps_o, Ru=Ru_o)
    ud, vd = pair.internal(u), pair.internal(v)
    Ru_d = pair.residual(ud, load)
    Jv = torch.empty_like(ud)
    _, eps_g = jfnk.jv(pair.gm, load, ud, Ru_d, vd, 0.0, Jv, pair.work, return_eps=True)
    assert eps_g == pytest.approx(eps_o, rel=1e-13)
    # same eps on both sides
    jfnk.jv(pair.gm, load, ud, Ru_d, vd, eps_o, Jv, pair.work)
    Jv_g = pair.external(Jv)
    rel = np.linalg.norm(Jv_g - Jv_o) / np.linalg.norm(Jv_o)
    print("jv rel err", rel)
    assert rel <= 1e-6
    # and against the exact directional derivative, within the FD budget
    exact = jv_complex_step(u, v, pair.pr, load)
    assert np.linalg.norm(Jv_g - exact) <= 1e-5 * np.linalg.norm(exact)
    # Ru computed internally when not supplied
    Jv2 = torch.empty_like(ud)
    jfnk.jv(pair.gm, load, ud, None, vd, eps_o, Jv2, pair.work)
    assert torch.equal(Jv, Jv2)


def test_jv_central_parity(pair):
    """Central-difference J v: the automatic step equals the oracle's, the
    product with the same step matches the oracle's central difference, and
    it is closer to the exact product than the forward difference."""
    jfnk = pair.jfnk
    u = _state(pair, 5, 1.0)
    v = np.random.default_rng(6).standard_normal(pair.n)
    load = 0.8
    ud, vd = pair.internal(u), pair.internal(v)
    work3 = jfnk.make_workspace(pair.gm, 3)
    J = torch.empty_like(ud)
    _, eps_g = jfnk.jv_central(pair.gm, load, ud, vd, 0.0, J, work3, return_eps=True)
    eps_c = eps_central(u, v)
    assert eps_g == pytest.approx(eps_c, rel=1e-13)
    Jo, _ = jv_fd_central(u, v, pair.pr, load, eps=eps_c)
    jfnk.jv_central(pair.gm, load, ud, vd, eps_c, J, work3)
    Jg = pair.external(J)
    rel = np.linalg.norm(Jg - Jo) / np.linalg.norm(Jo)
    exact = jv_complex_step(u, v, pair.pr, load)
    ec = np.linalg.norm(Jg - exact) / np.linalg.norm(exact)
    print("central jv rel err vs oracle", rel, "vs exact", ec)
    assert rel <= 1e-6
    assert ec <= 1e-8


def test_jv_zero_direction(pair):
    ud = pair.internal(_state(pair, 7, 0.5))
    Ru = pair.residual(ud)
    z = torch.zeros_like(ud)
    out = torch.full_like(ud, 7.0)
    _, e = pair.jfnk.jv(pair.gm, 1.0, ud, Ru, z, 0.0, out, pair.work, return_eps=True)
    assert e == 0.0
    assert torch.count_nonzero(out).item() == 0


def test_permutation_roundtrip(pair):
    x = torch.randn(pair.n, dtype=torch.float64, device="cuda")
    y = pair.gm.to_external(pair.gm.to_internal(x))
    assert torch.equal(x, y)
    order = pair.gm.old_of_new
    assert np.array_equal(np.sort(order), np.arange(pair.gm.n_cells))
