"""jfnk_jv_noalloc (the J v entry point that allocates nothing) against
jfnk_jv with a caller workspace: the same kernels on the same inputs, so
the outputs must be bitwise equal; checked on two calls in a row, the second
on a smaller mesh, with the automatic and an explicit step, with R(u) given
and computed, and against the oracle's FD J v (1e-6 relative, same eps)."""

import numpy as np
import pytest
import torch

import meshgen as mg
from oracle.fv import prepare, residual
from oracle.jacobian import jv_fd

from gpu_common import to_dev

pytestmark = pytest.mark.gpu


def _problem(lib, big):
    if big:
        m = mg.box_mesh_3d(26, 19, 15, 1.0, 0.8, 0.6, jitter=0.2, seed=41)
        mg.set_patch(m, "xmin", "displacement", (0.001, 0.0, -0.002))
        mg.set_patch(m, "xmax", "traction", (2e4, 1e4, 0.0))
        mat = mg.Material("neo_hookean", 1e6, 0.4)
    else:
        m = mg.box_mesh_2d(23, 17, 1.0, 0.8, jitter=0.2, seed=42)
        mg.set_patch(m, "ymin", "displacement", (0.0, 0.0))
        mg.set_patch(m, "ymax", "pressure", (3e6, 0, 0))
        mat = mg.Material("linear_elastic", 200e9, 0.3)
    return m, mat


def _check(lib, big):
    m, mat = _problem(lib, big)
    gm = lib.create_mesh(m, mat)
    work = lib.make_workspace(gm, 0)
    rng = np.random.default_rng(7 if big else 8)
    u = rng.standard_normal(gm.n_dof) * 1e-3
    v = rng.standard_normal(gm.n_dof)
    ud, vd = gm.to_internal(to_dev(u)), gm.to_internal(to_dev(v))
    R = torch.empty_like(ud)
    lib.residual(gm, 0.7, ud, R, work)
    for eps in (0.0, 3.0e-7):
        for Ru in (R, None):
            ref, e_used = lib.jv(gm, 0.7, ud, Ru, vd, eps, torch.empty_like(ud), work, return_eps=True)
            out = lib.jv_noalloc(gm, 0.7, ud, Ru, vd, eps, torch.full_like(ud, float("nan")))
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (big, eps, Ru is None)
    pr = prepare(m, mat)
    Ro = residual(u, pr, 0.7).reshape(-1)
    Jo, _ = jv_fd(u, v, pr, 0.7, eps=e_used, Ru=Ro)
    err = np.linalg.norm(gm.to_external(out).cpu().numpy() - Jo) / np.linalg.norm(Jo)
    print("jv_noalloc", "3-D NH" if big else "2-D LE", gm.n_cells, "cells, oracle rel", err, flush=True)
    assert err <= 1e-6
    gm.close()


def test_noalloc_matches_workspace_path(lib):
    _check(lib, big=True)
    _check(lib, big=False)   # second call, smaller input, same scratch


def test_noalloc_rejects_oversized_scratch(lib):
    """A mesh whose gradient record does not fit the fixed scratch is refused
    with a message (host-side check, nothing is launched)."""
    m = mg.box_mesh_3d(72, 72, 72, 1.0, 1.0, 1.0)
    mg.set_patch(m, "zmin", "displacement", (0.0, 0.0, 0.0))
    gm = lib.create_mesh(m, mg.Material("linear_elastic", 200e9, 0.3))
    lib.set_cell_passes(gm, 0)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.JfnkError) as ei:
        lib.jv_noalloc(gm, 1.0, u, u.clone(), u.clone() + 1.0, 0.0, torch.empty_like(u))
    assert ei.value.status == lib.E_ARG and "scratch" in str(ei.value)
    gm.close()
