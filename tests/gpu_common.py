"""Helpers shared by the GPU parity tests: build a mesh on both sides and
move vectors between the oracle's input cell order and the library."""

import numpy as np
import torch

import meshgen as mg
from oracle.fv import prepare


def to_dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64).reshape(-1), device="cuda")


class Pair:
    """A problem on both sides: oracle data (input order) + GPU mesh handle."""

    def __init__(self, jfnk, mesh, material):
        self.jfnk = jfnk
        self.mesh = mesh
        self.material = material
        self.pr = prepare(mesh, material)
        self.gm = jfnk.create_mesh(mesh, material)
        self.n = self.gm.n_dof
        self.work = jfnk.make_workspace(self.gm, 0)

    def internal(self, x_input_order):
        return self.gm.to_internal(to_dev(x_input_order))

    def external(self, x_dev):
        return self.gm.to_external(x_dev).cpu().numpy()

    def residual(self, u_int, load=1.0):
        R = torch.empty(self.n, dtype=torch.float64, device="cuda")
        self.jfnk.residual(self.gm, load, u_int, R, self.work)
        return R

    def close(self):
        self.gm.close()


def jittered(dim, shape, jitter=0.2, seed=1):
    if dim == 2:
        return mg.box_mesh_2d(shape[0], shape[1], 1.0, 0.8, jitter=jitter, seed=seed)
    return mg.box_mesh_3d(shape[0], shape[1], shape[2], 1.0, 0.8, 0.6, jitter=jitter, seed=seed)


def with_bcs(m, dim):
    mg.set_patch(m, "xmin", "displacement", (0.001, -0.002, 0.0005)[:dim])
    mg.set_patch(m, "xmax", "traction", (2e4, 1e4, -5e3)[:dim])
    mg.set_patch(m, "ymax", "pressure", (3e4, 0, 0))
    return m
