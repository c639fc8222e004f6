"""The five benchmark workloads as seeded synthetic inputs.

C1  2-D plane-strain unit square, 40x40 quads, clamped left edge, 1 MPa
    tension on the right edge, E=200 GPa, nu=0.3.
C2  3-D unit cube, 64^3 hexes with +-20% node jitter (seed 2), clamped
    bottom, 10 MPa pressure on top, E=200 GPa, nu=0.3.
C3  3-D neo-Hookean cantilever 10x1x1 m, 1000x100x10 hexes, clamped at
    x=0, dead shear traction on x=10 applied in 10 equal increments,
    E=1 MPa, nu=0.45.
C4  512 independent small linear-elastic block problems (seed 4).
C5  a Poisson request stream of block problems (seed 5).

Only inputs are produced here (meshes, material constants, loads,
solver settings, random vectors); see the package docstring.
"""

from dataclasses import dataclass, field, asdict
import math

import numpy as np

from .structured import box_mesh_2d, box_mesh_3d, set_patch


@dataclass
class Material:
    law: str = "linear_elastic"        # or "neo_hookean"
    E: float = 200e9
    nu: float = 0.3
    alpha_rc: float = 1.0              # Rhie-Chow scaling in the residual
    alpha_pc: float = 1.0              # Rhie-Chow scaling in the approximate Jacobian
    rho: float = 0.0                   # density (transient problems only)

    def as_dict(self):
        return asdict(self)


@dataclass
class SolverSettings:
    n_increments: int = 1
    max_newton_it: int = 20
    newton_rtol: float = 1e-6
    newton_atol: float = 1e-50
    eta: float = 1e-3                  # linear-solve relative tolerance inside Newton
    restart: int = 30
    max_krylov_it: int = 3000
    precond: str = "jacobi"            # "none" | "jacobi" | "amg32"
    flexible: bool = False
    cheb_degree: int = 3
    extra: dict = field(default_factory=dict)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def config_c1():
    m = box_mesh_2d(40, 40, 1.0, 1.0)
    set_patch(m, "xmin", "displacement", (0.0, 0.0))
    set_patch(m, "xmax", "traction", (1.0e6, 0.0))
    set_patch(m, "ymin", "traction", (0.0, 0.0))
    set_patch(m, "ymax", "traction", (0.0, 0.0))
    mat = Material("linear_elastic", 200e9, 0.3, 1.0, 1.0)
    s = SolverSettings(n_increments=1, max_newton_it=1, newton_rtol=1e-6, eta=1e-10,
                       restart=30, precond="jacobi")
    return dict(name="c1_square2d_40x40", mesh=m, material=mat, solver=s)


def config_c2(n=64, jitter=0.2, seed=2):
    m = box_mesh_3d(n, n, n, 1.0, 1.0, 1.0, jitter=jitter, seed=seed)
    set_patch(m, "zmin", "displacement", (0.0, 0.0, 0.0))
    set_patch(m, "zmax", "pressure", (10.0e6, 0.0, 0.0))
    mat = Material("linear_elastic", 200e9, 0.3, 1.0, 1.0)
    s = SolverSettings(n_increments=1, max_newton_it=1, eta=1e-10, restart=30, precond="jacobi")
    return dict(name="c2_cube3d_%d^3_jitter%g" % (n, jitter), mesh=m, material=mat, solver=s)


def cantilever_mesh(nx=1000, ny=100, nz=10, L=(10.0, 1.0, 1.0), tau=750.0):
    """Cantilever block clamped at x=0 with a dead shear traction tau*y on x=L."""
    m = box_mesh_3d(nx, ny, nz, L[0], L[1], L[2])
    set_patch(m, "xmin", "displacement", (0.0, 0.0, 0.0))
    set_patch(m, "xmax", "traction", (0.0, tau, 0.0))
    return m


def config_c3(nx=1000, ny=100, nz=10, n_increments=10, tau=750.0):
    m = cantilever_mesh(nx, ny, nz, tau=tau)
    mat = Material("neo_hookean", 1.0e6, 0.45, 1.0, 1.0)
    s = SolverSettings(n_increments=n_increments, max_newton_it=25, newton_rtol=1e-8,
                       eta=1e-3, restart=50, precond="amg32", flexible=True, cheb_degree=3)
    return dict(name="c3_cantilever_nh_%dx%dx%d" % (nx, ny, nz), mesh=m, material=mat, solver=s)


def bending_field(centroid_like_points, L=10.0, tip=3.0):
    """A smooth large-deflection-shaped displacement sampled at given points.

    Used as a representative deformed state for timing the neo-Hookean
    J.v on the cantilever (the cost of a J.v does not depend on the
    values).  Cubic Euler-Bernoulli shape u_y = tip*(x/L)^2*(3-x/L)/2 with
    the matching axial shortening of plane sections.
    """
    x = centroid_like_points[:, 0] / L
    y = centroid_like_points[:, 1] - 0.5
    uy = tip * x * x * (3.0 - x) / 2.0
    slope = tip * 3.0 * x * (2.0 - x) / (2.0 * L)
    ux = -y * slope
    out = np.zeros_like(centroid_like_points)
    out[:, 0] = ux
    out[:, 1] = uy
    return out


def random_unit_vector(n, seed):
    v = _rng(seed).standard_normal(n)
    return v / np.linalg.norm(v)


def random_field(n, seed, scale=1.0):
    return scale * _rng(seed).standard_normal(n)


def _block_problem(rng, n_cells_target, dim_choice=None, law="linear_elastic",
                   jitter=0.15, max_aspect=4.0):
    """One random block problem with roughly n_cells_target cells."""
    dim = dim_choice if dim_choice is not None else (2 if rng.random() < 0.5 else 3)
    aspect = np.exp(rng.uniform(0.0, np.log(max_aspect), size=dim))
    aspect /= aspect.min()
    # choose counts proportional to aspect with product ~ target
    s = (n_cells_target / np.prod(aspect)) ** (1.0 / dim)
    n = np.maximum(2, np.round(aspect * s).astype(int))
    Ls = tuple(float(a) for a in aspect)
    seed = int(rng.integers(0, 2**31 - 1))
    if dim == 2:
        m = box_mesh_2d(int(n[0]), int(n[1]), Ls[0], Ls[1], jitter=jitter, seed=seed)
        names = ["xmin", "xmax", "ymin", "ymax"]
    else:
        m = box_mesh_3d(int(n[0]), int(n[1]), int(n[2]), Ls[0], Ls[1], Ls[2], jitter=jitter, seed=seed)
        names = ["xmin", "xmax", "ymin", "ymax", "zmin", "zmax"]
    E = float(np.exp(rng.uniform(np.log(1e9), np.log(200e9)))) if law == "linear_elastic" \
        else float(np.exp(rng.uniform(np.log(1e5), np.log(1e7))))
    nu = float(rng.uniform(0.2, 0.45))
    order = rng.permutation(len(names))
    clamp = names[order[0]]
    set_patch(m, clamp, "displacement", (0.0,) * dim)
    n_trac = 1 + int(rng.integers(0, 2))
    target_strain = 1e-4 if law == "linear_elastic" else 0.005
    for t in range(n_trac):
        nm = names[order[1 + t]]
        d = rng.standard_normal(dim)
        d /= np.linalg.norm(d)
        mag = target_strain * E
        set_patch(m, nm, "traction", tuple(mag * d))
    mat = Material(law, E, nu, 1.0, 1.0)
    return m, mat


def config_c4(n_problems=512, seed=4, lo=1e3, hi=1e5):
    """Batched workload: list of (mesh, material) with log-uniform sizes."""
    rng = _rng(seed)
    probs = []
    for _ in range(n_problems):
        nc = float(np.exp(rng.uniform(math.log(lo), math.log(hi))))
        m, mat = _block_problem(rng, nc)
        probs.append(dict(mesh=m, material=mat))
    s = SolverSettings(n_increments=1, max_newton_it=1, eta=1e-8, restart=30,
                       precond="amg32", flexible=True)
    return dict(name="c4_batched_%d" % n_problems, problems=probs, solver=s)


def config_c5_stream(rate=200.0, duration=120.0, seed=5, lo=5e3, hi=2e6, nh_frac=0.3,
                     max_requests=None):
    """Poisson request stream: list of dict(t_arrival, mesh, material, n_increments)."""
    rng = _rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration:
            break
        nc = float(np.exp(rng.uniform(math.log(lo), math.log(hi))))
        law = "neo_hookean" if rng.random() < nh_frac else "linear_elastic"
        m, mat = _block_problem(rng, nc, dim_choice=3, law=law)
        inc = 1 if law == "linear_elastic" else int(rng.integers(1, 6))
        reqs.append(dict(t_arrival=t, mesh=m, material=mat, n_increments=inc))
        if max_requests is not None and len(reqs) >= max_requests:
            break
    return reqs
