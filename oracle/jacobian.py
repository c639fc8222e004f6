"""Jacobian-vector products and the compact-stencil approximate Jacobian.

Paper passages:
  * J v ~ (R(u + eps v) - R(u)) / eps: Section 3.2, Eq. (JF).  The paper
    leaves the choice of eps open; the reading used here is the
    Walker-Pernice form eps = sqrt(eps_mach) sqrt(1 + ||u||_2) / ||v||_2.
  * Exact directional derivative for checking the finite difference:
    complex step, J v = Im R(u + i h v) / h (all residual arithmetic is
    analytic in u).
  * Central difference (the symmetric form of Eq. JF, second order in
    eps): (R(u + eps v) - R(u - eps v)) / (2 eps) with the step
    eps_mach^(1/3) sqrt(1 + ||u||_2) / ||v||_2 (the cube-root step that
    balances its truncation and rounding errors).
  * Approximate Jacobian J_tilde: Section 3.1, the block diagonal and
    off-diagonal coefficients after Eq. (SegSys): off-diagonal
    alpha K_bar |Delta||Gamma|/|d| I, diagonal minus the sum over
    internal and displacement faces; no inertia term (static problems),
    alpha = alpha_pc; with inertia (a problem carrying rho and dt) the
    diagonal also gets -9/4 rho Omega_P / dt^2 (the BDF2 term of the block
    diagonal coefficient).  Without symmetry planes the blocks are scalar
    times identity, so the scalar matrix is returned (component
    decoupling, Eq. SegSysX-Z).
  * Symmetry faces add a block proportional to n (x) n to the diagonal
    block.  Reading: the block is the derivative of the symmetry sum of
    the compact diffusion term that J_tilde is defined from (Section 3.1,
    Eq. diffusion), alpha K_bar |Delta_s|/|d_s| |Gamma_s| (R u_P - u_P),
    i.e. -2 alpha K_bar |Delta_s|/|d_s| |Gamma_s| n (x) n; the printed
    coefficient lacks the factor 2 of R - I = -2 n n.  With the factor, the
    J_tilde of a half mesh equals the J_tilde of the mirrored full mesh
    folded across the plane.
"""

import numpy as np
import scipy.sparse as sp

from .fv import residual, DISP

SQRT_EPS_MACH = np.sqrt(np.finfo(np.float64).eps)


def eps_walker_pernice(u, v):
    nv = np.linalg.norm(v)
    if nv == 0.0:
        return 0.0
    return SQRT_EPS_MACH * np.sqrt(1.0 + np.linalg.norm(u)) / nv


def eps_central(u, v):
    nv = np.linalg.norm(v)
    if nv == 0.0:
        return 0.0
    return np.cbrt(np.finfo(np.float64).eps) * np.sqrt(1.0 + np.linalg.norm(u)) / nv


def jv_fd_central(u, v, pr, load=1.0, eps=None):
    """Central-difference J v; returns (Jv, eps)."""
    u = np.asarray(u, dtype=np.float64).reshape(-1)
    v = np.asarray(v, dtype=np.float64).reshape(-1)
    if eps is None:
        eps = eps_central(u, v)
    if eps == 0.0:
        return np.zeros_like(v), 0.0
    Rp = residual(u + eps * v, pr, load).reshape(-1)
    Rm = residual(u - eps * v, pr, load).reshape(-1)
    return (Rp - Rm) / (2.0 * eps), eps


def jv_fd(u, v, pr, load=1.0, eps=None, Ru=None):
    """Finite-difference J v (Eq. JF); returns (Jv, eps)."""
    u = np.asarray(u, dtype=np.float64).reshape(-1)
    v = np.asarray(v, dtype=np.float64).reshape(-1)
    if eps is None:
        eps = eps_walker_pernice(u, v)
    if eps == 0.0:
        return np.zeros_like(v), 0.0
    if Ru is None:
        Ru = residual(u, pr, load).reshape(-1)
    Rp = residual(u + eps * v, pr, load).reshape(-1)
    return (Rp - Ru) / eps, eps


def jv_complex_step(u, v, pr, load=1.0, h=1e-30):
    """Exact J v by the complex step: Im R(u + i h v) / h."""
    u = np.asarray(u, dtype=np.float64).reshape(-1)
    v = np.asarray(v, dtype=np.float64).reshape(-1)
    return residual(u + 1j * h * v, pr, load).reshape(-1).imag / h


def brute_force_jacobian(u, pr, load=1.0, h=1e-30):
    """Dense J, column j = complex-step J e_j (tiny meshes only)."""
    u = np.asarray(u, dtype=np.float64).reshape(-1)
    n = u.size
    J = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        J[:, j] = jv_complex_step(u, e, pr, load, h)
    return J


def approximate_jacobian(pr):
    """J_tilde as a sparse [n_cells*dim]^2 matrix (cells interleaved with
    components), including the n (x) n blocks of symmetry faces."""
    nc, dim = pr["nc"], pr["dim"]
    A = sp.kron(_scalar_part(pr), sp.identity(dim), format="csr")
    sym = pr["sym"]
    if sym.size == 0:
        return A
    c = pr["mat"]
    aK = c["alpha_pc"] * c["Kbar"]
    coef = 2.0 * aK / pr["magds"] * pr["magGb"][sym]      # |Delta_s| = 1
    ns = pr["ns"]
    blocks = -coef[:, None, None] * ns[:, :, None] * ns[:, None, :]
    Ps = pr["Ps"]
    shape = blocks.shape
    rows = np.broadcast_to(Ps[:, None, None] * dim + np.arange(dim)[None, :, None], shape)
    cols = np.broadcast_to(Ps[:, None, None] * dim + np.arange(dim)[None, None, :], shape)
    S = sp.csr_matrix((blocks.reshape(-1), (rows.reshape(-1), cols.reshape(-1))), shape=A.shape)
    return (A + S).tocsr()


def approximate_jacobian_scalar(pr):
    """Scalar matrix A with J_tilde = A (x) I_dim (cells interleaved with
    components); only for meshes without symmetry planes."""
    if pr["sym"].size:
        raise ValueError("J_tilde of a mesh with symmetry planes is not scalar; use approximate_jacobian")
    return _scalar_part(pr)


def _scalar_part(pr):
    """The scalar (component-independent) part of J_tilde."""
    c = pr["mat"]
    aK = c["alpha_pc"] * c["Kbar"]
    nc = pr["nc"]
    P, N = pr["P"], pr["N"]
    coef = aK * pr["magDelta"] / pr["magd"] * pr["magG"]
    m = pr["btype"] == DISP
    coef_b = aK * pr["magDeltab"][m] / pr["magdb"][m] * pr["magGb"][m]
    diag = -(np.bincount(P, weights=coef, minlength=nc) + np.bincount(N, weights=coef, minlength=nc)
             + np.bincount(pr["Pb"][m], weights=coef_b, minlength=nc))
    src = pr.get("source") or {}
    if "rho" in src:
        diag = diag - 2.25 * src["rho"] * pr["geo"]["V"] / src["dt"] ** 2
    rows = np.concatenate([P, N, np.arange(nc)])
    cols = np.concatenate([N, P, np.arange(nc)])
    vals = np.concatenate([coef, coef, diag])
    return sp.csr_matrix((vals, (rows, cols)), shape=(nc, nc))
