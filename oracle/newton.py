"""Jacobian-free Newton-Krylov with equal load increments.

Paper passages:
  * Newton-Raphson J(u_k) du = -R(u_k), u_{k+1} = u_k + s du with s = 1:
    Section 2.2, Eq. (NewtonRaphson).
  * Matrix-free J v by finite differences inside GMRES: Section 3.2.
  * Preconditioner from the compact-stencil approximate Jacobian
    J_tilde: Section 3.2 (physics-based preconditioner); the paper's
    direct-LU option is reproduced with a sparse LU of the scalar
    J_tilde applied to each displacement component.
  * Inexact Newton: the linear system is solved to a relative tolerance
    eta (three orders in the paper): Section 3.2, oversolving.
  * Convergence per load step: |R(u)| <= max(rtol |R(u_0)|, atol) with
    the Euclidean norm, or, when stol > 0, a correction |s du| <= stol |u|
    (the third check of Section 3.3; the paper runs with stol = 0, the
    default here).
  * Load increments: equal fractions k/N of the applied loads (the
    case descriptions apply loads in equal increments); the next
    increment starts from the previous converged displacement.
  * Globalisation by line search (Section 3.2): the step length s > 0
    only has to decrease the residual norm.  Reading: s = 1, 1/2, 1/4,
    ... and the first s with |R(u + s du)| < |R(u)| is taken (a NaN
    residual is no decrease); after max_backtrack halvings the last trial
    is taken.  Without line search s = 1.
  * Divergence: a residual above dtol |R(u_0)| ends the solve.
  * jv="complex_step" replaces the finite difference inside GMRES by the
    exact directional derivative Im R(u + i h v)/h (a Newton-Krylov solve
    with the exact Jacobian action).  The converged displacement is the
    same discrete solution; reference solutions use it because the
    finite difference of the neo-Hookean law as literally written loses
    digits to cancellation near the reference state.
"""

import numpy as np
import scipy.sparse.linalg as spla

from .fv import residual
from .jacobian import jv_fd, jv_complex_step, approximate_jacobian, approximate_jacobian_scalar
from .krylov import gmres


def make_preconditioner(pr, kind):
    """Return z = M r for r in interleaved [cell][component] order."""
    nc, dim = pr["nc"], pr["dim"]
    if kind in (None, "none"):
        return None
    if pr["sym"].size:
        # symmetry planes couple the components of J_tilde (n (x) n blocks):
        # the block matrix itself, in the interleaved order
        B = approximate_jacobian(pr).tocsc()
        if kind == "jacobi":
            dinv = 1.0 / B.diagonal()
            return lambda r: dinv * r
        if kind == "lu":
            lu = spla.splu(B)
            return lambda r: lu.solve(np.ascontiguousarray(r))
        if kind == "cg":
            dinv = 1.0 / B.diagonal()
            Md = spla.LinearOperator(B.shape, matvec=lambda x: dinv * x)
            Bcsr = B.tocsr()

            def apply_block(r):
                out, info = spla.cg(Bcsr, r, M=Md, rtol=1e-10, atol=0.0, maxiter=20000)
                if info != 0:
                    raise RuntimeError("cg preconditioner did not converge")
                return out
            return apply_block
        raise ValueError(kind)
    A = approximate_jacobian_scalar(pr).tocsc()
    if kind == "jacobi":
        dinv = 1.0 / A.diagonal()
        return lambda r: (r.reshape(nc, dim) * dinv[:, None]).reshape(-1)
    if kind == "lu":
        lu = spla.splu(A)
        return lambda r: lu.solve(np.ascontiguousarray(r.reshape(nc, dim))).reshape(-1)
    if kind == "cg":
        # the same A^{-1}, applied by a library conjugate-gradient solve per
        # component (diagonally scaled, to 1e-10 relative): for meshes whose
        # sparse LU fill is too large; the application is then slightly
        # inexact, which the flexible GMRES form allows
        dinv = 1.0 / A.diagonal()
        Md = spla.LinearOperator(A.shape, matvec=lambda x: dinv * x)
        Acsr = A.tocsr()

        def apply(r):
            rr = r.reshape(nc, dim)
            out = np.empty_like(rr)
            for k in range(dim):
                out[:, k], info = spla.cg(Acsr, rr[:, k], M=Md, rtol=1e-10, atol=0.0, maxiter=20000)
                if info != 0:
                    raise RuntimeError("cg preconditioner did not converge")
            return out.reshape(-1)
        return apply
    raise ValueError(kind)


def newton_solve(pr, u0=None, n_increments=1, rtol=1e-6, atol=1e-50, max_newton_it=20,
                 eta=1e-3, restart=30, precond="lu", max_krylov_it=5000, line_search=False,
                 max_backtrack=8, dtol=1e8, monitor=None, jv="fd", stol=0.0):
    """Solve R(u) = 0 under equal load increments; returns (u, stats).

    stats["status"] is "ok", "not_converged", "diverged" or "nan".
    monitor(increment, iteration, |R|/|R_0|, gmres iterations) is called
    after every Newton iteration when given (progress output only)."""
    nc, dim = pr["nc"], pr["dim"]
    u = np.zeros(nc * dim) if u0 is None else np.array(u0, dtype=np.float64).reshape(-1)
    M = make_preconditioner(pr, precond)
    stats = dict(newton_it=[], gmres_it=[], res0=[], res_final=[], converged=True, status="ok",
                 steps=[])
    for k in range(1, n_increments + 1):
        load = k / n_increments
        R = residual(u, pr, load).reshape(-1)
        r0 = np.linalg.norm(R)
        rn = r0
        it = 0
        gm = 0
        while True:
            rn = np.linalg.norm(R)
            if rn <= max(rtol * r0, atol):
                break
            if not np.isfinite(rn):
                stats["converged"] = False
                stats["status"] = "nan"
                break
            if it >= max_newton_it:
                stats["converged"] = False
                stats["status"] = "not_converged"
                break
            if rn > dtol * max(r0, 1e-300):
                stats["converged"] = False
                stats["status"] = "diverged"
                break
            Ru = R

            if jv == "complex_step":
                def A(z, u=u):
                    return jv_complex_step(u, z, pr, load)
            else:
                def A(z, u=u, Ru=Ru):
                    return jv_fd(u, z, pr, load, Ru=Ru)[0]

            du, info = gmres(A, -R, M=M, restart=restart, rtol=eta, max_it=max_krylov_it)
            gm += info["iterations"]
            s = 1.0
            u_new = u + du
            R_new = residual(u_new, pr, load).reshape(-1)
            if line_search:
                for _ in range(max_backtrack):
                    if np.linalg.norm(R_new) < rn:
                        break
                    s *= 0.5
                    u_new = u + s * du
                    R_new = residual(u_new, pr, load).reshape(-1)
            stats["steps"].append(s)
            small_step = stol > 0 and s * np.linalg.norm(du) <= stol * np.linalg.norm(u_new)
            u, R = u_new, R_new
            it += 1
            if monitor is not None:
                monitor(k, it, np.linalg.norm(R) / r0, info["iterations"])
            if small_step:
                break
        stats["newton_it"].append(it)
        stats["gmres_it"].append(gm)
        stats["res0"].append(r0)
        stats["res_final"].append(np.linalg.norm(R))
        if not stats["converged"]:
            break
    return u, stats


def dynamic_solve(pr, rho, dt, n_steps, body=None, predictor=True, **newton_kw):
    """Transient solve with the BDF2 inertia of Section 2.3.1, Eq. (inertia2).

    Starts from rest (u = v = 0; the values before the first step are taken
    equal to those at t = 0, and the acceleration at t = 0 is zero).  Each
    step solves R(u^{t+1}) = 0 with Newton (loads at their full value),
    starting from the truncated Taylor predictor of Section 3.2, Eq.
    (predictor), u^t + dt v^t + dt^2/2 a^t (or from u^t when predictor is
    False), then updates v^{t+1} by BDF2 and a^{t+1} by BDF2 of the
    velocities.  Returns (list of displacements per step, list of Newton
    stats per step)."""
    from .fv import with_source, bdf2_velocity
    nc, dim = pr["nc"], pr["dim"]
    u_n = np.zeros(nc * dim)
    u_nm1 = u_n.copy()
    v_n = np.zeros(nc * dim)
    v_nm1 = v_n.copy()
    a_n = np.zeros(nc * dim)
    us, stats = [], []
    for _ in range(n_steps):
        q = with_source(pr, body=body, rho=rho, dt=dt, u_n=u_n, u_nm1=u_nm1, v_n=v_n, v_nm1=v_nm1)
        guess = u_n + dt * v_n + 0.5 * dt * dt * a_n if predictor else u_n.copy()
        u, st = newton_solve(q, u0=guess, n_increments=1, **newton_kw)
        v = bdf2_velocity(u, u_n, u_nm1, dt)
        a_n = (3.0 * v - 4.0 * v_n + v_nm1) / (2.0 * dt)
        u_nm1, u_n = u_n, u
        v_nm1, v_n = v_n, v
        us.append(u.copy())
        stats.append(st)
    return us, stats
