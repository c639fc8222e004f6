"""Restarted, right-preconditioned (flexible) GMRES with CGS2 Arnoldi.

Paper: Section 3.2 uses GMRES as the inner Krylov solver of the
Jacobian-free Newton-Krylov method with right preconditioning,
J P^{-1} v ~ (R(u + eps P^{-1} v) - R(u)) / eps.  The orthogonalisation
(classical Gram-Schmidt applied twice) and the flexible form that keeps
the preconditioned vectors z_j = P^{-1} v_j (so the preconditioner may
change between steps) are the readings used here; for a fixed linear
preconditioner the flexible and the standard right-preconditioned
iterates coincide in exact arithmetic.

Algorithm per restart cycle (Saad's GMRES / FGMRES):
  r = b - A x, beta = |r|, v_0 = r / beta, g = beta e_0
  for j = 0..m-1:
     z_j = M v_j ; w = A z_j
     two passes of h = V_j^T w, w -= V_j h  (accumulate h)
     H[0..j, j] = h, H[j+1, j] = |w|, v_{j+1} = w / |w|
     Givens rotations reduce H to upper-triangular form; |g_{j+1}|
     is the residual norm of the least-squares problem
  y = H^{-1} g, x += Z y, then the true residual b - A x decides
  whether to restart.

Variants the paper's solver used (Section 3.2 and the solver settings of
Section 4): left preconditioning (left=True: the Arnoldi process runs on
M A with w = M A v_j, x += V y, and the residual that decides convergence is
M (b - A x) against rtol |M b|), and LGMRES augmentation (augment = k: in
every cycle after the first, the last k directions z_j are the normalised
corrections x_c - x_{c-1} of the most recent cycles, newest first, instead
of M v_j; Baker, Jessup & Manteuffel's augmented restarted GMRES written in
the flexible form).
"""

import numpy as np


def gmres(apply_A, b, x0=None, M=None, restart=30, rtol=1e-10, atol=0.0, max_it=10000,
          breakdown_rtol=1e-14, keep_basis=False, left=False, augment=0):
    """Return (x, info) with info = dict(converged, iterations, res_true, history).

    keep_basis=True also returns the last cycle's orthonormal basis in
    info["V"] (rows) for checking the orthogonalisation.
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    Mf = (lambda v: v) if M is None else M
    resid = (lambda v: Mf(v)) if left else (lambda v: v)
    bnorm = np.linalg.norm(resid(b))
    target = max(rtol * bnorm, atol)
    r = resid(b - apply_A(x)) if np.any(x) else resid(b)
    beta = np.linalg.norm(r)
    aug = []
    history = [beta]
    total = 0
    m = restart
    last_basis = None
    while True:
        if beta <= target or bnorm == 0.0:
            return x, _info(True, total, beta, history, last_basis)
        if total >= max_it:
            return x, _info(False, total, beta, history, last_basis)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            a = j - (m - augment)
            if left:
                w = Mf(apply_A(V[j]))
            else:
                Z[j] = aug[a] if 0 <= a < len(aug) else Mf(V[j])
                w = apply_A(Z[j])
            w0 = np.linalg.norm(w)
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rr = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / rr
            sn[j] = H[j + 1, j] / rr
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            history.append(abs(g[j + 1]))
            if hn <= breakdown_rtol * max(w0, 1e-300):
                break
            V[j + 1] = w / hn
            if abs(g[j + 1]) <= target or total >= max_it:
                break
        if keep_basis:
            last_basis = V[:k + 1].copy() if hn > breakdown_rtol * max(w0, 1e-300) else V[:k].copy()
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        delta = (V[:k] if left else Z[:k]).T @ y
        x = x + delta
        if augment > 0 and np.linalg.norm(delta) > 0:
            aug = ([delta / np.linalg.norm(delta)] + aug)[:augment]
        r = resid(b - apply_A(x))
        beta = np.linalg.norm(r)
        history.append(beta)


def _info(conv, total, beta, history, basis):
    out = dict(converged=conv, iterations=total, res_true=beta, history=history)
    if basis is not None:
        out["V"] = basis
    return out
