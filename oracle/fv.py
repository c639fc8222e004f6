"""Residual R(u) of the cell-centred finite-volume momentum balance.

Paper passages followed (Cardiff et al., arXiv 2502.17217):
  * Residual form R(u) = 0 and the static linear-geometry residual:
    Section 2.2, Eq. (residual); total Lagrangian form for finite strain:
    Appendix A, Eq. (momentum_TL), with F = I + (grad u)^T.
  * Surface integral by one-point quadrature per face: Section 2.3.2,
    Eq. (divStressDiscret): internal faces Gamma_f . sigma_f, displacement
    faces Gamma_d . sigma_P, traction faces |Gamma_t| T_bar.
  * Interpolation weight w_f = n.(x_N - x_f) / n.(x_N - x_P):
    Eq. (stressInterp).
  * Least-squares cell gradient: Eq. (leastSquaresGrad) and the G_P
    tensor that follows it; boundary faces are excluded.
  * Rhie-Chow stabilisation: Section 2.3.3, Eq. (RhieChow), with
    K_bar = 2 mu + lambda and Delta = d/(d.n).
  * Laws: Appendix B, Eq. (linearElastic), Eq. (neoHook) and the
    St. Venant-Kirchhoff law with Eq. (S2sigma).
  * Volume terms (Section 2.3.1, Eq. volume_integral, midpoint rule): the
    body force f_b Omega_P and the inertia -rho Omega_P a_P with the BDF2
    acceleration of Eq. (inertia2); both enter the residual of Section 2.2
    as R = surface terms + int f_b - int rho d2u/dt2.

Readings where the paper is silent or inconsistent (all listed in the
design notes of the repository):
  * LS weights: the gradient sum uses w_f|Gamma| but G_P uses
    (1-w_f)|Gamma|; the two agree only when w_f = 1/2.  One weight
    omega_f = |Gamma_f| is used in both, which keeps the stated
    exactness for linear fields on distorted meshes.
  * Face quantities: the face stress is sigma(grad u_f) with
    grad u_f = w_f grad u_P + (1 - w_f) grad u_N (identical to
    interpolating cell stresses for the linear law); the face gradient
    in the Rhie-Chow term uses the same interpolation.
  * Finite strain: total Lagrangian on the fixed reference mesh; the
    face traction is (cof F_f Gamma_o) . sigma(F_f); displacement faces
    use F_P.  The Rhie-Chow term keeps K_bar = 2 mu + lambda.
  * Prescribed boundary values (displacements, tractions, pressures) are
    all multiplied by the load factor of the current increment;
    a pressure patch applies the dead load -p Gamma_o.
  * Symmetry planes (Section 2.3.2, Eq. symm, and the symmetry sums of
    Eq. leastSquaresGrad and Eq. RhieChow): the face sees the mirror
    image of cell P, x_P' = x_P + d_s with d_s = 2 ((x_f - x_P).n) n,
    u_P' = R u_P and grad u_P' = R grad u_P R, R = I - 2 n n.  The face
    gradient is the average grad u_s = (grad u_P + R grad u_P R)/2 and the
    face stress is the law evaluated at it, as on internal faces (for the
    linear law this is (sigma_P + R sigma_P R)/2, whose traction is the
    normal part (n.sigma_P.n) n).  The printed second line of Eq. symm,
    (I - n n).sigma_P, has zero traction on the face and is not used.
    The least-squares weight is |Gamma_s| as on internal faces.
  * Plane strain (2-D): unit depth; the neo-Hookean law works on the
    3x3 tensors with F_zz = 1.

All functions accept real or complex displacements; nothing non-analytic
is applied to u, so the complex step gives exact derivatives.
"""

import numpy as np

from .geometry import mesh_geometry

DISP, TRAC, PRES, SYMM = 1, 2, 3, 4
_TYPE = {"displacement": DISP, "traction": TRAC, "pressure": PRES, "symmetry": SYMM}


def reflect_vector(u, n):
    """R u with R = I - 2 n n (mirror image across the plane of normal n)."""
    return u - 2.0 * np.einsum("fi,fi->f", u, n)[:, None] * n


def reflect_tensor(g, n):
    """R g R, the mirror image of a second-order tensor field."""
    gn = np.einsum("fij,fj->fi", g, n)          # g . n
    ng = np.einsum("fi,fij->fj", n, g)          # n . g
    ngn = np.einsum("fi,fi->f", ng, n)
    return (g - 2.0 * gn[:, :, None] * n[:, None, :] - 2.0 * n[:, :, None] * ng[:, None, :]
            + 4.0 * ngn[:, None, None] * n[:, :, None] * n[:, None, :])


def material_constants(mat):
    """Lame constants, bulk modulus and K_bar (Appendix B; Section 2.3.3)."""
    E, nu = float(mat.E), float(mat.nu)
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    kappa = E / (3.0 * (1.0 - 2.0 * nu))
    return dict(mu=mu, lam=lam, kappa=kappa, Kbar=2.0 * mu + lam,
                law=mat.law, alpha_rc=float(mat.alpha_rc), alpha_pc=float(mat.alpha_pc))


def _scatter(idx, vals, n):
    """out[idx[i]] += vals[i] along axis 0; works for real and complex."""
    if np.iscomplexobj(vals):
        return _scatter(idx, vals.real, n) + 1j * _scatter(idx, vals.imag, n)
    flat = vals.reshape(vals.shape[0], -1)
    out = np.stack([np.bincount(idx, weights=flat[:, k], minlength=n)
                    for k in range(flat.shape[1])], axis=1)
    return out.reshape((n,) + vals.shape[1:])


def prepare(mesh, mat):
    """Mesh-only and material-only quantities (computed once per mesh)."""
    dim = mesh["dim"]
    geo = mesh_geometry(mesh)
    n_int = mesh["n_internal"]
    nf = mesh["n_faces"]
    nc = mesh["n_cells"]
    P = mesh["owner"][:n_int].astype(np.int64)
    N = mesh["neighbour"].astype(np.int64)
    Gam = geo["Gamma"][:n_int]
    magG = np.linalg.norm(Gam, axis=1)
    n = Gam / magG[:, None]
    xP, xN, xf = geo["xc"][P], geo["xc"][N], geo["xf"][:n_int]
    d = xN - xP
    dn = np.einsum("fi,fi->f", d, n)
    if np.any(dn <= 0.0):
        raise ValueError("internal face with d.n <= 0")
    w = np.einsum("fi,fi->f", n, xN - xf) / dn          # Eq. (stressInterp)
    Delta = d / dn[:, None]                             # over-relaxed vector
    magd = np.linalg.norm(d, axis=1)
    magDelta = np.linalg.norm(Delta, axis=1)

    # boundary faces
    Pb = mesh["owner"][n_int:].astype(np.int64)
    Gb = geo["Gamma"][n_int:]
    magGb = np.linalg.norm(Gb, axis=1)
    nb_hat = Gb / magGb[:, None]
    db = geo["xf"][n_int:] - geo["xc"][Pb]
    dbn = np.einsum("fi,fi->f", db, nb_hat)
    btype = np.zeros(nf - n_int, dtype=np.int64)
    bval = np.zeros((nf - n_int, dim))
    for p in mesh["patches"]:
        s = slice(p["start"] - n_int, p["start"] - n_int + p["size"])
        btype[s] = _TYPE[p["type"]]
        if p.get("per_face") is not None:
            bval[s] = p["per_face"]
        else:
            bval[s] = np.asarray(p["value"][:dim])
    if np.any(btype == 0):
        raise ValueError("boundary face without a patch")
    disp = btype == DISP
    if np.any(dbn[disp] <= 0.0):
        raise ValueError("displacement face with d.n <= 0")
    with np.errstate(divide="ignore", invalid="ignore"):
        Deltab = np.where(disp[:, None], db / dbn[:, None], 0.0)

    # symmetry faces: the mirror image of x_P lies at x_P + d_s
    sym = np.nonzero(btype == SYMM)[0]
    if np.any(dbn[sym] <= 0.0):
        raise ValueError("symmetry face with d.n <= 0")
    Ps, ns = Pb[sym], nb_hat[sym]
    ds = 2.0 * dbn[sym][:, None] * ns
    magGs = magGb[sym]

    # least-squares vectors, omega_f = |Gamma_f| in both sum and G_P
    dd = np.einsum("fi,fi->f", d, d)
    outer = magG[:, None, None] * d[:, :, None] * d[:, None, :] / dd[:, None, None]
    G = _scatter(P, outer, nc) + _scatter(N, outer, nc)
    dds = np.einsum("fi,fi->f", ds, ds)
    if sym.size:
        G = G + _scatter(Ps, magGs[:, None, None] * ds[:, :, None] * ds[:, None, :] / dds[:, None, None], nc)
    Ginv = np.linalg.inv(G)
    c_own = magG[:, None] * np.einsum("fij,fj->fi", Ginv[P], d) / dd[:, None]
    c_nb = magG[:, None] * np.einsum("fij,fj->fi", Ginv[N], -d) / dd[:, None]
    c_sym = magGs[:, None] * np.einsum("fij,fj->fi", Ginv[Ps], ds) / dds[:, None]
    return dict(mesh=mesh, dim=dim, nc=nc, n_int=n_int, geo=geo, mat=material_constants(mat),
                P=P, N=N, Gam=Gam, magG=magG, n=n, d=d, magd=magd, w=w, Delta=Delta,
                magDelta=magDelta, G=G, c_own=c_own, c_nb=c_nb,
                Pb=Pb, Gb=Gb, magGb=magGb, db=db, magdb=np.linalg.norm(db, axis=1),
                Deltab=Deltab, magDeltab=np.linalg.norm(Deltab, axis=1),
                btype=btype, bval=bval,
                sym=sym, Ps=Ps, ns=ns, ds=ds, magds=np.linalg.norm(ds, axis=1), c_sym=c_sym)


def gradient(u, pr):
    """Least-squares cell gradient, (grad u)_P[i, j] = d u_j / d x_i.

    Eq. (leastSquaresGrad): sum over internal faces of c_{P,f} (x) (u_N - u_P)
    plus, over symmetry faces, c_{P,s} (x) (R_s u_P - u_P).
    """
    P, N = pr["P"], pr["N"]
    du = u[N] - u[P]
    g_own = pr["c_own"][:, :, None] * du[:, None, :]
    g_nb = pr["c_nb"][:, :, None] * (-du)[:, None, :]
    g = _scatter(P, g_own, pr["nc"]) + _scatter(N, g_nb, pr["nc"])
    if pr["sym"].size:
        Ps = pr["Ps"]
        dus = reflect_vector(u[Ps], pr["ns"]) - u[Ps]
        g = g + _scatter(Ps, pr["c_sym"][:, :, None] * dus[:, None, :], pr["nc"])
    return g


def stress_linear_elastic(g, c):
    """Eq. (linearElastic): sigma = mu grad u + mu grad u^T + lambda tr(grad u) I."""
    dim = g.shape[-1]
    tr = np.trace(g, axis1=-2, axis2=-1)
    eye = np.eye(dim)
    return c["mu"] * (g + np.swapaxes(g, -1, -2)) + c["lam"] * tr[..., None, None] * eye


def _embed3(g):
    if g.shape[-1] == 3:
        return g
    out = np.zeros(g.shape[:-2] + (3, 3), dtype=g.dtype)
    out[..., :2, :2] = g
    return out


def cofactor(F):
    """cof F = det(F) F^{-T} for 3x3 tensors (polynomial, so complex-safe)."""
    c = np.empty_like(F)
    c[..., 0, 0] = F[..., 1, 1] * F[..., 2, 2] - F[..., 1, 2] * F[..., 2, 1]
    c[..., 0, 1] = F[..., 1, 2] * F[..., 2, 0] - F[..., 1, 0] * F[..., 2, 2]
    c[..., 0, 2] = F[..., 1, 0] * F[..., 2, 1] - F[..., 1, 1] * F[..., 2, 0]
    c[..., 1, 0] = F[..., 0, 2] * F[..., 2, 1] - F[..., 0, 1] * F[..., 2, 2]
    c[..., 1, 1] = F[..., 0, 0] * F[..., 2, 2] - F[..., 0, 2] * F[..., 2, 0]
    c[..., 1, 2] = F[..., 0, 1] * F[..., 2, 0] - F[..., 0, 0] * F[..., 2, 1]
    c[..., 2, 0] = F[..., 0, 1] * F[..., 1, 2] - F[..., 0, 2] * F[..., 1, 1]
    c[..., 2, 1] = F[..., 0, 2] * F[..., 1, 0] - F[..., 0, 0] * F[..., 1, 2]
    c[..., 2, 2] = F[..., 0, 0] * F[..., 1, 1] - F[..., 0, 1] * F[..., 1, 0]
    return c


def neo_hookean(g, c):
    """Eq. (neoHook) with F = I + (grad u)^T (Appendix A).

    Returns (sigma, cof F), both 3x3.
    """
    g3 = _embed3(g)
    F = np.eye(3) + np.swapaxes(g3, -1, -2)
    cof = cofactor(F)
    J = np.einsum("...j,...j->...", F[..., 0, :], cof[..., 0, :])   # expansion along row 0
    b = F @ np.swapaxes(F, -1, -2)
    bbar = np.power(J, -2.0 / 3.0)[..., None, None] * b
    dev = bbar - (np.trace(bbar, axis1=-2, axis2=-1) / 3.0)[..., None, None] * np.eye(3)
    sigma = (c["mu"] / J)[..., None, None] * dev \
        + (0.5 * c["kappa"] * (J * J - 1.0) / J)[..., None, None] * np.eye(3)
    return sigma, cof


def st_venant_kirchhoff(g, c):
    """Appendix B: S = 2 mu E + lambda tr(E) I with the Green strain
    E = (grad u + grad u^T + grad u . grad u^T)/2, and Eq. (S2sigma)
    sigma = F S F^T / J.  Returns (sigma, cof F), both 3x3."""
    g3 = _embed3(g)
    F = np.eye(3) + np.swapaxes(g3, -1, -2)
    E = 0.5 * (g3 + np.swapaxes(g3, -1, -2) + g3 @ np.swapaxes(g3, -1, -2))
    trE = np.trace(E, axis1=-2, axis2=-1)
    S = 2.0 * c["mu"] * E + (c["lam"] * trE)[..., None, None] * np.eye(3)
    cof = cofactor(F)
    J = np.einsum("...j,...j->...", F[..., 0, :], cof[..., 0, :])
    sigma = F @ S @ np.swapaxes(F, -1, -2) / J[..., None, None]
    return sigma, cof


def traction(g, Gam, c):
    """Force on an area vector Gamma from the stress at displacement gradient g.

    Linear geometry: Gamma . sigma(g) (Eq. divStressDiscret).
    Total Lagrangian: (J F^{-T} Gamma_o) . sigma with J F^{-T} = cof F
    (Eq. momentum_TL).
    """
    dim = g.shape[-1]
    if c["law"] == "linear_elastic":
        s = stress_linear_elastic(g, c)
        return np.einsum("fi,fij->fj", Gam, s)
    if c["law"] in ("neo_hookean", "st_venant_kirchhoff"):
        s, cof = neo_hookean(g, c) if c["law"] == "neo_hookean" else st_venant_kirchhoff(g, c)
        G3 = np.zeros((Gam.shape[0], 3))
        G3[:, :dim] = Gam
        a = np.einsum("fik,fk->fi", cof, G3)
        t = np.einsum("fi,fij->fj", a, s)
        return t[:, :dim]
    raise ValueError("unknown law %r" % (c["law"],))


def face_forces(u, pr, load=1.0):
    """Per-face forces of Eq. (divStressDiscret) and Eq. (RhieChow).

    Returns dict(T_int, RC_int, T_b, RC_b, grad): the traction and the
    Rhie-Chow force on every internal face (owner side, outward from the
    owner) and every boundary face, and the cell gradients.
    """
    c = pr["mat"]
    nc, dim = pr["nc"], pr["dim"]
    u = np.asarray(u).reshape(nc, dim)
    g = gradient(u, pr)
    P, N, w = pr["P"], pr["N"], pr["w"]
    aK = c["alpha_rc"] * c["Kbar"]

    # internal faces
    gf = w[:, None, None] * g[P] + (1.0 - w)[:, None, None] * g[N]
    T_int = traction(gf, pr["Gam"], c)
    jump = (pr["magDelta"] / pr["magd"])[:, None] * (u[N] - u[P])
    Dg = np.einsum("fi,fij->fj", pr["Delta"], gf)
    RC_int = aK * (jump - Dg) * pr["magG"][:, None]

    # boundary faces
    Pb, bt = pr["Pb"], pr["btype"]
    T_b = np.zeros((Pb.shape[0], dim), dtype=np.result_type(u, float))
    RC_b = np.zeros_like(T_b)
    m = bt == DISP
    if np.any(m):
        gP = g[Pb[m]]
        T_b[m] = traction(gP, pr["Gb"][m], c)
        ubar = load * pr["bval"][m]
        jumpb = (pr["magDeltab"][m] / pr["magdb"][m])[:, None] * (ubar - u[Pb[m]])
        Dgb = np.einsum("fi,fij->fj", pr["Deltab"][m], gP)
        RC_b[m] = aK * (jumpb - Dgb) * pr["magGb"][m][:, None]
    sym = pr["sym"]
    if sym.size:
        # Eq. (symm): the face sees cell P and its mirror image
        Ps, ns = pr["Ps"], pr["ns"]
        gP = g[Ps]
        gs = 0.5 * (gP + reflect_tensor(gP, ns))
        T_b[sym] = traction(gs, pr["Gb"][sym], c)
        Deltas = pr["ds"] / np.einsum("fi,fi->f", pr["ds"], ns)[:, None]     # = n
        jumps = (np.linalg.norm(Deltas, axis=1) / pr["magds"])[:, None] * \
            (reflect_vector(u[Ps], ns) - u[Ps])
        Dgs = np.einsum("fi,fij->fj", Deltas, gs)
        RC_b[sym] = aK * (jumps - Dgs) * pr["magGb"][sym][:, None]
    m = bt == TRAC
    T_b[m] = load * pr["magGb"][m][:, None] * pr["bval"][m]
    m = bt == PRES
    T_b[m] = -load * pr["bval"][m][:, :1] * pr["Gb"][m]
    return dict(T_int=T_int, RC_int=RC_int, T_b=T_b, RC_b=RC_b, grad=g)


def with_source(pr, body=None, rho=0.0, dt=0.0, u_n=None, u_nm1=None, v_n=None, v_nm1=None):
    """A copy of the prepared problem whose residual includes volume terms:
    a body force density `body` [n_cells, dim] (force per unit volume,
    scaled by the load factor like every other load) and, with rho > 0 and
    dt > 0, the inertia of Eq. (inertia2) from the previous displacements
    u_n, u_nm1 and velocities v_n, v_nm1 ([n_cells, dim] each)."""
    q = dict(pr)
    nc, dim = pr["nc"], pr["dim"]
    src = {}
    if body is not None:
        src["body"] = np.asarray(body, dtype=np.float64).reshape(nc, dim)
    if rho > 0 and dt > 0:
        src.update(rho=float(rho), dt=float(dt),
                   u_n=np.asarray(u_n, dtype=np.float64).reshape(nc, dim),
                   u_nm1=np.asarray(u_nm1, dtype=np.float64).reshape(nc, dim),
                   v_n=np.asarray(v_n, dtype=np.float64).reshape(nc, dim),
                   v_nm1=np.asarray(v_nm1, dtype=np.float64).reshape(nc, dim))
    q["source"] = src
    return q


def bdf2_velocity(u, u_n, u_nm1, dt):
    """v^{t+1} = (3 u^{t+1} - 4 u^t + u^{t-1}) / (2 dt) (BDF2, Section 2.3.1)."""
    return (3.0 * u - 4.0 * u_n + u_nm1) / (2.0 * dt)


def bdf2_acceleration(u, src):
    """Eq. (inertia2): (3 v^{t+1} - 4 v^t + v^{t-1}) / (2 dt) with v^{t+1}
    the BDF2 velocity of u."""
    v = bdf2_velocity(u, src["u_n"], src["u_nm1"], src["dt"])
    return (3.0 * v - 4.0 * src["v_n"] + src["v_nm1"]) / (2.0 * src["dt"])


def volume_terms(u, pr, load=1.0):
    """Body force and inertia of cell P integrated by the midpoint rule:
    load f_b,P Omega_P - rho a_P Omega_P (zero when no source is set)."""
    src = pr.get("source") or {}
    nc, dim = pr["nc"], pr["dim"]
    u = np.asarray(u).reshape(nc, dim)
    V = pr["geo"]["V"][:, None]
    out = np.zeros((nc, dim), dtype=np.result_type(u, float))
    if "body" in src:
        out = out + load * src["body"] * V
    if "rho" in src:
        out = out - src["rho"] * V * bdf2_acceleration(u, src)
    return out


def residual(u, pr, load=1.0, parts=False):
    """R(u) per cell, shape [n_cells, dim] (Eq. residual).

    R_P = sum_f [traction_f + Rhie-Chow_f] with outward orientation: each
    internal face is evaluated once from its owner's side and added to the
    owner and subtracted from the neighbour; plus the volume terms (body
    force, inertia) when the problem carries them (with_source).
    """
    nc = pr["nc"]
    P, N, Pb = pr["P"], pr["N"], pr["Pb"]
    ff = face_forces(u, pr, load)

    def assemble(fint, fb):
        return (_scatter(P, fint, nc) - _scatter(N, fint, nc) + _scatter(Pb, fb, nc))

    if parts:
        return dict(traction=assemble(ff["T_int"], ff["T_b"]), rc=assemble(ff["RC_int"], ff["RC_b"]),
                    grad=ff["grad"], volume=volume_terms(u, pr, load))
    R = assemble(ff["T_int"] + ff["RC_int"], ff["T_b"] + ff["RC_b"])
    if pr.get("source"):
        R = R + volume_terms(u, pr, load)
    return R
