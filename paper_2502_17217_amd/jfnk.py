"""Python binding of libjfnk.so (include/jfnk.h): argument marshalling only.

Every computation runs in the HIP library; this module converts mesh
dictionaries (see ``meshgen``) and torch CUDA tensors into the C ABI's
structures and raw device pointers.  Torch is used for device memory and
streams only.  If the library is not built, importing this module fails.
"""

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjfnk.so")

OK, E_ARG, E_MESH, E_OOM, E_HIP, E_NOT_CONVERGED, E_DIVERGED, E_NAN, E_BREAKDOWN, E_BUSY = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_MESH", -3: "E_OOM", -4: "E_HIP", -5: "E_NOT_CONVERGED",
                -6: "E_DIVERGED", -7: "E_NAN", -8: "E_BREAKDOWN", -9: "E_BUSY"}
BC = {"displacement": 1, "traction": 2, "pressure": 3, "symmetry": 4}
LAW = {"linear_elastic": 0, "neo_hookean": 1, "st_venant_kirchhoff": 2}
PC_NONE, PC_JACOBI, PC_AMG32, PC_AMG64 = 0, 1, 2, 3
PC_Z32 = 16  # ORed into a precond value: the flexible-GMRES directions stored in FP32
PRECOND = {"none": PC_NONE, "jacobi": PC_JACOBI, "amg32": PC_AMG32, "amg64": PC_AMG64}


class jfnk_patch(C.Structure):
    _fields_ = [("type", C.c_int32), ("start", C.c_int64), ("size", C.c_int64),
                ("value", C.c_double * 3), ("per_face", C.c_void_p)]


class jfnk_mesh_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_points", C.c_int64), ("points", C.c_void_p),
                ("n_cells", C.c_int64), ("n_faces", C.c_int64), ("n_internal", C.c_int64),
                ("face_ptr", C.c_void_p), ("face_pts", C.c_void_p), ("owner", C.c_void_p),
                ("neighbour", C.c_void_p), ("n_patches", C.c_int32), ("patches", C.c_void_p)]


class jfnk_material(C.Structure):
    _fields_ = [("law", C.c_int32), ("E", C.c_double), ("nu", C.c_double),
                ("alpha_rc", C.c_double), ("alpha_pc", C.c_double), ("rho", C.c_double)]


class jfnk_mesh_info(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("dim", C.c_int32), ("n_dof", C.c_int64),
                ("n_internal_faces", C.c_int64), ("n_boundary_faces", C.c_int64),
                ("bandwidth", C.c_int64), ("device_bytes", C.c_int64), ("setup_ms", C.c_double),
                ("n_slots", C.c_int64), ("n_segments", C.c_int32), ("n_dof_external", C.c_int64),
                ("tiled", C.c_int32), ("tile_halo_max", C.c_int32), ("tile_halo_total", C.c_int64),
                ("tile_incoming_total", C.c_int64), ("tile_ring2_max", C.c_int32),
                ("tile_ring2_total", C.c_int64), ("tile_faces_max", C.c_int32), ("tile_entries_max", C.c_int32),
                ("fused", C.c_int32)]


class jfnk_gmres_opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_it", C.c_int32), ("rtol", C.c_double),
                ("atol", C.c_double), ("precond", C.c_int32), ("cheb_degree", C.c_int32),
                ("eps", C.c_double), ("step_chunk", C.c_int32), ("graphs", C.c_int32),
                ("left", C.c_int32), ("augment", C.c_int32), ("fd_central", C.c_int32), ("orth", C.c_int32)]


class jfnk_newton_opts(C.Structure):
    _fields_ = [("n_increments", C.c_int32), ("max_newton_it", C.c_int32), ("rtol", C.c_double),
                ("atol", C.c_double), ("eta", C.c_double), ("gmres", jfnk_gmres_opts),
                ("dtol", C.c_double), ("line_search", C.c_int32), ("max_backtrack", C.c_int32),
                ("inc_begin", C.c_int32), ("inc_end", C.c_int32), ("stol", C.c_double),
                ("central_below", C.c_double)]


class jfnk_segregated_opts(C.Structure):
    _fields_ = [("n_increments", C.c_int32), ("max_outer_it", C.c_int32), ("rtol", C.c_double),
                ("atol", C.c_double), ("inner_rtol", C.c_double), ("max_inner_it", C.c_int32),
                ("precond", C.c_int32), ("cheb_degree", C.c_int32)]


class jfnk_stats(C.Structure):
    _fields_ = [("newton_it", C.c_int32), ("gmres_it", C.c_int32), ("restarts", C.c_int32),
                ("jv_evals", C.c_int32), ("res0", C.c_double), ("res_final", C.c_double),
                ("eps_last", C.c_double), ("t_ms", C.c_double * 8)]

    def as_dict(self):
        return dict(newton_it=self.newton_it, gmres_it=self.gmres_it, restarts=self.restarts,
                    jv_evals=self.jv_evals, res0=self.res0, res_final=self.res_final,
                    eps_last=self.eps_last, t_ms=list(self.t_ms))


class jfnk_tune_report(C.Structure):
    _fields_ = [("lds_kernels", C.c_int32), ("persist", C.c_int32), ("step_chunk", C.c_int32),
                ("graphs", C.c_int32), ("n_jv", C.c_int32), ("jv_lds", C.c_int32 * 16),
                ("jv_persist", C.c_int32 * 16), ("jv_ms", C.c_double * 16), ("n_solve", C.c_int32),
                ("solve_chunk", C.c_int32 * 8), ("solve_graphs", C.c_int32 * 8), ("solve_ms", C.c_double * 8),
                ("orth", C.c_int32), ("orth_ms", C.c_double * 2)]

    def as_dict(self):
        return {"lds_kernels": self.lds_kernels, "persist": self.persist, "step_chunk": self.step_chunk,
                "graphs": self.graphs,
                "jv": [{"lds": self.jv_lds[i], "persist": self.jv_persist[i], "ms": self.jv_ms[i]}
                       for i in range(self.n_jv)],
                "solve": [{"step_chunk": self.solve_chunk[i], "graphs": self.solve_graphs[i],
                           "ms": self.solve_ms[i]} for i in range(self.n_solve)],
                "orth": self.orth, "orth_ms": list(self.orth_ms)}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libjfnk.so is not built (run __graft_entry__.build() or "
                          "python paper_2502_17217_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "jfnk_create_mesh": [vp, vp, vp, C.POINTER(vp)],
        "jfnk_create_batch": [vp, vp, i32, vp, C.POINTER(vp)],
        "jfnk_segment_info": [vp, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)],
        "jfnk_newton_solve_batch": [vp, vp, C.POINTER(jfnk_newton_opts), vp, vp, vp, vp, vp],
        "jfnk_destroy_mesh": [vp],
        "jfnk_inspect_mesh": [vp, vp, C.POINTER(jfnk_mesh_info), vp, vp],
        "jfnk_get_mesh_info": [vp, C.POINTER(jfnk_mesh_info)],
        "jfnk_mesh_order": [vp, vp],
        "jfnk_to_internal": [vp, vp, vp, vp],
        "jfnk_to_external": [vp, vp, vp, vp],
        "jfnk_workspace_size": [vp, i32, i32, i32, C.POINTER(C.c_size_t)],
        "jfnk_residual": [vp, d, vp, vp, vp, vp],
        "jfnk_jv": [vp, d, vp, vp, vp, d, vp, vp, vp, vp],
        "jfnk_gmres": [vp, d, vp, vp, vp, vp, C.POINTER(jfnk_gmres_opts), vp, vp, vp],
        "jfnk_newton_solve": [vp, C.POINTER(jfnk_newton_opts), vp, vp, vp, vp],
        "jfnk_profile_enable": [vp, i32],
        "jfnk_profile_read": [vp, vp, vp, i32],
        "jfnk_autotune": [vp, C.POINTER(jfnk_gmres_opts), vp, d, vp, vp, vp],
        "jfnk_set_cell_passes": [vp, i32, i32],
        "jfnk_jv_noalloc": [vp, d, vp, vp, vp, d, vp, vp],
        "jfnk_set_body_force": [vp, vp, vp],
        "jfnk_set_inertia": [vp, d, vp, vp, vp, vp, vp],
        "jfnk_dynamic_step": [vp, d, i32, C.POINTER(jfnk_newton_opts), vp, vp, vp, vp, vp, vp, vp, vp],
        "jfnk_segregated_solve": [vp, C.POINTER(jfnk_segregated_opts), vp, vp, vp, vp],
        "jfnk_jv_central": [vp, d, vp, vp, d, vp, vp, vp, vp],
        "jfnk_amg_info_get": [vp, i32, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.jfnk_last_error.restype = C.c_char_p
    lib.jfnk_last_error.argtypes = []
    lib.jfnk_version.restype = C.c_char_p
    lib.jfnk_version.argtypes = []
    return lib


_lib = _load()


class JfnkError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.jfnk_last_error().decode(errors="replace")
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES.get(status, status), msg))


def _check(status, where, allow=()):
    if status != OK and status not in allow:
        raise JfnkError(status, where)
    return status


def version():
    return _lib.jfnk_version().decode()


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _dptr(t, n=None, name="tensor", dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor" % (name, dtype))
    if n is not None and t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return C.c_void_p(t.data_ptr())


class Workspace:
    """Device workspace (torch uint8 buffer) with a 256-byte aligned pointer."""

    def __init__(self, nbytes, device="cuda"):
        self.nbytes = int(nbytes)
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        self.ptr = (base + 255) & ~255

    @property
    def c(self):
        return C.c_void_p(self.ptr)


def _make_desc(mesh):
    """Build a jfnk_mesh_desc; returns (desc, keepalive list of host arrays)."""
    keep = []
    dim = int(mesh["dim"])
    pts = np.ascontiguousarray(mesh["points"], dtype=np.float64)
    fptr = np.ascontiguousarray(mesh["face_ptr"], dtype=np.int64)
    fpts = np.ascontiguousarray(mesh["face_pts"], dtype=np.int32)
    own = np.ascontiguousarray(mesh["owner"], dtype=np.int32)
    nb = np.ascontiguousarray(mesh["neighbour"], dtype=np.int32)
    keep += [pts, fptr, fpts, own, nb]
    patches = (jfnk_patch * max(1, len(mesh["patches"])))()
    for i, p in enumerate(mesh["patches"]):
        patches[i].type = BC[p["type"]]
        patches[i].start = p["start"]
        patches[i].size = p["size"]
        for k in range(3):
            patches[i].value[k] = float(p["value"][k])
        if p.get("per_face") is not None:
            pf = np.ascontiguousarray(p["per_face"], dtype=np.float64)
            keep.append(pf)
            patches[i].per_face = pf.ctypes.data
        else:
            patches[i].per_face = None
    keep.append(patches)
    desc = jfnk_mesh_desc(dim, pts.shape[0], pts.ctypes.data, int(mesh["n_cells"]),
                          int(mesh["n_faces"]), int(mesh["n_internal"]), fptr.ctypes.data,
                          fpts.ctypes.data, own.ctypes.data, nb.ctypes.data,
                          len(mesh["patches"]), C.cast(patches, C.c_void_p))
    return desc, keep


def _make_material(material):
    get = (lambda k: getattr(material, k)) if hasattr(material, "law") else (lambda k: material[k])
    try:
        rho = float(get("rho"))
    except (AttributeError, KeyError):
        rho = 0.0
    return jfnk_material(LAW[get("law")], get("E"), get("nu"), get("alpha_rc"), get("alpha_pc"), rho)


def _info_dict(info):
    return {k: getattr(info, k) for k, _ in jfnk_mesh_info._fields_}


def inspect_mesh(mesh, material, geometry=False):
    """Host-only validation and preprocessing (no GPU needed).

    Returns the info dict, plus (xc, vol) in input cell order if geometry=True.
    """
    desc, keep = _make_desc(mesh)
    mat = _make_material(material)
    info = jfnk_mesh_info()
    xc = vol = None
    if geometry:
        xc = np.zeros((int(mesh["n_cells"]), int(mesh["dim"])))
        vol = np.zeros(int(mesh["n_cells"]))
    _check(_lib.jfnk_inspect_mesh(C.byref(desc), C.byref(mat), C.byref(info),
                                  xc.ctypes.data if geometry else None,
                                  vol.ctypes.data if geometry else None), "jfnk_inspect_mesh")
    del keep
    return (_info_dict(info), xc, vol) if geometry else _info_dict(info)


class Mesh:
    """Owner of a jfnk_mesh handle: one mesh, or a batch of meshes (segments).

    Internal vectors (n_dof entries) are component-major in the library's
    cell order; external vectors (n_dof_external entries) are the meshes'
    interleaved input-order vectors, concatenated for a batch.
    """

    def __init__(self, mesh, material, stream=None):
        meshes = mesh if isinstance(mesh, (list, tuple)) else [mesh]
        mats = material if isinstance(material, (list, tuple)) else [material] * len(meshes)
        if len(mats) != len(meshes):
            raise ValueError("one material per mesh")
        descs = (jfnk_mesh_desc * len(meshes))()
        cmats = (jfnk_material * len(meshes))()
        keep = []
        for i, (m, mt) in enumerate(zip(meshes, mats)):
            d, k = _make_desc(m)
            descs[i] = d
            keep.append(k)
            cmats[i] = _make_material(mt)
        h = C.c_void_p()
        _check(_lib.jfnk_create_batch(descs, cmats, len(meshes), _stream(stream), C.byref(h)),
               "jfnk_create_batch")
        del keep
        self.handle = h
        info = jfnk_mesh_info()
        _check(_lib.jfnk_get_mesh_info(h, C.byref(info)), "jfnk_get_mesh_info")
        self.info = _info_dict(info)
        self.dim = info.dim
        self.n_cells = info.n_cells
        self.n_dof = info.n_dof
        self.n_dof_external = info.n_dof_external
        self.n_segments = info.n_segments
        self.segments = []
        for s in range(self.n_segments):
            co, nc, eo = C.c_int64(), C.c_int64(), C.c_int64()
            _check(_lib.jfnk_segment_info(h, s, C.byref(co), C.byref(nc), C.byref(eo)), "jfnk_segment_info")
            self.segments.append(dict(cell_off=co.value, n_cells=nc.value, ext_off=eo.value))
        order = np.empty(info.n_dof_external // info.dim, dtype=np.int32)
        _check(_lib.jfnk_mesh_order(h, order.ctypes.data), "jfnk_mesh_order")
        self.old_of_new = order

    def segment_slice_external(self, s):
        g = self.segments[s]
        return slice(g["ext_off"] * self.dim, (g["ext_off"] + g["n_cells"]) * self.dim)

    def close(self):
        if getattr(self, "handle", None):
            _lib.jfnk_destroy_mesh(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # vectors in internal order <-> input order (device permutation kernels)
    def to_internal(self, x, out=None, stream=None):
        out = torch.empty(self.n_dof, dtype=torch.float64, device=x.device) if out is None else out
        _check(_lib.jfnk_to_internal(self.handle, _dptr(x, self.n_dof_external, "x"),
                                     _dptr(out, self.n_dof, "out"), _stream(stream)), "jfnk_to_internal")
        return out

    def to_external(self, x, out=None, stream=None):
        out = torch.empty(self.n_dof_external, dtype=torch.float64, device=x.device) if out is None else out
        _check(_lib.jfnk_to_external(self.handle, _dptr(x, self.n_dof, "x"),
                                     _dptr(out, self.n_dof_external, "out"), _stream(stream)),
               "jfnk_to_external")
        return out


def create_mesh(mesh, material, stream=None):
    return Mesh(mesh, material, stream)


def create_batch(meshes, materials, stream=None):
    return Mesh(list(meshes), list(materials), stream)


def _pc(precond):
    """A precond value from an int or a name ("amg32", "jacobi+z32", ...)."""
    if not isinstance(precond, str):
        return int(precond)
    base, _, flag = precond.partition("+")
    if flag not in ("", "z32"):
        raise ValueError("unknown preconditioner flag %r" % flag)
    return PRECOND[base] | (PC_Z32 if flag else 0)


def workspace_size(mesh, op=0, restart=30, precond=PC_JACOBI):
    n = C.c_size_t()
    _check(_lib.jfnk_workspace_size(mesh.handle, op, restart, _pc(precond), C.byref(n)), "jfnk_workspace_size")
    return n.value


def make_workspace(mesh, op=0, restart=30, precond=PC_JACOBI):
    return Workspace(workspace_size(mesh, op, restart, precond))


def residual(mesh, load, u, R, work, stream=None):
    _check(_lib.jfnk_residual(mesh.handle, float(load), _dptr(u, mesh.n_dof, "u"), _dptr(R, mesh.n_dof, "R"),
                              work.c, _stream(stream)), "jfnk_residual")
    return R


def jv(mesh, load, u, Ru, v, eps, Jv, work, stream=None, return_eps=False):
    """J v into Jv; with return_eps also the step(s) used (scalar, or one per batch mesh)."""
    e = (C.c_double * mesh.n_segments)()
    _check(_lib.jfnk_jv(mesh.handle, float(load), _dptr(u, mesh.n_dof, "u"),
                        _dptr(Ru, mesh.n_dof, "Ru") if Ru is not None else None,
                        _dptr(v, mesh.n_dof, "v"), float(eps), _dptr(Jv, mesh.n_dof, "Jv"),
                        C.cast(e, C.c_void_p) if return_eps else None, work.c, _stream(stream)), "jfnk_jv")
    if not return_eps:
        return Jv
    return (Jv, e[0]) if mesh.n_segments == 1 else (Jv, list(e))


def jv_central(mesh, load, u, v, eps, Jv, work, stream=None, return_eps=False):
    """Central-difference J v (R(u + eps v) - R(u - eps v)) / (2 eps) into Jv
    (workspace op 3); with return_eps also the step(s) used."""
    e = (C.c_double * mesh.n_segments)()
    _check(_lib.jfnk_jv_central(mesh.handle, float(load), _dptr(u, mesh.n_dof, "u"), _dptr(v, mesh.n_dof, "v"),
                                float(eps), _dptr(Jv, mesh.n_dof, "Jv"),
                                C.cast(e, C.c_void_p) if return_eps else None, work.c, _stream(stream)),
           "jfnk_jv_central")
    if not return_eps:
        return Jv
    return (Jv, e[0]) if mesh.n_segments == 1 else (Jv, list(e))


def jv_noalloc(mesh, load, u, Ru, v, eps, Jv, stream=None):
    """J v like jv(), with the library's fixed device scratch instead of a
    workspace (no device allocation; calls overlapping on one GPU race)."""
    _check(_lib.jfnk_jv_noalloc(mesh.handle, float(load), _dptr(u, mesh.n_dof, "u"),
                                None if Ru is None else _dptr(Ru, mesh.n_dof, "Ru"),
                                _dptr(v, mesh.n_dof, "v"), float(eps), _dptr(Jv, mesh.n_dof, "Jv"),
                                _stream(stream)), "jfnk_jv_noalloc")
    return Jv


def set_body_force(mesh, body, stream=None):
    """Body force per unit volume, [n_cells, dim] in input order (None removes it)."""
    if body is None:
        _check(_lib.jfnk_set_body_force(mesh.handle, None, _stream(stream)), "jfnk_set_body_force")
        return
    b = np.ascontiguousarray(body, dtype=np.float64).reshape(-1)
    if b.size != mesh.n_dof_external:
        raise ValueError("body force has %d values, expected %d" % (b.size, mesh.n_dof_external))
    _check(_lib.jfnk_set_body_force(mesh.handle, b.ctypes.data, _stream(stream)), "jfnk_set_body_force")


def set_inertia(mesh, dt, u_n=None, u_nm1=None, v_n=None, v_nm1=None, stream=None):
    """BDF2 inertia from previous states (internal-layout device tensors); dt <= 0 removes it."""
    if dt <= 0:
        _check(_lib.jfnk_set_inertia(mesh.handle, 0.0, None, None, None, None, _stream(stream)), "jfnk_set_inertia")
        return
    _check(_lib.jfnk_set_inertia(mesh.handle, float(dt), _dptr(u_n, mesh.n_dof, "u_n"),
                                 _dptr(u_nm1, mesh.n_dof, "u_nm1"), _dptr(v_n, mesh.n_dof, "v_n"),
                                 _dptr(v_nm1, mesh.n_dof, "v_nm1"), _stream(stream)), "jfnk_set_inertia")


def dynamic_step(mesh, dt, opts, u, u_prev, v, v_prev, a, work, predictor=True, stream=None,
                 allow=(E_NOT_CONVERGED,)):
    """One BDF2 time step in place on (u, u_prev, v, v_prev, a); returns (status, stats)."""
    st = (jfnk_stats * mesh.n_segments)()
    s = _lib.jfnk_dynamic_step(mesh.handle, float(dt), 1 if predictor else 0, C.byref(opts),
                               _dptr(u, mesh.n_dof, "u"), _dptr(u_prev, mesh.n_dof, "u_prev"),
                               _dptr(v, mesh.n_dof, "v"), _dptr(v_prev, mesh.n_dof, "v_prev"),
                               _dptr(a, mesh.n_dof, "a"), C.cast(st, C.c_void_p), work.c, _stream(stream))
    _check(s, "jfnk_dynamic_step", allow)
    out = [x.as_dict() for x in st]
    return s, (out[0] if mesh.n_segments == 1 else out)


ORTH = {"cgs2": 0, "dcgs2": 1, "auto": 2}


def gmres_opts(restart=30, max_it=1000, rtol=1e-10, atol=0.0, precond=PC_JACOBI, cheb_degree=3, eps=0.0,
               step_chunk=0, graphs=2, left=0, augment=0, fd_central=0, orth=0):
    """orth: 0 or "cgs2" (Gram-Schmidt twice), 1 or "dcgs2" (delayed reorthogonalisation),
    2 or "auto" (the handle's choice, see autotune)."""
    orth = ORTH[orth] if isinstance(orth, str) else int(orth)
    return jfnk_gmres_opts(restart, max_it, rtol, atol, _pc(precond), cheb_degree, eps, step_chunk, graphs,
                           int(left), int(augment), int(fd_central), orth)


def newton_opts(n_increments=1, max_newton_it=20, rtol=1e-6, atol=1e-50, eta=1e-3, dtol=0.0,
                line_search=0, max_backtrack=0, inc_begin=0, inc_end=0, stol=0.0, central_below=0.0, **gm):
    return jfnk_newton_opts(n_increments, max_newton_it, rtol, atol, eta, gmres_opts(**gm), dtol,
                            line_search, max_backtrack, inc_begin, inc_end, stol, central_below)


def gmres(mesh, load, u, Ru, b, x, opts, work, stream=None, allow=(E_NOT_CONVERGED, E_BREAKDOWN)):
    st = (jfnk_stats * mesh.n_segments)()
    s = _lib.jfnk_gmres(mesh.handle, float(load), _dptr(u, mesh.n_dof, "u"), _dptr(Ru, mesh.n_dof, "Ru"),
                        _dptr(b, mesh.n_dof, "b"), _dptr(x, mesh.n_dof, "x"), C.byref(opts),
                        C.cast(st, C.c_void_p), work.c, _stream(stream))
    _check(s, "jfnk_gmres", allow)
    out = [x.as_dict() for x in st]
    return s, (out[0] if mesh.n_segments == 1 else out)


def newton_solve(mesh, opts, u, work, stream=None, allow=(E_NOT_CONVERGED,)):
    st = (jfnk_stats * mesh.n_segments)()
    s = _lib.jfnk_newton_solve(mesh.handle, C.byref(opts), _dptr(u, mesh.n_dof, "u"), C.cast(st, C.c_void_p),
                               work.c, _stream(stream))
    _check(s, "jfnk_newton_solve", allow)
    out = [x.as_dict() for x in st]
    return s, (out[0] if mesh.n_segments == 1 else out)


def segregated_opts(n_increments=1, max_outer_it=100000, rtol=1e-6, atol=1e-50, inner_rtol=0.9,
                    max_inner_it=200, precond="amg32", cheb_degree=3):
    pc = _pc(precond)
    return jfnk_segregated_opts(n_increments, max_outer_it, rtol, atol, inner_rtol, max_inner_it, pc, cheb_degree)


def segregated_solve(mesh, opts, u, work, stream=None, allow=(E_NOT_CONVERGED,)):
    """The segregated quasi-Newton iteration with J_tilde (single mesh);
    returns (status, stats: newton_it = outer iterations, gmres_it = CG
    iterations)."""
    st = jfnk_stats()
    s = _lib.jfnk_segregated_solve(mesh.handle, C.byref(opts), _dptr(u, mesh.n_dof, "u"), C.byref(st),
                                   work.c, _stream(stream))
    _check(s, "jfnk_segregated_solve", allow)
    return s, st.as_dict()


def newton_solve_batch(mesh, opts, u, work, n_increments=None, stream=None, allow=(E_NOT_CONVERGED,)):
    """Batched Newton; returns (status, per-mesh stats list, per-mesh status list)."""
    S = mesh.n_segments
    st = (jfnk_stats * S)()
    seg = (C.c_int * S)()
    inc = None
    if n_increments is not None:
        inc = (C.c_int32 * S)(*[int(k) for k in n_increments])
    s = _lib.jfnk_newton_solve_batch(mesh.handle, C.cast(inc, C.c_void_p) if inc is not None else None,
                                     C.byref(opts), _dptr(u, mesh.n_dof, "u"), C.cast(st, C.c_void_p),
                                     C.cast(seg, C.c_void_p), work.c, _stream(stream))
    _check(s, "jfnk_newton_solve_batch", allow)
    return s, [x.as_dict() for x in st], list(seg)


def autotune(mesh, opts, u, work, load=1.0, stream=None):
    """Time the equivalent launch shapes and Arnoldi schedules on this handle
    and keep the fastest (see include/jfnk.h); returns the report."""
    rep = jfnk_tune_report()
    _check(_lib.jfnk_autotune(mesh.handle, C.byref(opts), _dptr(u, mesh.n_dof, "u"), float(load), work.c,
                              _stream(stream), C.byref(rep)), "jfnk_autotune")
    return rep.as_dict()


class jfnk_amg_info(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("coarse_dense", C.c_int32), ("rows", C.c_int64 * 16),
                ("nnz", C.c_int64 * 16), ("lanes", C.c_int32 * 16), ("operator_complexity", C.c_double),
                ("setup_ms", C.c_double), ("device_bytes", C.c_int64)]


def amg_info(mesh, precond=PC_AMG32):
    """Shape of the handle's AMG hierarchy (built by a solve or autotune)."""
    i = jfnk_amg_info()
    _check(_lib.jfnk_amg_info_get(mesh.handle, _pc(precond), C.cast(C.pointer(i), C.c_void_p)), "jfnk_amg_info_get")
    n = i.n_levels
    return {"levels": n, "rows": list(i.rows[:n]), "nnz": list(i.nnz[:n]), "lanes": list(i.lanes[:n]),
            "coarse": "dense" if i.coarse_dense else "diagonal", "operator_complexity": i.operator_complexity,
            "setup_ms": i.setup_ms, "device_bytes": i.device_bytes}


def set_cell_passes(mesh, passes, persist=0):
    """Pin the cell passes of R and J v: 0 gathers, 1 LDS-staged gradient and
    flux passes, 2 one fused pass per tile; persist = persistent grid size."""
    _check(_lib.jfnk_set_cell_passes(mesh.handle, int(passes), int(persist)), "jfnk_set_cell_passes")


def profile_enable(mesh, on=True):
    _check(_lib.jfnk_profile_enable(mesh.handle, 1 if on else 0), "jfnk_profile_enable")


def profile_read(mesh, reset=True):
    """Accumulated kernel milliseconds and call counts: eps, gradient, flux,
    preconditioner, orthogonalisation, other solver vector work."""
    ms = (C.c_double * 6)()
    calls = (C.c_int64 * 6)()
    _check(_lib.jfnk_profile_read(mesh.handle, ms, calls, 1 if reset else 0), "jfnk_profile_read")
    names = ["eps", "gradient", "flux", "precond", "orth", "other"]
    return {n: (ms[i], calls[i]) for i, n in enumerate(names)}


# ---------------------------------------------------------------- serving
class jfnk_server_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_slots", C.c_int32), ("max_queue", C.c_int32),
                ("dry_run_us_per_kcell", C.c_double)]


class jfnk_request_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("state", C.c_int32), ("t_submit_ms", C.c_double),
                ("t_start_ms", C.c_double), ("t_done_ms", C.c_double), ("latency_ms", C.c_double),
                ("footprint_bytes", C.c_int64), ("n_cells", C.c_int64), ("stats", jfnk_stats),
                ("error", C.c_char * 160)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("stats", "error")}
        d["stats"] = self.stats.as_dict()
        d["error"] = self.error.decode(errors="replace")
        return d


class jfnk_server_metrics(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("running", C.c_int64), ("queued", C.c_int64), ("hbm_in_use", C.c_int64),
                ("hbm_peak", C.c_int64), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("mean_ms", C.c_double), ("max_ms", C.c_double), ("solves_per_s", C.c_double),
                ("cancelled", C.c_int64)]


def _server_sigs():
    vp, i32 = C.c_void_p, C.c_int32
    sig = {
        "jfnk_server_create": [C.POINTER(jfnk_server_opts), C.POINTER(vp)],
        "jfnk_server_submit": [vp, vp, vp, C.POINTER(jfnk_newton_opts), vp, C.POINTER(C.c_uint64)],
        "jfnk_server_poll": [vp, C.c_uint64, C.POINTER(jfnk_request_info)],
        "jfnk_server_wait": [vp, C.c_uint64, C.POINTER(jfnk_request_info)],
        "jfnk_server_metrics_get": [vp, C.POINTER(jfnk_server_metrics)],
        "jfnk_server_destroy": [vp],
        "jfnk_server_cancel_queued": [vp, C.POINTER(C.c_int64)],
    }
    for name, args in sig.items():
        f = getattr(_lib, name)
        f.argtypes = args
        f.restype = C.c_int


_server_sigs()


class Server:
    """Request loop of the library: continuous admission onto concurrent
    streams under an HBM budget (see include/jfnk.h)."""

    def __init__(self, hbm_budget, max_slots=4, max_queue=1 << 20, dry_run_us_per_kcell=0.0):
        o = jfnk_server_opts(int(hbm_budget), int(max_slots), int(max_queue), float(dry_run_us_per_kcell))
        h = C.c_void_p()
        _check(_lib.jfnk_server_create(C.byref(o), C.byref(h)), "jfnk_server_create")
        self.handle = h
        self._out = {}

    def submit(self, mesh, material, opts, keep_solution=True):
        desc, keep = _make_desc(mesh)
        mat = _make_material(material)
        out = np.zeros(int(mesh["n_cells"]) * int(mesh["dim"])) if keep_solution else None
        t = C.c_uint64()
        _check(_lib.jfnk_server_submit(self.handle, C.byref(desc), C.byref(mat), C.byref(opts),
                                       out.ctypes.data if out is not None else None, C.byref(t)),
               "jfnk_server_submit")
        del keep
        self._out[t.value] = out
        return t.value

    def poll(self, ticket):
        info = jfnk_request_info()
        _check(_lib.jfnk_server_poll(self.handle, ticket, C.byref(info)), "jfnk_server_poll")
        return info.as_dict()

    def wait(self, ticket):
        info = jfnk_request_info()
        _check(_lib.jfnk_server_wait(self.handle, ticket, C.byref(info)), "jfnk_server_wait")
        return info.as_dict(), self._out.get(ticket)

    def cancel_queued(self):
        """Drop every request no worker has started; returns how many."""
        n = C.c_int64()
        _check(_lib.jfnk_server_cancel_queued(self.handle, C.byref(n)), "jfnk_server_cancel_queued")
        return n.value

    def submit_nowait(self, mesh, material, opts, keep_solution=False):
        """submit() that returns None instead of raising when the queue is full."""
        try:
            return self.submit(mesh, material, opts, keep_solution)
        except JfnkError as e:
            if e.status == E_BUSY:
                return None
            raise

    def metrics(self):
        m = jfnk_server_metrics()
        _check(_lib.jfnk_server_metrics_get(self.handle, C.byref(m)), "jfnk_server_metrics_get")
        return {k: getattr(m, k) for k, _ in m._fields_}

    def close(self):
        if getattr(self, "handle", None):
            _check(_lib.jfnk_server_destroy(self.handle), "jfnk_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
