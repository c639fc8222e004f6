/*
 * jfnk.h -- C ABI of the MI355X (gfx950) Jacobian-free Newton-Krylov library
 * for cell-centred finite-volume solid mechanics.
 *
 * The operations follow Cardiff, Armfield, Tukovic & Batistic, "A
 * Jacobian-free Newton-Krylov method for cell-centred finite volume solid
 * mechanics" (arXiv 2502.17217):
 *   - mesh, cells, faces and boundary classes: Section 2.3 (cell-centred
 *     finite volume discretisation), boundary types of Section 2.1;
 *   - residual R(u) = 0: Section 2.2, Eq. (residual); total Lagrangian form
 *     Appendix A, Eq. (momentum_TL); laws Appendix B;
 *   - J v ~ (R(u + eps v) - R(u)) / eps: Section 3.2, Eq. (JF);
 *   - right-preconditioned GMRES with the compact-stencil approximate
 *     Jacobian as preconditioner: Section 3.2; the approximate Jacobian
 *     itself: Section 3.1 (coefficients after Eq. SegSys);
 *   - Newton-Raphson, Eq. (NewtonRaphson), with the convergence checks of
 *     Section 3.3 and equal load increments.
 *
 * Conventions
 *   Vectors: device pointers to n_cells * dim FP64 values in the INTERNAL
 *   layout: the mesh's bandwidth-reducing (reverse Cuthill-McKee) cell order,
 *   component-major ([component][cell], one contiguous array per displacement
 *   component, so that consecutive GPU lanes touch consecutive addresses).
 *   The EXTERNAL layout is the paper's blocked vector of Section 2.2:
 *   interleaved [cell][component] in input cell order.  jfnk_to_internal()
 *   and jfnk_to_external() convert on the device; jfnk_mesh_order() returns
 *   the cell map.
 *   Ownership: the caller owns every vector and the workspace (e.g. torch
 *   tensors).  The library owns only the mesh handle (its packed device
 *   geometry and a few pinned host scalars), freed by jfnk_destroy_mesh().
 *   It never frees caller memory.
 *   Streams: `stream` is a hipStream_t (NULL = default stream).  jfnk_residual,
 *   jfnk_jv and the permutations only enqueue work; solvers synchronise the
 *   stream to read convergence scalars and return when finished.
 *   Errors: every call returns a jfnk_status; no C++ exception crosses the
 *   ABI.  jfnk_last_error() gives a thread-local message for the last
 *   failing call on this thread.  A call that fails with JFNK_E_ARG or
 *   JFNK_E_MESH enqueues no device work.
 *   Sign convention: R is the out-of-balance force of Eq. (residual); its
 *   Jacobian is negative (semi-)definite for small strains, like J_tilde.
 */
#ifndef JFNK_H
#define JFNK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  JFNK_OK = 0,
  JFNK_E_ARG = -1,            /* invalid argument (null pointer, bad size, bad option) */
  JFNK_E_MESH = -2,           /* invalid mesh: index out of range, open cell, d.n <= 0, singular G_P */
  JFNK_E_OOM = -3,            /* device or pinned host allocation failed */
  JFNK_E_HIP = -4,            /* HIP runtime error */
  JFNK_E_NOT_CONVERGED = -5,  /* iteration limit reached; outputs hold the last iterate */
  JFNK_E_DIVERGED = -6,       /* residual grew beyond the divergence limit */
  JFNK_E_NAN = -7,            /* NaN/Inf in a residual or Krylov quantity */
  JFNK_E_BREAKDOWN = -8,      /* Krylov stagnation: no progress over a restart cycle */
  JFNK_E_BUSY = -9            /* server: no capacity for the request right now */
} jfnk_status;

/* Boundary classes of Section 2.3: prescribed displacement, prescribed
 * traction, symmetry plane; a pressure patch is a traction -p n on the
 * undeformed face (dead load).  A symmetry face (Eq. symm and the symmetry
 * sums of Eq. leastSquaresGrad and Eq. RhieChow) sees the mirror image of
 * its cell across the face's plane: the face gradient is the average of
 * the cell's gradient and its mirror image, the face stress the law at that
 * gradient (normal traction only), and the Rhie-Chow term acts on the
 * normal displacement; its value and per_face entries are ignored.  Its
 * block of the approximate Jacobian is not scalar times identity; the
 * preconditioners keep the diagonal of that block per component. */
typedef enum {
  JFNK_BC_DISPLACEMENT = 1,
  JFNK_BC_TRACTION = 2,
  JFNK_BC_PRESSURE = 3,
  JFNK_BC_SYMMETRY = 4
} jfnk_bc_type;

/* One boundary patch: faces [start, start + size) of the face list.
 * value: displacement vector, traction vector, or value[0] = pressure.
 * per_face: NULL, or host array [size][dim] overriding value face by face.
 * Every prescribed value is multiplied by the current load factor. */
typedef struct {
  int32_t type;
  int64_t start;
  int64_t size;
  double value[3];
  const double* per_face;
} jfnk_patch;

/* Polyhedral mesh, OpenFOAM conventions (Section 2.3, Figure of cell P):
 * internal faces first; face f has vertices face_pts[face_ptr[f] ..
 * face_ptr[f+1]) ordered so that the right-hand normal points out of
 * owner[f]; 2-D (plane strain, unit depth) faces are edges p0 -> p1 whose
 * outward side is on the right.  All arrays are host memory and are only
 * read during jfnk_create_mesh. */
typedef struct {
  int32_t dim;                 /* 2 or 3 */
  int64_t n_points;
  const double* points;        /* [n_points][dim] */
  int64_t n_cells;
  int64_t n_faces;
  int64_t n_internal;
  const int64_t* face_ptr;     /* [n_faces + 1] */
  const int32_t* face_pts;     /* [face_ptr[n_faces]] */
  const int32_t* owner;        /* [n_faces] */
  const int32_t* neighbour;    /* [n_internal] */
  int32_t n_patches;
  const jfnk_patch* patches;   /* must cover faces [n_internal, n_faces) exactly */
} jfnk_mesh_desc;

/* Appendix B: Hooke's law (linear geometry), and the total Lagrangian
 * hyperelastic laws neo-Hookean and St. Venant-Kirchhoff. */
typedef enum { JFNK_LINEAR_ELASTIC = 0, JFNK_NEO_HOOKEAN = 1, JFNK_ST_VENANT_KIRCHHOFF = 2 } jfnk_law;

/* Appendix B laws.  alpha_rc scales the Rhie-Chow term of the residual
 * (Eq. RhieChow); alpha_pc scales the approximate Jacobian used for
 * preconditioning (unity in the paper, Section 3.1); rho is the density,
 * used only by the inertia term of transient solves (jfnk_dynamic_step). */
typedef struct {
  int32_t law;
  double E;
  double nu;
  double alpha_rc;
  double alpha_pc;
  double rho;
} jfnk_material;

typedef struct jfnk_mesh jfnk_mesh;

typedef struct {
  int64_t n_cells;             /* internal cells (a batch adds alignment padding between meshes) */
  int32_t dim;
  int64_t n_dof;               /* length of an internal vector: n_cells * dim */
  int64_t n_internal_faces;
  int64_t n_boundary_faces;
  int64_t bandwidth;           /* max |P - N| over internal faces after renumbering */
  int64_t device_bytes;        /* device memory owned by the handle */
  double setup_ms;             /* host time spent in jfnk_create_mesh */
  int64_t n_slots;             /* cell-face slots in the packed slot map (incl. padding) */
  int32_t n_segments;          /* meshes in the handle (1, or the batch size) */
  int64_t n_dof_external;      /* length of an external vector (sum over meshes of n_cells * dim) */
  int32_t tiled;               /* 1: cells ordered in compact tiles of 256 and the LDS-staged kernels run */
  int32_t tile_halo_max;       /* largest number of outside neighbours of one tile (0 if not tiled) */
  int64_t tile_halo_total;     /* sum over tiles of their outside neighbours (0 if not tiled) */
  int64_t tile_incoming_total; /* sum over tiles of the faces they take from an earlier tile */
  int32_t tile_ring2_max;      /* largest second ring of a tile: outside cells adjacent to its halo */
  int64_t tile_ring2_total;    /* sum over tiles of their second rings */
  int32_t tile_faces_max;      /* largest number of internal faces touching one tile */
  int32_t tile_entries_max;    /* largest number of faces (internal and boundary) touching one tile */
  int32_t fused;               /* 1: the single-pass J.v kernel fits (tile, two rings and faces in LDS) */
} jfnk_mesh_info;

/* Build the mesh handle: validates the mesh, renumbers cells, computes the
 * geometry of Section 2.3 in FP64 on the host (face area vectors and
 * centroids by fan triangulation, cell volumes and centroids by pyramids,
 * interpolation weights of Eq. stressInterp) and uploads packed arrays.
 * Errors: JFNK_E_ARG (null/inconsistent sizes), JFNK_E_MESH (see above, the
 * message names the offending cell or face), JFNK_E_OOM, JFNK_E_HIP. */
jfnk_status jfnk_create_mesh(const jfnk_mesh_desc* desc, const jfnk_material* mat,
                             void* stream, jfnk_mesh** out);
jfnk_status jfnk_destroy_mesh(jfnk_mesh* mesh);

/* Host-only dry run of jfnk_create_mesh: the same validation and
 * preprocessing, no device work.  Fills *info (device_bytes is what the
 * handle would allocate); if non-NULL, xc_out [n_cells][dim] and vol_out
 * [n_cells] receive the cell centroids and volumes in INPUT cell order.
 * Used for admission control (memory footprint) and host-side checks. */
jfnk_status jfnk_inspect_mesh(const jfnk_mesh_desc* desc, const jfnk_material* mat,
                              jfnk_mesh_info* info, double* xc_out, double* vol_out);
jfnk_status jfnk_get_mesh_info(const jfnk_mesh* mesh, jfnk_mesh_info* info);

/* old_of_new[i] = input cell index of internal cell i (host array [n_cells]). */
jfnk_status jfnk_mesh_order(const jfnk_mesh* mesh, int32_t* old_of_new);
/* External (interleaved [cell][dim], input order) -> internal ([dim][cell],
 * internal order), and the inverse.  Out-of-place; asynchronous. */
jfnk_status jfnk_to_internal(const jfnk_mesh* mesh, const double* d_in, double* d_out, void* stream);
jfnk_status jfnk_to_external(const jfnk_mesh* mesh, const double* d_in, double* d_out, void* stream);

/* Workspace bytes for jfnk_residual / jfnk_jv (op = 0), for jfnk_gmres,
 * jfnk_newton_solve and jfnk_segregated_solve with the given restart length
 * and preconditioner (op = 1), for jfnk_dynamic_step (op = 2), or for
 * jfnk_jv_central (op = 3).  precond may carry JFNK_PC_Z32 (ops 1 and 2),
 * and the solve given this workspace must then carry it too (and the
 * other way round).  The caller allocates at least that many bytes
 * of device memory, 256-byte aligned, and passes it as d_work. */
jfnk_status jfnk_workspace_size(const jfnk_mesh* mesh, int32_t op, int32_t restart,
                                int32_t precond, size_t* bytes);

/* R(u) of Eq. (residual) (static, no body force) at load factor `load`.
 * d_u, d_R: internal layout; d_R may not alias d_u.  Asynchronous. */
jfnk_status jfnk_residual(jfnk_mesh* mesh, double load, const double* d_u, double* d_R,
                          void* d_work, void* stream);

/* J v ~ (R(u + eps v) - R(u)) / eps (Eq. JF) using the cached d_Ru = R(u)
 * (if d_Ru is NULL it is computed first, into the workspace).
 * eps > 0 is used as given; eps <= 0 selects
 *   eps = sqrt(eps_mach) * sqrt(1 + ||u||_2) / ||v||_2
 * computed on the device (a zero v gives J v = 0).
 * If eps_used is non-NULL (host pointer) the call synchronises the stream
 * and stores the eps used; otherwise it is fully asynchronous. */
jfnk_status jfnk_jv(jfnk_mesh* mesh, double load, const double* d_u, const double* d_Ru,
                    const double* d_v, double eps, double* d_Jv, double* eps_used,
                    void* d_work, void* stream);

/* J v exactly as jfnk_jv computes it (same kernels, same bits), for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  It takes no workspace
 * and allocates nothing: its scratch (step-size partial sums, per-segment
 * eps, arrival counters, and the per-cell gradient record when the mesh's
 * cell passes are not the fused single pass; R(u) too when d_Ru is NULL)
 * lives in a fixed 32 MiB device array of the library, one per GPU, held
 * until the process ends.  Arguments as for jfnk_jv (no eps_used: the step
 * stays on the device).  Errors: JFNK_E_ARG when the mesh needs more
 * scratch than 32 MiB (the message gives the size; about 96 bytes per cell
 * for a 3-D mesh on the two-pass kernels), when profiling is enabled on
 * the mesh, or on the argument errors of jfnk_jv.  Every call on a GPU
 * uses that GPU's one array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.  Asynchronous
 * on `stream`. */
/* Central-difference J v (Section 3.2, Eq. JF with the symmetric
 * difference): Jv = (R(u + eps v) - R(u - eps v)) / (2 eps), second order in
 * eps.  eps <= 0 selects eps_mach^(1/3) sqrt(1 + |u|_2) / |v|_2 per mesh
 * segment (0 when v = 0, then Jv = 0); eps > 0 is used as given.  Costs two
 * residual passes and needs no R(u).  d_work: jfnk_workspace_size op 3.
 * eps_used (host, may be NULL): the step per segment.  Errors as jfnk_jv. */
jfnk_status jfnk_jv_central(jfnk_mesh* mesh, double load, const double* d_u, const double* d_v, double eps,
                            double* d_Jv, double* eps_used, void* d_work, void* stream);

jfnk_status jfnk_jv_noalloc(jfnk_mesh* mesh, double load, const double* d_u, const double* d_Ru,
                            const double* d_v, double eps, double* d_Jv, void* stream);

typedef enum { JFNK_PC_NONE = 0, JFNK_PC_JACOBI = 1, JFNK_PC_AMG32 = 2, JFNK_PC_AMG64 = 3 } jfnk_precond;

/* Flag ORed into a preconditioner value (the GMRES options' precond, and
 * the precond of jfnk_workspace_size, which must then carry it too): the
 * directions z_j = P^{-1} v_j of the flexible GMRES (Section 3.2) are
 * stored in FP32, halving that region of the workspace (restart * n_dof
 * floats plus one FP64 vector instead of restart * n_dof doubles).  Each
 * direction is rounded to FP32 when formed and its J v takes the rounded
 * value, so the Arnoldi relation holds for the stored basis.  With AMG32 the
 * V-cycle's output is already an FP32 value and the solve gives the same
 * bits as with the FP64 basis; with JACOBI, AMG64 or NONE the rounding
 * perturbs the preconditioner by one FP32 rounding (the solve stays
 * flexible GMRES and converges to the same tolerance).  Right
 * preconditioning without augmentation only (JFNK_E_ARG otherwise); not
 * for jfnk_segregated_solve. */
#define JFNK_PC_Z32 16

/* GMRES options (Section 3.2; restarted, right preconditioned, classical
 * Gram-Schmidt applied twice).  The run stops when the true residual
 * |b - J x| <= max(rtol |b|, atol), after max_it Arnoldi steps, or on
 * stagnation.  precond: J_tilde (alpha_pc) as diagonal (Jacobi, FP64) or
 * as an aggregation-AMG V-cycle with Chebyshev smoothing (flexible GMRES),
 * stored and applied in FP32 (AMG32) or FP64 (AMG64: the same hierarchy
 * and cycle in full precision, the reference for the mixed-precision
 * path).  eps <= 0 selects the automatic J v step.
 * The Givens rotations and the small least-squares problem are updated on
 * the device, so Arnoldi steps are enqueued in runs of step_chunk steps
 * between host checks of the convergence flags (0: the handle's value,
 * chosen by jfnk_autotune, default 1); graphs = 1 replays each run from a
 * HIP graph captured on first use, 0 launches directly, 2 takes the
 * handle's choice (default: graphs); results are identical either way.
 * left = 1: left preconditioning (the paper's choice in Section 3.2): the
 * Arnoldi vectors are P^{-1} J v, the solution update uses the basis V, and
 * convergence is judged on the preconditioned residual |P^{-1}(b - J x)|
 * against rtol |P^{-1} b|.  augment = k > 0 (right preconditioning only):
 * LGMRES, the augmented restarted GMRES the paper runs (LGMRES(30)+2): the
 * last k of the restart directions of a cycle are the normalised
 * corrections x_c - x_{c-1} of the previous k cycles instead of
 * preconditioned basis vectors (graph replay is not used then).
 * precond | JFNK_PC_Z32 stores the directions z_j in FP32 (see the flag).
 * fd_central = 1: every product J v is the central difference
 * (R(u + eps v) - R(u - eps v)) / (2 eps), second order in eps where the
 * forward difference of Eq. JF is first order, at the cost of one more
 * residual pass; the automatic step is then
 * eps_mach^(1/3) sqrt(1 + |u|) / |v| (the step that balances its truncation
 * and rounding errors), an explicit eps is used as given.
 * orth: the Arnoldi orthogonalisation.  0: classical Gram-Schmidt applied
 * twice (three passes over the basis per step, four reads of it).
 * 1: classical Gram-Schmidt with delayed reorthogonalisation (DCGS2): each
 * step reads the basis twice, once for the dots of the new vector J z_j and
 * of the previous step's vector against the basis, once to reorthogonalise
 * that previous vector and orthogonalise the new one; the Hessenberg column
 * of step j is completed, and its Givens rotation taken, in step j + 1, so
 * the solve notices convergence one J v later.  Same Krylov space and
 * arithmetic precision; the iterates differ from orth = 0 by rounding.
 * Right preconditioning only, restart <= 250 (JFNK_E_ARG otherwise).
 * 2: the handle's choice (jfnk_autotune times both; DCGS2 until tuned),
 * CGS2 wherever DCGS2 does not apply. */
typedef struct {
  int32_t restart;
  int32_t max_it;
  double rtol;
  double atol;
  int32_t precond;
  int32_t cheb_degree;
  double eps;
  int32_t step_chunk;
  int32_t graphs;
  int32_t left;
  int32_t augment;
  int32_t fd_central;
  int32_t orth;
} jfnk_gmres_opts;

/* Newton options (Eq. NewtonRaphson, Section 3.3): per load increment
 * k = 1..n_increments the loads are scaled by k/n_increments; iterate until
 * |R(u)| <= max(rtol |R(u_0)|, atol), or, with stol > 0, until a Newton
 * correction satisfies |s du| <= stol |u| (the step test of Section 3.3;
 * stol = 0 as in the paper switches it off); each linear solve uses
 * relative tolerance eta.  A residual above dtol |R(u_0)| stops the increment with
 * JFNK_E_DIVERGED (dtol <= 0: 1e8).
 * line_search (the globalisation of Section 3.2, which asks only for a step
 * s > 0 that decreases |R|): 0 takes the full step s = 1; 1 tries
 * s = 1, 1/2, 1/4, ... and accepts the first with |R(u + s du)| < |R(u)|
 * (a NaN residual counts as no decrease); after max_backtrack halvings
 * (<= 0: 8) the last trial is accepted.
 * inc_begin, inc_end (1-based, inclusive; <= 0: the first and the last):
 * solve only increments inc_begin .. inc_end of the n_increments, starting
 * from the given d_u (e.g. the converged state of increment inc_begin - 1),
 * so that a caller can inspect every increment.
 * central_below > 0: the linear solves of the Newton iterations that start
 * with |R(u)| <= central_below |R(u_0)| use the central difference for J v
 * (gmres.fd_central), whose smaller error lets the last iterations of a
 * stiff problem reach a tight rtol that the forward difference stalls
 * above. */
typedef struct {
  int32_t n_increments;
  int32_t max_newton_it;
  double rtol;
  double atol;
  double eta;
  jfnk_gmres_opts gmres;
  double dtol;
  int32_t line_search;
  int32_t max_backtrack;
  int32_t inc_begin;
  int32_t inc_end;
  double stol;
  double central_below;
} jfnk_newton_opts;

/* Segregated solution procedure (Section 3.1, Eq. SegSys and the
 * component systems Eq. SegSysX-Z), the classic algorithm the paper
 * compares against: per load increment, u_{k+1} = u_k + du with
 * J_tilde du = -R(u_k), each displacement component's system solved by
 * preconditioned conjugate gradients on -J_tilde until its residual has
 * fallen by the factor inner_rtol (Section 3.2 uses 0.9); converged when
 * |R(u)| <= max(rtol |R(u_0)|, atol) (no step test, as in Section 3.3).
 * precond: JFNK_PC_JACOBI, JFNK_PC_AMG32 or JFNK_PC_AMG64 (one V-cycle per
 * CG iteration; the paper used incomplete Cholesky), cheb_degree as in
 * jfnk_gmres_opts. */
typedef struct {
  int32_t n_increments;
  int32_t max_outer_it;        /* per increment */
  double rtol;
  double atol;
  double inner_rtol;           /* in (0, 1) */
  int32_t max_inner_it;        /* CG iterations per outer iteration */
  int32_t precond;
  int32_t cheb_degree;
} jfnk_segregated_opts;

typedef struct {
  int32_t newton_it;           /* total Newton iterations */
  int32_t gmres_it;            /* total Arnoldi steps */
  int32_t restarts;            /* GMRES restart cycles */
  int32_t jv_evals;
  double res0;                 /* |R| at the start of the last increment (Newton) or |b| (GMRES) */
  double res_final;            /* final |R| (Newton) or true |b - J x| (GMRES) */
  double eps_last;             /* last J v step used */
  double t_ms[8];              /* host wall times: 0 total, 2 Arnoldi steps (J.v, preconditioner and
                                  orthogonalisation, enqueued asynchronously), 4 Newton residuals,
                                  5 preconditioner setup, 6 true residuals and cycle ends; 1, 3, 7
                                  unused (per-kernel times: jfnk_profile_read) */
} jfnk_stats;

/* Solve J(u) x = b with J v from Eq. (JF) at state d_u (load factor `load`,
 * cached d_Ru = R(u), required).  d_x holds the initial guess on entry and
 * the solution on return.  Returns JFNK_OK, JFNK_E_NOT_CONVERGED,
 * JFNK_E_BREAKDOWN or JFNK_E_NAN (d_x then holds the last iterate). */
jfnk_status jfnk_gmres(jfnk_mesh* mesh, double load, const double* d_u, const double* d_Ru,
                       const double* d_b, double* d_x, const jfnk_gmres_opts* opts,
                       jfnk_stats* stats, void* d_work, void* stream);

/* Newton-Raphson with load increments; d_u holds the initial guess on entry
 * and the final iterate on return. */
jfnk_status jfnk_newton_solve(jfnk_mesh* mesh, const jfnk_newton_opts* opts, double* d_u,
                              jfnk_stats* stats, void* d_work, void* stream);

/* ---- Volume terms and transient solves (Section 2.3.1) ----
 * Body force: h_body is a host array [n_cells][dim] in input cell order
 * (for a batch, the meshes' arrays concatenated), a force per unit volume,
 * integrated over each cell by the midpoint rule and scaled by the load
 * factor like every other load: R_P += load f_b,P Omega_P.  NULL removes
 * it.  Copied to the device; jfnk_residual, jfnk_jv, jfnk_gmres and the
 * solvers include it from then on.  Errors: JFNK_E_ARG (non-finite value),
 * JFNK_E_OOM. */
jfnk_status jfnk_set_body_force(jfnk_mesh* mesh, const double* h_body, void* stream);

/* Inertia: with dt > 0 the residual gets -rho Omega_P a_P, a_P the BDF2
 * acceleration of Eq. (inertia2) of the unknown u from the previous
 * displacements u^t = d_u_n, u^{t-1} = d_u_nm1 and velocities v^t = d_v_n,
 * v^{t-1} = d_v_nm1 (device, internal layout, caller-owned, read while the
 * setting is in force); the approximate Jacobian used for preconditioning
 * gets -9/4 rho Omega_P / dt^2 on its diagonal (Section 3.1).  rho comes from
 * each mesh's material.  dt <= 0 removes the term.  J v differences only the
 * surface terms and adds the inertia's exact derivative.  Errors:
 * JFNK_E_ARG (null pointers, no mesh with rho > 0). */
jfnk_status jfnk_set_inertia(jfnk_mesh* mesh, double dt, const double* d_u_n, const double* d_u_nm1,
                             const double* d_v_n, const double* d_v_nm1, void* stream);

/* One BDF2 time step (Section 2.3.1, Eq. inertia2) with the loads at their
 * full value: on entry d_u, d_u_prev, d_v, d_v_prev, d_a hold u^t, u^{t-1},
 * v^t, v^{t-1} and a^t (device, internal layout; from rest all zero); the
 * step starts Newton from the truncated Taylor predictor of Section 3.2,
 * Eq. (predictor), u^t + dt v^t + dt^2/2 a^t (predictor != 0) or from u^t,
 * solves R(u^{t+1}) = 0 with the options' Newton and GMRES settings
 * (n_increments and the increment range are ignored), and on return holds
 * u^{t+1}, u^t, v^{t+1}, v^t, a^{t+1} with v^{t+1} = (3u^{t+1} - 4u^t +
 * u^{t-1})/(2 dt) and a^{t+1} = (3v^{t+1} - 4v^t + v^{t-1})/(2 dt).  A body
 * force set on the mesh applies.  d_work: jfnk_workspace_size op 2.
 * Returns the Newton status (the histories are updated either way). */
jfnk_status jfnk_dynamic_step(jfnk_mesh* mesh, double dt, int32_t predictor, const jfnk_newton_opts* opts,
                              double* d_u, double* d_u_prev, double* d_v, double* d_v_prev, double* d_a,
                              jfnk_stats* stats, void* d_work, void* stream);

/* Kernel timing for measurement tools.  While enabled, every residual / J v
 * evaluation on this mesh records HIP events around each of its kernels on
 * the caller's stream.  jfnk_profile_read() waits for the recorded events and
 * returns accumulated milliseconds and launch counts per kernel class:
 * [0] step-size norms, [1] gradient pass, [2] flux/divergence pass (or the
 * fused single pass, which has no separate gradient pass),
 * [3] preconditioner, [4] Arnoldi orthogonalisation (both Gram-Schmidt
 * passes, norm, Givens update, basis scaling), [5] other solver vector work
 * (solution update and true residual of a cycle), then optionally resets.
 * While profiling is on, GMRES launches directly (no graph replay).  Not for
 * concurrent callers. */
jfnk_status jfnk_profile_enable(jfnk_mesh* mesh, int32_t on);
jfnk_status jfnk_profile_read(jfnk_mesh* mesh, double* ms /*[6]*/, int64_t* calls /*[6]*/,
                              int32_t reset);

/* ---- Batches: many independent meshes solved together ----
 * A batch handle holds n meshes (segments) with their own materials.  Its
 * internal vectors cover all meshes: mesh s occupies internal cells
 * [cell_off_s, cell_off_s + n_cells_s) with cell_off_s a multiple of 256
 * (the gaps are padding cells whose entries stay zero), and every mesh is
 * processed by its own workgroups in the same kernel launches.  External
 * vectors concatenate the meshes' interleaved input-order vectors
 * (ext_off_s cells into the concatenation).  On a batch, jfnk_residual /
 * jfnk_jv / jfnk_gmres act on every mesh with its own material, J v step
 * (eps_used, stats: host arrays [n]), and convergence; the preconditioners
 * are built on the block-diagonal union of the meshes' approximate
 * Jacobians.  All meshes of a batch must have the same dim. */
jfnk_status jfnk_create_batch(const jfnk_mesh_desc* descs, const jfnk_material* mats, int32_t n,
                              void* stream, jfnk_mesh** out);
jfnk_status jfnk_segment_info(const jfnk_mesh* mesh, int32_t seg, int64_t* cell_off, int64_t* n_cells,
                              int64_t* ext_off);
/* Newton with load increments for every mesh of a batch in lockstep;
 * n_increments: host [n] (NULL: opts->n_increments for all).  Meshes finish
 * independently; stats and seg_status (host [n], may be NULL) are per mesh;
 * the return value is the first non-OK mesh status. */
/* Segregated solve of a single-mesh handle (see jfnk_segregated_opts)
 * from the given d_u.  d_work: a solve workspace (jfnk_workspace_size op 1)
 * for opts->precond, any restart.  stats: newton_it counts the outer
 * iterations, gmres_it the CG iterations, res0 / res_final the residual
 * norms of the last increment, t_ms[0] the wall time.  Returns JFNK_OK,
 * JFNK_E_NOT_CONVERGED (max_outer_it reached in an increment; d_u holds the
 * last iterate), JFNK_E_NAN, or JFNK_E_ARG (batch handle, bad option). */
jfnk_status jfnk_segregated_solve(jfnk_mesh* mesh, const jfnk_segregated_opts* opts, double* d_u,
                                  jfnk_stats* stats, void* d_work, void* stream);

jfnk_status jfnk_newton_solve_batch(jfnk_mesh* mesh, const int32_t* n_increments,
                                    const jfnk_newton_opts* opts, double* d_u, jfnk_stats* stats,
                                    jfnk_status* seg_status, void* d_work, void* stream);

/* ---- Serving: a request loop with continuous admission ----
 * Requests (a mesh, its material and Newton options) are queued in arrival
 * order.  Each of max_slots workers owns a HIP stream; a free worker takes
 * the next request, validates and preprocesses its mesh on the host, then
 * reserves the request's device footprint (mesh arrays + solver workspace +
 * preconditioner) from hbm_budget, waiting in arrival order until it fits,
 * and runs the solve on its stream.  Requests that arrive while others run
 * are admitted as soon as a slot and memory are free, and their kernels
 * overlap with the running ones on the device.  Each solve keeps its mesh,
 * Krylov basis and Newton state on the device until it completes; the
 * solution is copied to the caller's host array.  A request's result does
 * not depend on what else is running (same kernels, same order).
 * Latency = completion - submission (server clock).  dry_run_us_per_kcell
 * > 0 replaces the solve by a host sleep of that many microseconds per
 * 1000 cells and never touches the GPU (scheduler tests). */
typedef struct jfnk_server jfnk_server;

typedef struct {
  size_t hbm_budget;             /* device bytes the server may hold for requests */
  int32_t max_slots;             /* concurrent requests (one HIP stream each), >= 1 */
  int32_t max_queue;             /* queued requests before submit returns JFNK_E_BUSY */
  double dry_run_us_per_kcell;   /* > 0: scheduler-only mode, see above */
} jfnk_server_opts;

typedef struct {
  int32_t status;                /* jfnk_status of the request */
  int32_t state;                 /* 0 queued, 1 running, 2 done */
  double t_submit_ms, t_start_ms, t_done_ms;   /* server clock; start = HBM reservation granted */
  double latency_ms;             /* t_done - t_submit */
  int64_t footprint_bytes;
  int64_t n_cells;
  jfnk_stats stats;
  char error[160];             /* message of a failed request (empty otherwise) */
} jfnk_request_info;

typedef struct {
  int64_t submitted, completed, rejected, running, queued;
  int64_t hbm_in_use, hbm_peak;
  double p50_ms, p99_ms, mean_ms, max_ms;      /* latency of completed requests */
  double solves_per_s;           /* completed / (last completion - first submission) */
  int64_t cancelled;             /* requests removed by jfnk_server_cancel_queued */
} jfnk_server_metrics;

jfnk_status jfnk_server_create(const jfnk_server_opts* opts, jfnk_server** out);
/* Copies the mesh description; u_out (host [n_cells * dim], interleaved
 * input order, may be NULL) is written when the request completes and must
 * stay valid until then.  Returns JFNK_E_BUSY when the queue is full. */
jfnk_status jfnk_server_submit(jfnk_server* srv, const jfnk_mesh_desc* desc, const jfnk_material* mat,
                               const jfnk_newton_opts* opts, double* u_out, uint64_t* ticket);
jfnk_status jfnk_server_poll(jfnk_server* srv, uint64_t ticket, jfnk_request_info* info);
/* Blocks until the request is done. */
jfnk_status jfnk_server_wait(jfnk_server* srv, uint64_t ticket, jfnk_request_info* info);
jfnk_status jfnk_server_metrics_get(jfnk_server* srv, jfnk_server_metrics* m);
/* Removes every request that no worker has taken yet (their state becomes
 * done with status JFNK_E_BUSY and the message "cancelled before it
 * started"); running requests continue.  *n_cancelled (may be NULL) gets the
 * count.  For ending a measurement window or shedding a backlog. */
jfnk_status jfnk_server_cancel_queued(jfnk_server* srv, int64_t* n_cancelled);
/* Finishes running and queued requests, then stops the workers. */
jfnk_status jfnk_server_destroy(jfnk_server* srv);

/* ---- Tuning ----
 * jfnk_autotune times, on this handle's own mesh (or batch) and state u
 * (device, internal layout, load factor `load`), the launch shapes and
 * schedules that give identical results and keeps the fastest in the
 * handle: the cell passes of J v (one fused pass per tile, LDS-staged
 * gradient and flux passes, or direct gathers; one workgroup per tile or a
 * persistent grid), and the Arnoldi schedule
 * (steps per host check, HIP-graph replay) on one GMRES solve of
 * J x = -R(u) with `opts`, then the orthogonalisation (CGS2 or DCGS2) on
 * the same solve under the chosen schedule.  Later solves use the choice
 * when their options ask for the handle's values (step_chunk = 0,
 * graphs = 2, orth = 2).  d_work: a
 * solve workspace (op 1) for opts.restart and opts.precond.  The report
 * (may be NULL) lists every candidate and its time. */
typedef struct {
  int32_t lds_kernels;         /* chosen cell passes: 2 fused, 1 LDS-staged, 0 gathers */
  int32_t persist;             /* chosen: workgroups of a persistent launch (0: one per tile) */
  int32_t step_chunk;          /* chosen Arnoldi steps per host check */
  int32_t graphs;              /* chosen: 1 replay step runs from HIP graphs */
  int32_t n_jv;
  int32_t jv_lds[16], jv_persist[16];
  double jv_ms[16];            /* mean time of one J v per candidate */
  int32_t n_solve;
  int32_t solve_chunk[8], solve_graphs[8];
  double solve_ms[8];          /* time of the same GMRES solve per candidate */
  int32_t orth;                /* chosen orthogonalisation: 0 CGS2, 1 DCGS2 */
  double orth_ms[2];           /* the solve with CGS2 and with DCGS2 (0: not timed, DCGS2 not applicable) */
} jfnk_tune_report;

jfnk_status jfnk_autotune(jfnk_mesh* mesh, const jfnk_gmres_opts* opts, const double* d_u, double load,
                          void* d_work, void* stream, jfnk_tune_report* report);

/* Sets the cell passes of R(u) and J v by hand (what jfnk_autotune
 * chooses; every choice gives the same bits): passes 0 = direct gathers,
 * 1 = LDS-staged gradient and flux passes (mesh info `tiled`), 2 = one
 * fused pass per tile that recomputes the halo's gradients from a two-ring
 * copy in LDS (mesh info `fused`); persist = workgroups of a persistent
 * launch (0: one per tile; rounded up to a multiple of 8).  Call it between
 * solves, not while one runs on the handle.  Errors: JFNK_E_ARG (null mesh,
 * passes outside 0..2 or not supported by the mesh, persist < 0). */
jfnk_status jfnk_set_cell_passes(jfnk_mesh* mesh, int32_t passes, int32_t persist);

/* Shape of a handle's AMG hierarchy (Section 3.2's preconditioner built on
 * J_tilde of Section 3.1) for precond AMG32 or AMG64, once a solve or
 * jfnk_autotune has built it: levels from the finest, the scalar unknowns
 * (rows) of each, the stored nonzeros of each level's operator and the
 * lanes that share a row in its kernels (both 0 at the coarsest level,
 * which is solved by a dense inverse or, when its rows are uncoupled, a
 * diagonal), operator complexity, set-up time and device bytes.  Errors:
 * JFNK_E_ARG (null arguments, precond not AMG32 or AMG64, hierarchy not
 * built). */
typedef struct {
  int32_t n_levels;
  int32_t coarse_dense;        /* coarsest level: 1 dense inverse, 0 diagonal */
  int64_t rows[16];
  int64_t nnz[16];
  int32_t lanes[16];
  double operator_complexity;  /* sum of the levels' nonzeros over the finest level's */
  double setup_ms;
  int64_t device_bytes;
} jfnk_amg_info;

jfnk_status jfnk_amg_info_get(const jfnk_mesh* mesh, int32_t precond, jfnk_amg_info* info);

/* Thread-local message describing the last non-OK status on this thread. */
const char* jfnk_last_error(void);

/* Library version string. */
const char* jfnk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* JFNK_H */
