/*
 * feasm.h -- C ABI of the MI355X finite-element assembly + PCG library.
 *
 * Scope (paper: Oyarzun, Mira, Houzeaux, "Performance assessment of CUDA and
 * OpenACC in large scale combustion simulations"): the two operations that
 * take 99.84 % of a time step (Section 2, Table 1) -- element-by-element
 * matrix assembly into CSR (Section 4.2, Listing 1; Algorithm 1, first and
 * fourth steps) and the preconditioned conjugate-gradient pressure solve with
 * its SpMV, AXPY and dot kernels (Algorithm 1, last step; Section 5.2).
 *
 * General conventions
 *  - Every function returns fe_status; no C++ exception crosses the ABI.  On
 *    a non-OK status the outputs are unspecified unless stated, and
 *    fe_ctx_last_error() holds a message.
 *  - "device" pointers are HIP device memory on the context's device (for
 *    instance torch tensors' data_ptr()); "host" pointers are ordinary host
 *    memory, borrowed for the call only (never retained).
 *  - All device work is ordered on the context's stream.  Calls that return
 *    a result to the host (status words, CG scalars) synchronise that stream.
 *  - Mesh numbering: fe_mesh_upload may renumber nodes and elements for
 *    memory locality (the paper's renumbering by element type, Section 4.3,
 *    generalised to a space-filling-curve order).  Every per-node device
 *    array exchanged with the library (fields, values, rhs, x, g) is in MESH
 *    numbering; fe_mesh_node_perm() gives mesh index -> user node id and
 *    fe_mesh_to_mesh_order()/fe_mesh_to_user_order() convert device arrays.
 *  - Node ids and row/column indices are int32 (< 2^31); counts are int64.
 *  - A context is bound to one device and one stream; it and its meshes are
 *    not thread-safe (one host thread at a time).
 */
#ifndef FEASM_H
#define FEASM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FE_OK = 0,
    FE_EINVAL = 1,      /* bad argument (null pointer, negative count, bad enum) */
    FE_ENOMEM = 2,      /* device or host allocation failed, or budget exceeded */
    FE_EBADMESH = 3,    /* connectivity out of range, node in no element, row too long */
    FE_EBADELEM = 4,    /* det J <= 0 at a Gauss point (index in fe_asm_info) */
    FE_ENOCONV = 5,     /* CG reached max_iter (x still written) */
    FE_EBREAKDOWN = 6,  /* CG: p.Ap <= 0 or a non-finite scalar */
    FE_EDEVICE = 7,     /* a HIP call failed */
    FE_EBUSY = 8        /* serving: no slot free */
} fe_status;

/* Element types, value = nodes per element (the paper's meshes mix
 * tetrahedra, pyramids, prisms and hexahedra: Sections 3 and 4.2). */
typedef enum { FE_TET04 = 4, FE_PYR05 = 5, FE_PEN06 = 6, FE_HEX08 = 8 } fe_elem_type;
typedef enum { FE_FP64 = 0, FE_MIXED = 1 } fe_precision;
typedef enum { FE_OP_MOMENTUM = 0, FE_OP_SCALAR = 1, FE_OP_POISSON = 2 } fe_operator;

/* fe_mesh_upload flags */
#define FE_UPLOAD_RENUMBER 1u   /* reorder elements along a Morton curve, nodes by first touch */
#define FE_UPLOAD_COLOURED 2u   /* single-type meshes: assemble the matrix operators with the coloured
                                 * element blocks (the serving runtime's form, and always that of hybrid
                                 * meshes) instead of the owner groups; the two agree to rounding order */
#define FE_UPLOAD_GENERAL_SPMV 4u   /* fe_cg_solve runs the general SpMV on this mesh and never builds
                                     * the symmetric one's map: for a mesh solved once or a few times,
                                     * where building the map on the host (~3 ns per nonzero on 8
                                     * threads) costs more than the solves save (see fe_cg_solve) */

typedef struct fe_ctx_s *fe_ctx;
typedef struct fe_mesh_s *fe_mesh;

/* ---- context ------------------------------------------------------------ */

/* Bind to HIP device `device` and stream `hip_stream` (a hipStream_t; NULL =
 * the legacy default stream).  *out receives the context. */
fe_status fe_ctx_create(int device, void *hip_stream, fe_ctx *out);
/* Frees the context and every mesh still alive on it. */
void fe_ctx_destroy(fe_ctx ctx);
/* Message for the last non-OK status on this context (never NULL). */
const char *fe_ctx_last_error(fe_ctx ctx);
/* Re-bind the context (and its meshes) to another stream of the same device. */
fe_status fe_ctx_set_stream(fe_ctx ctx, void *hip_stream);

/* ---- mesh ----------------------------------------------------------------- */

/*
 * Preprocess and upload a single-type mesh (Section 4.2: unstructured mesh;
 * Section 4.3: elements grouped and renumbered for SIMD/SIMT execution).
 *   coords  host [n_nodes][3] float64 (user numbering)
 *   conn    host [n_elems][nen] int32, 0-based, every element positively
 *           oriented (det J > 0).  Node orders:
 *           HEX08 0:(-,-,-) 1:(+,-,-) 2:(+,+,-) 3:(-,+,-) 4:(-,-,+) 5:(+,-,+)
 *                 6:(+,+,+) 7:(-,+,+) in the reference cube [-1,1]^3;
 *           PEN06 (prism) 0,1,2 a triangle, 3,4,5 the nodes opposite 0,1,2
 *                 (reference triangle (0,0),(1,0),(0,1) at zeta = -1, +1);
 *           PYR05 (pyramid) 0-3 the quadrilateral base, counter-clockwise
 *                 seen from the apex 4 (reference (+-1,+-1,0), apex (0,0,1));
 *           TET04 vertices 0-3 of (0,0,0),(1,0,0),(0,1,0),(0,0,1).
 *   dirichlet_nodes host [n_dirichlet] user node ids, or NULL if n_dirichlet = 0
 * Builds the canonical CSR pattern (row i = every node sharing an element
 * with node i, columns ascending, explicit zeros kept), the element blocks,
 * their colouring and the scatter plan.  Errors: FE_EINVAL, FE_EBADMESH
 * (a connectivity entry out of range, a node in no element, or a node whose
 * CSR row would hold more than 255 entries: the scatter plans store in-row
 * positions as bytes; a hexahedral node may lie in up to 36 elements, a
 * tetrahedral one in up to ~80), FE_ENOMEM, FE_EDEVICE.  The mesh owns all
 * its device memory.  The planner keeps its host temporaries on the calling
 * thread for the next upload while they total at most 256 MiB (meshes up to
 * about 100^3 hexahedra); larger ones are released before the call returns.
 */
fe_status fe_mesh_upload(fe_ctx ctx, fe_elem_type type, int64_t n_nodes, const double *coords,
                         int64_t n_elems, const int32_t *conn, int64_t n_dirichlet,
                         const int32_t *dirichlet_nodes, uint32_t flags, fe_mesh *out);

/*
 * Hybrid mesh (the paper's meshes mix element types; Section 4.3 groups the
 * elements by type for vector execution): as fe_mesh_upload, with
 *   elem_types host [n_elems] uint8, the node count of each element
 *              (4 TET04, 5 PYR05, 6 PEN06, 8 HEX08)
 *   conn       host [n_elems][8] int32: element e's nodes in its first
 *              elem_types[e] slots, in its type's node order; the other
 *              slots are ignored.
 * Elements are grouped by type, every element block holds one type, and an
 * assembly runs one launch per (colour, type).  Errors: FE_EINVAL for an
 * unknown type, as fe_mesh_upload otherwise.
 */
fe_status fe_mesh_upload_mixed(fe_ctx ctx, int64_t n_nodes, const double *coords, int64_t n_elems,
                               const uint8_t *elem_types, const int32_t *conn, int64_t n_dirichlet,
                               const int32_t *dirichlet_nodes, uint32_t flags, fe_mesh *out);

typedef struct {
    int32_t nen;              /* nodes per element (the largest type of a hybrid mesh) */
    int64_t n_nodes, n_elems, nnz;
    const int32_t *rowptr;    /* device [n_nodes+1], mesh numbering */
    const int32_t *colidx;    /* device [nnz], ascending per row */
    int64_t n_blocks;         /* element blocks (one wavefront each) */
    int32_t n_colors;         /* block colours (assembly launches per operator: one per colour and type) */
    int32_t max_row;          /* longest CSR row */
    int64_t n_dirichlet;
    size_t device_bytes;      /* device memory held by the mesh */
} fe_mesh_desc;

fe_status fe_mesh_info(fe_mesh mesh, fe_mesh_desc *out);
/* host perm[n_nodes]: perm[mesh index] = user node id.  elem_perm likewise
 * for elements (either pointer may be NULL). */
fe_status fe_mesh_perm(fe_mesh mesh, int32_t *node_perm, int32_t *elem_perm);
/* Copy the CSR pattern to host arrays rowptr[n_nodes+1], colidx[nnz]
 * (mesh numbering; either pointer may be NULL).  Synchronises the stream. */
fe_status fe_mesh_pattern_host(fe_mesh mesh, int32_t *rowptr, int32_t *colidx);
/* Device permutation of ncomp node arrays stored [ncomp][n_nodes]. */
fe_status fe_mesh_to_mesh_order(fe_mesh mesh, const double *user_in, double *mesh_out, int32_t ncomp);
fe_status fe_mesh_to_user_order(fe_mesh mesh, const double *mesh_in, double *user_out, int32_t ncomp);
void fe_mesh_free(fe_mesh mesh);

/* ---- assembly --------------------------------------------------------------- */

/* Nodal fields, device arrays in mesh numbering. */
typedef struct {
    fe_operator op;
    double dt;            /* time step, > 0 */
    const double *u;      /* [3][n_nodes] velocity */
    const double *rho;    /* [n_nodes] density */
    const double *mu;     /* [n_nodes] viscosity (MOMENTUM only) */
    int32_t n_scalars;    /* SCALAR: 1..8 */
    const double *Y;      /* SCALAR: [n_scalars][n_nodes] transported scalars */
    const double *D;      /* SCALAR: HOST [n_scalars] diffusivities */
} fe_fields;

typedef struct {
    double min_detJ;         /* smallest det J met (FP64) */
    int64_t first_bad_elem;  /* user element id of the first det J <= 0, or -1 */
} fe_asm_info;

/*
 * Element-by-element assembly (Section 4.2, Listing 1, generalised to the
 * operators of Eq. (1) in a reduced form: Galerkin advective convection
 * linearised about the nodal velocity, Laplacian-form viscous term, one
 * scalar operator shared by the three velocity components):
 *   MOMENTUM: values[1][nnz] = M_rho/dt + C(u) + K_mu,  rhs[3][n_nodes] = M_rho u_i/dt
 *   SCALAR  : values[k][nnz] = M_rho/dt + C(u) + K_{rho D_k}, rhs[k][n_nodes] = M_rho Y_k/dt
 *   POISSON : values[1][nnz] = L (constant coefficient), rhs[1][n_nodes] = (1/dt) int grad N . (rho u)
 * values and rhs are caller-owned device arrays and are overwritten (not
 * added to).  FE_FP64 does everything in FP64; FE_MIXED forms the Gauss-point
 * products and elemental sums in FP32 while the Jacobian, its determinant
 * and inverse and the CSR accumulation stay FP64.  The scatter is
 * deterministic: the same inputs give bitwise the same outputs.  Returns
 * after reading back a device status word; FE_EBADELEM reports the element
 * in *info (info may be NULL).
 */
fe_status fe_assemble(fe_mesh mesh, const fe_fields *fields, fe_precision prec, double *values,
                      double *rhs, fe_asm_info *info);

/*
 * The implicit momentum operator of Eq. (1) with the viscous term in its
 * full-stress form -div(2 mu eps(u)) (Section 2), which couples the three
 * velocity components: 3x3 blocks on the mesh's scalar CSR pattern.  Testing
 * with N_a e_i, row (a, i) and column (b, k) of the element matrix are
 *   delta_ik (M_ab/dt + C_ab + K_ab + E_ab) + T_ab[i][k],
 *   T_ab[i][k] = int mu (dN_a/dx_k)(dN_b/dx_i)       (form FE_FORM_FULL_STRESS),
 *   E_ab       = int rho (div u) N_a N_b              (form FE_FORM_EMAC: the
 *                (div u) u term of the EMAC convection, u frozen at the nodal
 *                velocity),
 * with M_rho, C(u), K_mu those of fe_assemble(MOMENTUM); a term whose bit is
 * clear is left out (form 0 = fe_assemble(MOMENTUM)'s matrix times the
 * identity).  FP64.
 *   u [3][n_nodes], rho, mu [n_nodes]: device, mesh numbering
 *   values: device [nnz][3][3], overwritten: block (i, k) of CSR entry p at
 *           values[9 p + 3 i + k] (pattern of fe_mesh_info, mesh numbering)
 *   rhs:    device [3][n_nodes], overwritten: M_rho u_i / dt
 * With b = rhs, b - A u equals rows 0-2 of fe_residual(u, form) (the mass
 * terms cancel).  Every CSR block row is written once (no
 * read-back); the sums run in a fixed order, so the result is bitwise
 * reproducible.  The first call on a mesh plans the row-owner assembly on the
 * host and keeps the plan on the device (about 14 bytes per element node).
 * Errors: FE_EINVAL, FE_EBADELEM (element in *info), FE_EBADMESH if a node
 * lies in more than 64 elements, FE_ENOMEM, FE_EDEVICE.
 */
fe_status fe_assemble_block(fe_mesh mesh, uint32_t form, double dt, const double *u, const double *rho,
                            const double *mu, double *values, double *rhs, fe_asm_info *info);

/*
 * Symmetric Dirichlet elimination on the mesh's Dirichlet nodes, in place:
 * free rows i: rhs_i -= sum_{j in D} A_ij g_j, A_ij = 0 (j in D);
 * Dirichlet rows: off-diagonals 0, diagonal kept, rhs_i = A_ii g_i.
 * g: device [n_nodes] or NULL for g = 0.
 */
fe_status fe_apply_dirichlet(fe_mesh mesh, double *values, double *rhs, const double *g);

/* ---- solver kernels (Section 5.2: SpMV, AXPY, dot) -------------------------- */

/* y = A x on the mesh pattern (device arrays, FP64). */
fe_status fe_spmv(fe_mesh mesh, const double *values, const double *x, double *y);
/* *out (host) = x . y over n entries; deterministic two-stage reduction. */
fe_status fe_dot(fe_ctx ctx, int64_t n, const double *x, const double *y, double *out);
/* y += a x over n entries. */
fe_status fe_axpy(fe_ctx ctx, int64_t n, double a, const double *x, double *y);

typedef struct {
    int32_t iterations;        /* inner (FP32 in mixed mode) CG iterations in total */
    int32_t outer_iterations;  /* refinement steps (mixed); 1 for FE_FP64 */
    double rel_residual;       /* ||r||/||b|| from the recurrence (FP64 outer residual in mixed) */
    double true_rel_residual;  /* ||b - A x||/||b|| recomputed in FP64 */
    int32_t symmetric_spmv;    /* 1: the FP64 iterations ran the symmetric SpMV (see fe_cg_solve), else 0 */
} fe_cg_info;

/*
 * Jacobi-preconditioned CG on the assembled SPD system (Algorithm 1, last
 * step).  x: device [n_nodes], in = x0, out = solution.  Stops when
 * ||r||_2 <= rtol ||b||_2; rtol <= 0 runs exactly max_iter iterations and
 * returns FE_OK.  FE_MIXED runs FP32 Jacobi-PCG on an FP32 copy of the
 * matrix inside FP64 iterative refinement (residual and norms in FP64).
 * FE_FP64 iterations use a symmetric SpMV when the matrix is symmetric:
 * each pair a_ij, a_ji whose rows fall in one SpMV row block is read once,
 * from the upper entry.  The call checks every such pair first (|a_ij -
 * a_ji| <= 2^-40 max(|a_ij|, |a_ji|, sqrt|a_ii a_jj|), both finite) and
 * otherwise runs the general SpMV; info->symmetric_spmv says which ran.
 * The first FP64 solve on a mesh builds the symmetric map on the host and
 * keeps it, with a packed copy of the values, on the device (about 8
 * bytes per nonzero; without room for them the general SpMV runs).
 * The two SpMVs round differently; the true residual is always computed
 * with `values` as given.  Returns FE_ENOCONV (x written) at max_iter,
 * FE_EBREAKDOWN on p.Ap <= 0 or non-finite scalars.  info may be NULL.
 */
fe_status fe_cg_solve(fe_mesh mesh, const double *values, const double *rhs, double *x, double rtol,
                      int32_t max_iter, fe_precision prec, fe_cg_info *info);

/*
 * Allocation-free FP64 Jacobi-PCG, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same solve, arguments and errors as
 * fe_cg_solve(..., FE_FP64, ...) with the general SpMV (the symmetric one
 * needs the packed values, which would need an allocation): results agree
 * with fe_cg_solve's to rounding, and are bitwise its results whenever
 * fe_cg_solve runs the general SpMV too.  The work vectors r, z, p, q, D^-1, the residual, the partial
 * sums, the per-iteration scalars and the stop word live in one fixed device
 * area of FE_NOALLOC_BYTES per device (a static device array, held from the
 * first fe_ctx_create on that device until the process ends) instead of
 * buffers allocated on the mesh; every iteration is launched on its own (no
 * graph is recorded).  The call allocates nothing.  It needs
 *   6 * round256(8 n_nodes) + 65792 + round256(8 (4 max(max_iter + 2, 256) + 4))
 * bytes of the area (about 1.39 M nodes at 64 MiB): FE_ENOMEM otherwise,
 * with the sizes in fe_ctx_last_error().  Every call on one device shares
 * that device's area and leaves its contents behind (each call initialises
 * what it reads): calls that overlap on one device -- two streams, two
 * contexts, two host threads -- race and give wrong results.  Synchronises
 * the stream.
 */
#define FE_NOALLOC_BYTES ((size_t)64 << 20)
fe_status fe_cg_solve_noalloc(fe_mesh mesh, const double *values, const double *rhs, double *x, double rtol,
                              int32_t max_iter, fe_cg_info *info);

/* ---- explicit step (Algorithm 1: Runge-Kutta momentum stages, pressure,
 *      velocity correction) ---------------------------------------------------
 * The paper's time step assembles the momentum equations inside Runge-Kutta
 * stages, solves the pressure equation with PCG and corrects the velocity
 * (Algorithm 1; the scheme itself is in a reference the paper cites).  The
 * stages use the operator of fe_assemble(MOMENTUM) without its mass term,
 * applied to the velocity element by element (no matrix is formed).  All
 * arrays are device, mesh numbering, [k][n_nodes] rows, FP64.  Each call
 * synchronises the stream and fails with FE_EBADELEM on det J <= 0. */

/* Scalar transport (the heat and species equations, which the paper
 * advances with the same Runge-Kutta stages and no algebraic solver,
 * Section 2).  fe_scalar_residual: out[2][n], out_0 = -(C(u) + K_{rho D}) Y,
 * i.e. -sum_e int rho (N_a (u . grad Y) + D grad N_a . grad Y), and out_1 =
 * the lumped rho-mass.  fe_scalar_step: one three-stage SSP Runge-Kutta step
 * of M_L dY/dt = fe_scalar_residual(Y), Y [n] in/out held at the mesh's
 * Dirichlet nodes (work buffer of 3 n doubles on the mesh).  D >= 0. */
fe_status fe_scalar_residual(fe_mesh mesh, const double *u, const double *rho, const double *Y, double D,
                             double *out);
fe_status fe_scalar_step(fe_mesh mesh, double dt, const double *u, const double *rho, double D, double *Y);

/* Operator variants of Eq. (1) for the residual (bits of `form`; 0 = the
 * advective convection and Laplacian viscous forms of fe_assemble). */
#define FE_FORM_FULL_STRESS 1u   /* viscous term div(2 mu eps(u)): adds mu (d u_j/d x_i)(d N_a/d x_j) */
#define FE_FORM_EMAC 2u          /* convective term 2 eps(u) u + (div u) u - grad(|u|^2)/2 at the Gauss
                                  * points, i.e. (u . grad) u + (div u) u: adds rho N_a (div u) u_i */

/* out[4][n]: out_i = -(C(u) + K_mu) u_i for i = 0, 1, 2, i.e. per node a
 *   -sum_e int rho N_a (u . grad u_i) + mu grad N_a . grad u_i
 * (with the terms `form` adds), and out_3 = the rho-weighted lumped mass
 * int rho N_a (row sums of M_rho).  FE_EINVAL for unknown form bits. */
fe_status fe_residual(fe_mesh mesh, const double *u, const double *rho, const double *mu, uint32_t form,
                      double *out);
/* g[3][n]: g_j = int N_a d p / d x_j (the pressure gradient tested with N_a). */
fe_status fe_gradient(fe_mesh mesh, const double *p, double *g);
/* f[n] = (1/dt) int grad N_a . (rho u): the right-hand side of
 * fe_assemble(POISSON) without its matrix. */
fe_status fe_divergence(fe_mesh mesh, double dt, const double *u, const double *rho, double *f);

/*
 * Boundary assembly of the wall model (Algorithm 1; the paper names the wall
 * model without its law).  An equilibrium law of the wall, Reichardt's with
 * kappa = 0.41, at exchange distance delta: at each Gauss point of a wall
 * face the tangential part u_t of the interpolated velocity gives u_tau from
 * |u_t| = u_tau u+(delta u_tau / nu), nu = mu / rho (16 Newton steps from
 * the laminar guess), and the traction t = -rho u_tau^2 u_t / |u_t| is
 * integrated against the face's shape functions.
 *
 * fe_wall_faces registers (or, with n_faces = 0, clears) the mesh's wall
 * faces: face_nen host [n_faces] 3 (triangle: 3-point rule) or 4
 * (quadrilateral, nodes in cyclic order: 2x2 Gauss); face_conn host
 * [n_faces][4] user node ids (a triangle's fourth slot is ignored); delta
 * > 0.  Faces must have non-zero area.  Errors: FE_EINVAL, FE_ENOMEM,
 * FE_EDEVICE; after a failed call the mesh has no wall faces.  The call
 * synchronises the stream before it replaces faces already registered.
 * fe_wall_traction: out[3][n] (device, mesh numbering) = the traction's
 * nodal vector, zero away from the wall; deterministic (fixed summation
 * order).  fe_fractional_step adds it to every Runge-Kutta stage's residual
 * when wall faces are registered.
 */
fe_status fe_wall_faces(fe_mesh mesh, int64_t n_faces, const uint8_t *face_nen, const int32_t *face_conn,
                        double delta);
fe_status fe_wall_traction(fe_mesh mesh, const double *u, const double *rho, const double *mu, double *out);

typedef struct {
    int32_t cg_iterations;        /* PCG iterations of the pressure solve */
    double cg_true_rel_residual;  /* ||f - L p|| / ||f|| in FP64 */
} fe_step_info;

/*
 * One fractional step:
 *   1. predictor: three-stage strong-stability-preserving Runge-Kutta
 *      (Shu-Osher) on M_L du/dt = fe_residual(u, form) (+ fe_wall_traction(u)
 *      when wall faces are registered), M_L the lumped rho-mass;
 *      u at the mesh's Dirichlet nodes is held;
 *   2. pressure: L p = fe_divergence(u*) with zero at the Dirichlet rows,
 *      fe_cg_solve to rtol in precision prec (FE_MIXED: FP32 PCG inside FP64
 *      refinement) starting from p (in: initial guess);
 *   3. correction: u = u* - dt M_L^-1 fe_gradient(p) at the free nodes.
 * L: device [nnz] values of the Poisson matrix after fe_apply_dirichlet
 * (assembled once, Algorithm 1, first step).  u [3][n] in/out, p [n] in/out.
 * Work buffers (11 n doubles) are allocated on the mesh at the first call.
 * Returns FE_ENOCONV / FE_EBREAKDOWN from the solve (u then holds u*).
 */
fe_status fe_fractional_step(fe_mesh mesh, double dt, const double *rho, const double *mu, const double *L,
                             uint32_t form, double *u, double *p, double rtol, int32_t max_iter,
                             fe_precision prec, fe_step_info *info);

/* ---- serving: continuous batching of assemble + solve requests -------------
 * The time-step workload of the paper (Algorithm 1: momentum assembly, the
 * pressure system's assembly and its PCG solve; Section 2) offered as a
 * service for many independent meshes.  A server owns one device arena of
 * hbm_budget bytes (allocated once at creation: requests never call
 * hipMalloc), host planner threads and one dispatcher thread with its own
 * HIP stream.  A request runs in four stages:
 *   1. a planner thread validates and plans its mesh (the fe_mesh_upload
 *      preprocessing, renumbering on) and computes its device footprint;
 *   2. admission: when a slot is free and the footprint fits in the arena's
 *      free space, the dispatcher uploads the mesh and fields and queues the
 *      momentum assembly (M/dt + C + K with its 3 right-hand sides), the
 *      Poisson assembly, the Dirichlet elimination and the PCG set-up;
 *   3. batched PCG: every iteration advances all admitted requests with
 *      three launches in total (SpMV with p.Ap, the x/r/z update, the
 *      p update), each request keeping its own scalars and stop test;
 *   4. completion: the FP64 true residual, copies back to the host, and the
 *      request's arena space is returned for the next admission.
 * A request's numbers do not depend on the other requests in flight: its
 * work-group counts and summation orders are the ones of a request served
 * alone (and of fe_cg_solve_noalloc on the same system, the mesh uploaded
 * with FE_UPLOAD_COLOURED: served meshes are assembled by coloured element
 * blocks, since the owner plan's host time exceeds the assembly time it saves
 * for a mesh assembled once; the batched PCG runs the general SpMV).
 *
 * Host arrays of a request are borrowed from fe_serve_submit until the
 * request is reported done; they must stay valid and unchanged until then.
 * The server keeps up to host_threads planned images of finished requests
 * (their host arrays' capacity, as large as the largest mesh planned) and
 * each planner thread its planning temporaries (up to 256 MiB), reused by
 * the next plans; fe_serve_destroy releases them.
 * The server functions may be called from any host thread. */
typedef struct fe_server_s *fe_server;

typedef struct {
    fe_elem_type type;
    int64_t n_nodes;
    const double *coords;           /* host [n_nodes][3] */
    int64_t n_elems;
    const int32_t *conn;            /* host [n_elems][nen], user node ids */
    int64_t n_dirichlet;
    const int32_t *dirichlet_nodes; /* host [n_dirichlet]: homogeneous Dirichlet nodes of the Poisson system */
    double dt;
    const double *u;                /* host [3][n_nodes] velocity, user numbering */
    const double *rho;              /* host [n_nodes] */
    const double *mu;               /* host [n_nodes] */
    double rtol;                    /* PCG stop: ||r||_2 <= rtol ||b||_2 (> 0) */
    int32_t max_iter;
    double *x;                      /* host [n_nodes] out: pressure solution, user numbering */
    double *mom_rhs;                /* host [3][n_nodes] out (user numbering) or NULL */
    const uint8_t *elem_types;      /* NULL: every element is `type`; else a hybrid mesh as in
                                     * fe_mesh_upload_mixed: host [n_elems] node counts, conn
                                     * [n_elems][8] (type is then ignored) */
} fe_job;

typedef struct {
    fe_status status;               /* FE_OK, FE_ENOCONV (x written), FE_EBADELEM, FE_EBADMESH, ... */
    int32_t iterations;
    double rel_residual;            /* recursive ||r||/||b|| at the last iteration */
    double true_rel_residual;       /* ||b - A x|| / ||b|| recomputed in FP64 */
    double min_detJ;
    int64_t first_bad_elem;         /* user element id with det J <= 0, or -1 */
    double plan_ms;                 /* submit -> planned */
    double wait_ms;                 /* planned -> admitted */
    double run_ms;                  /* admitted -> results on the host */
    double total_ms;                /* submit -> done */
    char message[128];              /* detail for a non-OK status */
} fe_job_result;

/* max_slots: requests in flight on the device (1..32); host_threads:
 * planner threads (>= 1).  hbm_budget: arena bytes. */
fe_status fe_serve_create(fe_ctx ctx, size_t hbm_budget, int32_t max_slots, int32_t host_threads,
                          fe_server *out);
/* Queues a request; *ticket identifies it.  FE_ENOMEM (reported through the
 * result) if its footprint exceeds the whole arena. */
fe_status fe_serve_submit(fe_server server, const fe_job *job, int64_t *ticket);
/* *done = 1 and *result filled once the request is complete (then the
 * ticket is released); *done = 0 otherwise.  FE_EINVAL for an unknown ticket. */
fe_status fe_serve_poll(fe_server server, int64_t ticket, int32_t *done, fe_job_result *result);
/* Blocks until the request is complete, fills *result, releases the ticket. */
fe_status fe_serve_wait(fe_server server, int64_t ticket, fe_job_result *result);
/* Counters: requests completed, batched PCG iterations launched, sum over
 * those launches of the requests they carried (occupancy = ratio). */
fe_status fe_serve_stats(fe_server server, int64_t *completed, int64_t *batches, int64_t *batched_requests);
/* Waits for every submitted request, then frees the server. */
void fe_serve_destroy(fe_server server);

/* ---- measurement hooks --------------------------------------------------------
 * With profiling on, the library brackets its launches with HIP events on the
 * context's stream: slot 0 = the SpMV launch of one PCG iteration (fused with
 * p.Ap), slot 1 = one fe_assemble call (all colours), slot 2 = the vector
 * updates of one PCG iteration, slot 3 = fe_apply_dirichlet, slot 4 = one
 * element-vector pass (fe_residual, fe_gradient, fe_divergence and those of
 * fe_fractional_step).
 * fe_ctx_profile() clears the records; fe_ctx_profile_read() synchronises
 * and returns the number of bracketed intervals and their summed duration. */
fe_status fe_ctx_profile(fe_ctx ctx, int enable);
fe_status fe_ctx_profile_read(fe_ctx ctx, int slot, int64_t *launches, double *total_ms);

/* ---- host-only preprocessing (no device needed; used to test the planner) --- */

typedef struct fe_plan_s *fe_plan;
typedef struct {
    int64_t n_nodes, n_elems, nnz, n_blocks;
    int32_t n_colors, max_row, max_block_nodes, max_block_slots, max_phases;
} fe_plan_desc;

/* Same preprocessing as fe_mesh_upload, kept on the host. */
fe_status fe_plan_create(fe_elem_type type, int64_t n_nodes, const double *coords, int64_t n_elems,
                         const int32_t *conn, uint32_t flags, fe_plan *out);
fe_status fe_plan_info(fe_plan plan, fe_plan_desc *out);
/* Copy host arrays out (any pointer may be NULL):
 *   node_perm[n_nodes], elem_perm[n_elems], rowptr[n_nodes+1], colidx[nnz],
 *   block_elem_ptr[n_blocks+1], block_color[n_blocks],
 *   block_node_ptr[n_blocks+1] then block_nodes[block_node_ptr[n_blocks]]. */
fe_status fe_plan_export(fe_plan plan, int32_t *node_perm, int32_t *elem_perm, int32_t *rowptr,
                         int32_t *colidx, int32_t *block_elem_ptr, int32_t *block_color,
                         int32_t *block_node_ptr, int32_t *block_nodes);
/* Same preprocessing as fe_mesh_upload_mixed, kept on the host. */
fe_status fe_plan_create_mixed(int64_t n_nodes, const double *coords, int64_t n_elems, const uint8_t *elem_types,
                               const int32_t *conn, uint32_t flags, fe_plan *out);
/* Types of the plan (any pointer may be NULL): elem_types[n_elems] per
 * element in mesh order, block_types[n_blocks], and the assembly launches as
 * launches[3 * n_launches] = {nodes per element, first, count} over the
 * colour-ordered block list (*n_launches receives their number; size the
 * array by a first call with launches = NULL). */
fe_status fe_plan_export_types(fe_plan plan, uint8_t *elem_types, uint8_t *block_types, int32_t *launches,
                               int64_t *n_launches);
/* color_blocks[n_blocks]: the blocks in launch order (by colour, then type). */
fe_status fe_plan_export_color_blocks(fe_plan plan, int32_t *color_blocks);
/*
 * Owner plan of the matrix assembly of a single-type mesh (Section 4.2's
 * element loop regrouped by the CSR rows it writes; fe_assemble runs it for
 * MOMENTUM, SCALAR and POISSON on single-type meshes uploaded without
 * FE_UPLOAD_COLOURED, and the coloured element blocks otherwise and for
 * hybrid meshes).  Rows, in mesh numbering, are
 * cut into groups of consecutive rows; a work-group owns one group and
 * computes every element contribution to its rows.  A task is one lane's
 * share: an element's rows that the group owns -- for HEX08 at most 4, with
 * the element presented in a rotated node order that puts them on its first
 * face (two tasks when they lie on no single face), for the other types all
 * of the element's rows, the rows the group does not own being dropped.
 * fe_plan_owner_info: counts, and *wave_private = 1 when each wavefront (64
 * consecutive tasks of a group) accumulates into its own copy of the
 * group's rows (the copies then summed in wave order; phases are then per
 * wave), 0 for one shared copy with phases over the group (HEX08);
 * FE_EINVAL for a hybrid plan.
 * fe_plan_export_owner (any pointer may be NULL):
 *   groups[4 n_groups] = {first task, tasks, first row, rows},
 *   node_ptr[n_groups + 1], nodes[node_ptr[n_groups]]: each group's touched
 *     nodes, its own rows first (in order), then the others ascending,
 *   nphase[n_groups]: phases of the group's LDS accumulation,
 *   task_elem[n_tasks]: mesh element; task_ln[n_tasks * ln_stride] (16-bit):
 *     the group-local node of each (rotated) element node; task_off[n_tasks *
 *     off_stride]: for row r < rows_per_task and column b, the position of
 *     node b in row r's CSR columns at r * nodes_per_element + b (0 for rows
 *     the group does not own); task_phase[n_tasks].
 */
fe_status fe_plan_owner_info(fe_plan plan, int64_t *n_groups, int64_t *n_tasks, int32_t *rows_per_task,
                             int32_t *ln_stride, int32_t *off_stride, int32_t *wave_private);
fe_status fe_plan_export_owner(fe_plan plan, int32_t *groups, int32_t *node_ptr, int32_t *nodes, uint8_t *nphase,
                               int32_t *task_elem, uint16_t *task_ln, uint8_t *task_off, uint8_t *task_phase);
void fe_plan_free(fe_plan plan);
/* Message for the last failure of fe_plan_create(_mixed) on this thread. */
const char *fe_plan_last_error(void);

/* Pack layout of Section 4.3: n_elems elements of one type in packs of
 * vector_size, the last pack zero-padded.  *packs, *padded receive counts. */
fe_status fe_pack_layout(int64_t n_elems, int32_t vector_size, int64_t *packs, int64_t *padded);

#ifdef __cplusplus
}
#endif
#endif /* FEASM_H */
