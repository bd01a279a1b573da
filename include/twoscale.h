/*
 * twoscale.h -- C ABI of the MI355X two-scale surrogate-stencil library.
 *
 * Method: Bauer, Mohr, Ruede, Weismueller, Wittmann, Wohlmuth, "A two-scale
 * approach for efficient on-the-fly operator assembly in massively parallel
 * high performance multigrid codes" (arXiv 1608.06473).  The library solves
 * -Laplace(u) = f on a spherical shell with u = 0 on the boundary (Sec. 2.1,
 * eq. model_eq) with P1 finite elements on hierarchically refined macro
 * tetrahedra mapped by a blending function (Sec. 2.2), and replaces the
 * on-the-fly element assembly of the 15-point volume stencils by surrogate
 * polynomials fitted per macro and level (Sec. 3).
 *
 * Conventions used by every call:
 *  - level: N = 2^level fine intervals per macro edge (the paper's level l
 *    is level - 2; level 2 has one interior node per macro and is the
 *    coarsest multigrid level).  Valid levels are 2..9.
 *  - Vector layout ("block layout"): macro-major; inside macro m all
 *    (N+1)(N+2)(N+3)/6 nodes (i, j, k) >= 0, i + j + k <= N, plane k outer,
 *    row j, index i inner:
 *        slot = m * B + (tet(N+1) - tet(N+1-k)) + j (N+1-k) - j (j-1)/2 + i,
 *    tet(n) = n (n+1) (n+2) / 6, B = tet(N+1).  Macro m's fine node (i,j,k)
 *    has barycentric weights (N-i-j-k, i, j, k)/N of its vertices in the
 *    order given to ts_mesh_create.  Nodes on faces, edges and vertices of
 *    the macro mesh appear once in every macro that contains them; library
 *    calls take inputs whose copies agree and keep outputs that way.
 *    Dirichlet nodes (on a face of the mesh boundary) hold 0.
 *  - Canonical order (for exchange with other codes): vertices by id; edges
 *    (g0 < g1) lexicographic, points a = 1..N-1 (weight of g1 = a/N); faces
 *    (g0 < g1 < g2) lexicographic, points b = 1..N-2, a = 1..N-1-b (weights
 *    of g1, g2 = a/N, b/N); then per macro its interior points in block
 *    order.
 *  - Vectors are device pointers owned by the caller (float64 for TS_F64,
 *    float32 for TS_F32 and TS_F16W).  Library objects own their device
 *    memory and free it in *_destroy.  Work is enqueued on the given HIP
 *    stream (NULL: the default stream) and is asynchronous unless stated.
 *  - Every call returns TS_OK or an error code; ts_last_error() describes the
 *    last failure of the calling thread.  No C++ exception crosses the ABI.
 */
#ifndef TWOSCALE_H
#define TWOSCALE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ts_mesh ts_mesh;
typedef struct ts_op ts_op;
typedef struct ts_solver ts_solver;
typedef void *ts_stream; /* hipStream_t */

enum {
    TS_OK = 0,
    TS_EINVAL = 1,     /* bad argument */
    TS_ENOMEM = 2,     /* device allocation failed or exceeds a budget */
    TS_EHIP = 3,       /* HIP runtime error */
    TS_ENOCONV = 4,    /* solver did not reach the tolerance (info filled) */
    TS_ENONFINITE = 5  /* NaN or Inf in an input or an iterate */
};

enum { TS_GEOM_SHELL = 0, TS_GEOM_AFFINE = 1 };
/* TS_LSQP_SYM: the symmetric surrogate of the remark at the end of Sec. 3.4,
 * one polynomial per edge direction evaluated at the edge midpoint, fitted by
 * least squares like LSQP to the exact weights of both directions; the centre
 * weight is minus the sum of the others (the operator's centre mode is set to
 * TS_CENTER_ROWSUM), so the volume rows of a macro form a symmetric matrix. */
/* TS_CONS: the constant-stencil operator the paper takes as the lower bound
 * of the method's cost (Sec. 4.2.1 Tab. flops: 29 FLOP per update; Sec. 5
 * introduction: the cycle time on unprojected geometry).  Each macro's volume
 * rows use one stencil, the exact stencil of the macro's unmapped fine
 * tetrahedra (Phi = Id there); the lower-primitive rows are those of the
 * mesh geometry, as for every method.  On a TS_GEOM_AFFINE mesh it is the
 * exact operator.  q, sample_j are ignored; no face surrogate, no fallback
 * check. */
enum { TS_IFEM = 0, TS_LSQP = 1, TS_IPOLY = 2, TS_LSQP_SYM = 3, TS_CONS = 4 };
enum { TS_CENTER_POLY = 0, TS_CENTER_ROWSUM = 1 };
enum { TS_F64 = 0, TS_F32 = 1, TS_F16W = 2 };
enum { TS_RHS_MANUFACTURED = 0, TS_RHS_BUMPS = 1, TS_RHS_ONE = 2 };

typedef struct {
    int level;
    int N;
    int64_t n_macros;
    int64_t block_size;   /* B */
    int64_t vec_len;      /* n_macros * B */
    int64_t n_unique;     /* unique nodes incl. Dirichlet */
    int64_t n_free;       /* unknowns */
    int64_t n_volume;     /* interior (volume-primitive) nodes */
} ts_layout_info;

typedef struct {
    int method;   /* TS_LSQP, TS_IPOLY, TS_LSQP_SYM, TS_CONS or TS_IFEM (exact
                     on-the-fly assembly) */
    int q;        /* surrogate degree 1..4 (IPOLY: 2) */
    int sample_j; /* LSQP sampling set M_{m(l,j)}, m = min(l, max(1, j)) */
    int center;   /* TS_CENTER_POLY or TS_CENTER_ROWSUM */
    double fallback_tol; /* selective surrogate (remark in Sec. 3.4): a macro
                            keeps IFEM volume rows on a level if at one of the
                            check points (1,1,1), (N-3,1,1), (1,N-3,1),
                            (1,1,N-3), (N/4,N/4,N/4) its surrogate centre
                            weight is <= 0 or differs from the exact one by
                            more than fallback_tol times it; <= 0: never */
    int face_surrogate;  /* non-zero: the rows of free interior-face nodes also
                            come from surrogate polynomials (the remark after
                            eq. numInteriorPoints): per face and level each of
                            the 15 row entries (the node, the other
                            directions of its first macro that stay in it,
                            the inward directions of the second macro) is a
                            2D polynomial of degree q in the face, fitted by
                            least squares to the exact rows at the face nodes
                            of the LSQP sampling lattice (m = min(l, max(1,
                            sample_j))); centre from its own polynomial.  On
                            levels where the selective surrogate keeps IFEM
                            volume rows on some macro, and in exact residuals,
                            every face keeps its exact rows.  0: exact face
                            rows (default) */
    int coarse_from_finest; /* non-zero: the coarser levels evaluate the
                               finest level's surrogate polynomials (the
                               remark in Sec. 3.4 on using the fine-level
                               polynomial on the coarser meshes): their
                               volume coefficients are the finest level's
                               times 2^(max_level - l), the ratio of the mesh
                               sizes (stiffness weights scale with h), and no
                               fit runs on them; face fits and the fallback
                               check stay per level.  Ignored by TS_IFEM and
                               TS_CONS; TS_EINVAL with TS_LSQP_SYM (its node
                               coefficients hold a shift of half a mesh step,
                               which differs per level).  0: one fit per
                               level (default) */
} ts_op_params;

typedef struct {
    int nu1, nu2;        /* V(nu1, nu2), default 3, 3 */
    int max_cycles;      /* cap on outer iterations */
    int precision;       /* TS_F64, TS_F32 (FP32 cycles + FP64 refinement) or
                            TS_F16W (FP16 weight evaluation + refinement) */
    double rtol;         /* stop when ||f - L u||_2 <= rtol ||f||_2 (free rows) */
    int diverge_window;  /* stop with TS_ENOCONV after this many consecutive
                            residual increases (0: default 3) */
    int dd;              /* non-zero: double discretisation (Sec. 4 introduction).  The
                            smoothing sweeps use the operator's surrogate
                            stencils, every residual of the cycle the exact
                            element-wise (IFEM) rows; the two operators
                            compete, so the solve stops on the update instead,
                            ||u_c - u_(c-1)||_2 <= rtol ||u_c||_2 (free rows).
                            TS_F64 precision only (TS_EINVAL otherwise);
                            IFEM rows limit it to level 8 */
} ts_solve_params;

#define TS_MAX_HIST 256
typedef struct {
    int cycles;          /* outer iterations done */
    int status;          /* TS_OK, TS_ENOCONV or TS_ENONFINITE */
    double rel_residual; /* final ||f - L u|| / ||f|| in FP64; with dd the
                            last relative update */
    int n_hist;
    double hist[TS_MAX_HIST]; /* relative residual before each iteration and at
                                 the end; with dd the relative update of each
                                 cycle */
} ts_solve_info;

const char *ts_last_error(void);

/* ---- mesh (Sec. 2.2: macro mesh T_-2, blending map Phi) -----------------
 * vtx: nv x 3 host doubles; tet: nt x 4 host int64 vertex ids (copied).  The
 * vertex order of each macro is its (i, j, k) frame.  geom: TS_GEOM_SHELL
 * maps every fine node radially, x = rho(y) y/|y| with y the affine point and
 * rho the barycentric blend of the vertex radii (nodes of interior macros
 * form spherical layers); TS_GEOM_AFFINE keeps x = y (Phi = Id).  Fails with
 * TS_EINVAL if a face is shared by more than two macros, an id is out of
 * range or a macro is degenerate (the volume spanned by its edges from
 * vertex 0 at most 1e-12 times the cube of the longest of them). */
int ts_mesh_create(const double *vtx, int64_t nv, const int64_t *tet, int64_t nt, int geom,
                   ts_mesh **out);
int ts_mesh_destroy(ts_mesh *mesh);
/* Check that the mesh is a shell r_in <= |x| <= r_out (Sec. 2.1: the domain
 * of the model problem, whose boundary is the two spheres): every vertex
 * lies within [r_in - tol, r_out + tol], and every face of the mesh boundary
 * (a face of one macro only) has its three vertices on the same sphere,
 * | |v| - r | <= tol for r = r_in or r = r_out.  Host only, no device work.
 * TS_EINVAL with the first offending vertex or face in ts_last_error().
 * ts_mesh_create does not require it (TS_GEOM_AFFINE meshes need not be
 * shells). */
int ts_mesh_check_shell(const ts_mesh *mesh, double r_in, double r_out, double tol);
/* A mesh with the connectivity of `like` and its own vertex coordinates (vtx:
 * nv x 3 host doubles, copied).  The levels already built on `like` (index
 * lists, tiles, lane orders: everything that depends on the connectivity
 * only) are shared, not rebuilt; everything that depends on the coordinates
 * is the new mesh's own (Sec. 2.2: the blending map depends on the vertices
 * only).  Levels built later are built per mesh.  `like` may be destroyed
 * before the new mesh.  Building levels on `like` while this call runs is
 * not allowed.  TS_EINVAL if a macro is degenerate. */
int ts_mesh_create_like(const ts_mesh *like, const double *vtx, ts_mesh **out);
/* Replace the vertex coordinates (vtx: nv x 3 host doubles, copied) of a mesh
 * and keep its connectivity and every level built on it (interface lists,
 * tiles, lane orders), so that a caller solving many problems on one macro
 * layout with different radii builds the levels once (Sec. 2.2: the blending
 * map depends on the vertices only).  Stored coordinates and stored interface
 * stencils are recomputed on next use.  Fails with TS_EINVAL while an
 * operator created on the mesh is alive (its coefficients describe the old
 * geometry) or if a macro becomes degenerate (the mesh is then unchanged);
 * no work that reads the mesh may be in flight. */
int ts_mesh_set_vertices(ts_mesh *mesh, const double *vtx);
int ts_layout(ts_mesh *mesh, int level, ts_layout_info *out);

/* Layout helpers (Sec. 2.3: the nodes of a refined macro and their
 * primitives; the canonical order numbers each unique node once).
 * canonical <-> block conversions of float64 device vectors.  to_block zeroes
 * Dirichlet slots; to_canon reads the first copy of every node. */
int ts_canon_to_block(ts_mesh *mesh, int level, const double *canon, double *block,
                      ts_stream s);
int ts_block_to_canon(ts_mesh *mesh, int level, const double *block, double *canon,
                      ts_stream s);
/* blended coordinates of every block slot (Sec. 2.2: x = Phi_T(Psi_T(.)) of
 * the fine node): xyz is 3 * vec_len doubles (slot-major, x y z). */
int ts_node_coords(ts_mesh *mesh, int level, double *xyz, ts_stream s);

/* Load vector f_l = M_l I_l f (Sec. 2.2 eq. algebraic with the consistent P1
 * mass matrix of the mapped fine tetrahedra applied to the nodal
 * interpolant of f), float64 block vector, Dirichlet slots 0.
 *   TS_RHS_MANUFACTURED: f = -Laplace(sin(pi (r - r1)/(r2 - r1)) x y z),
 *       params = {r1, r2};
 *   TS_RHS_BUMPS: sum of Gaussians a exp(-|x - c|^2 / (2 s^2)), params =
 *       records (cx, cy, cz, s, a);
 *   TS_RHS_ONE: f = 1.
 * f is evaluated once per block slot into a temporary of one block vector
 * (allocated and freed in stream order on s, TS_ENOMEM if it does not fit);
 * the call returns once f is written. */
int ts_rhs(ts_mesh *mesh, int level, int kind, const double *params, int nparams, double *f,
           ts_stream s);

/* ---- operator (Sec. 3: IPOLY / LSQP surrogate; Sec. 2.3: IFEM) ----------
 * Builds the surrogate coefficients of every macro on levels 3..max_level on
 * the device: exact stencils at the sampling points (Sec. 3.1 for IPOLY, eq.
 * samplingSetFunctions for LSQP), then the FP64 normal equations
 * (A^T A) a = A^T b with one Cholesky factor per level (the matrix A is the
 * same for all macros).  Basis: monomials xi^l eta^m zeta^n with
 * xi = i/N - 1/4 (same for j, k), degree <= q, ordered by degree, then l
 * descending, then m descending.  The mesh must outlive the operator. */
int ts_op_create(ts_mesh *mesh, int max_level, const ts_op_params *p, ts_stream s,
                 ts_op **out);
int ts_op_destroy(ts_op *op);
/* coefficients of one level: n_macros x 15 x m_q host doubles (stencil
 * direction order mc mw me ms mn mse mnw bc be bn bnw tc tw ts tse);
 * synchronous.  Import replaces them (checkpoint / shared coefficients). */
int ts_op_coeffs_export(ts_op *op, int level, double *host, size_t n);
int ts_op_coeffs_import(ts_op *op, int level, const double *host, size_t n);
/* per-macro flags of one level (1: IFEM volume rows, selective surrogate);
   n_macros host bytes, synchronous */
int ts_op_macro_flags(ts_op *op, int level, unsigned char *host, size_t n);

/* y = L x (Sec. 3.4 eq. ts): volume rows from the surrogate (IFEM rows for a
 * TS_IFEM operator or on level 2), lower-primitive rows by element-wise
 * assembly over all adjacent macros; Dirichlet rows 0. */
int ts_apply(ts_op *op, int level, int dtype, const void *x, void *y, ts_stream s);
/* the volume rows only (interior nodes of every macro); other slots of y
 * are left untouched */
int ts_apply_volume(ts_op *op, int level, int dtype, const void *x, void *y, ts_stream s);
/* r = f - L u */
int ts_residual(ts_op *op, int level, int dtype, const void *f, const void *u, void *r,
                ts_stream s);
/* multicolour Gauss-Seidel (eq. iteration-scheme), in place: per sweep the
 * phases vertices; edge points by a mod 2; face points by (a + 2b) mod 3;
 * volume points by (i + 2j + 3k) mod 4.  Inside a phase every point is
 * updated from the values at the start of the phase. */
int ts_smooth(ts_op *op, int level, int dtype, const void *f, void *u, int sweeps,
              ts_stream s);
/* grid transfer between level and level - 1: linear interpolation in index
 * space P and its transpose R = P^T (Dirichlet rows 0). */
int ts_restrict(ts_op *op, int level, int dtype, const void *rf, void *rc, ts_stream s);
int ts_prolongate_add(ts_op *op, int level, int dtype, const void *uc, void *uf, ts_stream s);
/* sqrt(sum over free nodes of x^2), each node once: the Euclidean norm of
 * the coefficient vector in the stopping test of the solver (Sec. 4
 * introduction: relative residual); synchronous, deterministic (fixed
 * reduction order). */
int ts_norm2(ts_mesh *mesh, int level, int dtype, const void *x, double *out, ts_stream s);

/* ts_norm2 without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same kernels and reduction order as ts_norm2, so
 * the same bits; the norm is written to the device double *out (caller's
 * memory) asynchronously on s, and nothing is synchronised or copied to the
 * host.  The partial sums go to a fixed device array of the library (8 MiB
 * per GPU, kept until the process ends): TS_EINVAL if the level needs more
 * than its 2^20 partial sums (a message gives both counts), if the level has
 * not been built on the mesh yet (ts_layout builds it), or if the mesh's
 * device is not the current one.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (two streams, two threads) race and
 * must be ordered by the caller.  No entry of the array needs clearing: each
 * call writes every entry it reads. */
int ts_norm2_noalloc(ts_mesh *mesh, int level, int dtype, const void *x, double *out,
                     ts_stream s);

/* ---- multigrid (Sec. 4 introduction: V(3,3) with Gauss-Seidel smoothing) --
 * Coarsest level 2 is solved exactly in FP64 with the inverse of its IFEM
 * matrix (computed on the device at creation).  Workspace owned by the
 * solver, all of it allocated by ts_solver_create (per-level cycle vectors of
 * the solve's precision, the outer residual and correction, stored interface
 * rows).  TS_EINVAL above level 8 if the solve would need element-wise
 * volume rows there (dd, a TS_IFEM operator, or macros the selective
 * surrogate keeps exact). */
int ts_solver_create(ts_op *op, int level, const ts_solve_params *p, ts_solver **out);
int ts_solver_destroy(ts_solver *sv);
/* Moves a solver, its operator and its mesh to new vertex coordinates of the
 * same connectivity (vtx: nv x 3 host doubles, copied), as if all three had
 * been created anew for them: the blending geometry (Sec. 2.2), the
 * surrogate fits, per-macro fallback flags and face fits of every level of
 * the operator (Sec. 3), the stored interface rows and the coarse inverse
 * are rebuilt on s, in the device buffers they have (a buffer is replaced
 * only where a length changes, e.g. when macros switch between surrogate
 * and element-wise volume rows).  For request loops that keep solvers
 * resident and reuse them for problems on differently scaled shells.
 * Synchronous.  The mesh must carry this operator only (TS_EINVAL
 * otherwise), and no solve of the solver may be in progress (ts_solve_begin
 * without TS_SOLVE_DONE: TS_EINVAL).  Non-finite coordinates: TS_ENONFINITE
 * with nothing changed.  After any other failure the objects are in an
 * undefined state and must be destroyed. */
int ts_solver_set_vertices(ts_solver *sv, const double *vtx, ts_stream s);
/* one V(nu1, nu2) cycle on L u = f at the solver's level, in place */
int ts_vcycle(ts_solver *sv, int dtype, const void *f, void *u, ts_stream s);
/* full solve: u (float64, initial guess on entry) until the FP64 relative
 * residual <= rtol.  TS_F32 / TS_F16W precision: FP64 residual, FP32 V-cycle
 * on the correction, FP64 update (iterative refinement).  Synchronous once
 * per iteration (residual norm).  Returns TS_ENOCONV / TS_ENONFINITE with
 * info filled when it stops early. */
int ts_solve(ts_solver *sv, const double *f, double *u, ts_solve_info *info, ts_stream s);

/* ---- asynchronous solve (request loops, continuous batching) ------------
 * The same outer iteration as ts_solve, split so that a host loop can keep
 * many solves in flight on their own streams and advance each when its last
 * step has finished, without blocking:
 *   ts_solve_begin enqueues ||f|| and the first residual on s and returns;
 *   ts_solve_query never blocks and sets *state to TS_SOLVE_RUNNING (work in
 *     flight), TS_SOLVE_READY (call ts_solve_step next) or TS_SOLVE_DONE
 *     (info->status is final: TS_OK, TS_ENOCONV or TS_ENONFINITE); info
 *     (optional) gets the history so far;
 *   ts_solve_step enqueues one outer iteration on the stream given to
 *     ts_solve_begin (TS_EINVAL unless the state is TS_SOLVE_READY).  A step
 *     allocates nothing (ts_solver_create allocated every vector it uses);
 *     if enqueuing fails part-way (TS_EHIP) the solve ends: TS_SOLVE_DONE
 *     with info.status set to the error code.
 * f and u are the caller's device vectors and must stay valid until DONE; u
 * holds the initial guess.  Results are bitwise identical to ts_solve with
 * the same inputs.  One host thread at a time per solver (and per mesh). */
enum { TS_SOLVE_RUNNING = 1, TS_SOLVE_READY = 2, TS_SOLVE_DONE = 3 };
int ts_solve_begin(ts_solver *sv, const double *f, double *u, ts_stream s);
int ts_solve_step(ts_solver *sv);
int ts_solve_query(ts_solver *sv, int *state, ts_solve_info *info);
/* The batched step of a request loop: one outer iteration on each of the n
 * distinct solvers v[0..n-1], enqueued in the order given (the loop's
 * priority order).  Every solver must be TS_SOLVE_READY as ts_solve_query
 * last reported it (as for ts_solve_step); otherwise nothing is enqueued and
 * TS_EINVAL is returned.  Each solver's launches go to its
 * own stream: requests carry their own meshes and coefficients, so no
 * launch spans two of them, and the hardware queues overlap the streams.
 * A HIP error part-way returns TS_EHIP with the solvers before the failing
 * one stepped (their state is then TS_SOLVE_RUNNING); the failing solver's
 * solve ends (TS_SOLVE_DONE, info.status = the error code, u holds a partly
 * applied cycle) and the solvers after it are not stepped.  n = 0 is a
 * no-op. */
int ts_solve_batch_step(ts_solver *const *v, int n);

/* device memory currently held by all meshes, operators and solvers of the
 * process (bytes; excludes the caller's vectors) */
int ts_device_bytes(int64_t *bytes);

#ifdef __cplusplus
}
#endif

#endif /* TWOSCALE_H */
