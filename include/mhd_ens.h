/*
 * mhd_ens.h -- C ABI of the MI355X ensemble MHD time-step library (libmhd_ens.so).
 *
 * The library computes one time step of the decoupled ensemble scheme for the
 * Elsasser variables v = u + sqrt(s) B, w = u - sqrt(s) B (paper, Section 1,
 * (els1)-(els3)), fully discretised as Algorithm 1 of Section 3 ((weaknew1),
 * (weaknew2)) with Taylor-Hood P2-P1 elements on structured triangulations,
 * or Scott-Vogelius elements (P2, discontinuous P1) on their barycentric
 * refinement (mhd_mesh_desc.element).
 * In each step the v-subproblem and the w-subproblem have ONE coefficient
 * matrix shared by all J members (Section 1: A [x_1|...|x_J] = [b_1|...|b_J]),
 * assembled from the ensemble mean of the other variable, the mean
 * viscosities and the mixing-length eddy viscosity nu_T = mu dt l^2,
 * l(x) = max_j |z_j'(x)|; the J right-hand sides carry each member's explicit
 * fluctuation terms.
 *
 * Conventions for every call:
 *  - Return value: mhd_status.  MHD_OK on success; on failure a message is
 *    available from mhd_ens_last_error() (thread-local).  Argument checks
 *    happen on the host before any device work is enqueued.
 *  - Device arrays are plain device pointers (hipMalloc'd or from a tensor
 *    allocator) owned by the caller; they must stay valid until the work
 *    enqueued on the given stream has completed.  Host arrays are marked
 *    "host".  Opaque handles are owned by the library and freed by their
 *    *_free call.
 *  - Member blocks are row-major with the member index fastest:
 *      vector P2 field  (nP2, 2, J):  z[(i*2 + c)*J + j]
 *      scalar P1 field  (nP1, J):     p[k*J + j]
 *      unknown block    (n, J):       velocity rows 2*i + c (i P2 node,
 *                                     c component) then pressure rows
 *                                     2*nP2 + k, n = 2 nP2 + nP1.
 *  - Node numbering (Taylor-Hood; Scott-Vogelius meshes: see mhd_mesh_desc):
 *    P2 nodes are the points of the (2 nx + 1) x (2 ny + 1) half-step grid of
 *    the cell grid that belong to a kept cell, in row-major order (y
 *    slowest); P1 nodes are the vertices (even half-step grid points) in the
 *    same order.  mhd_ens_mesh_coords returns the coordinates.
 *  - All device work is asynchronous on the caller's stream (0 = the null
 *    stream).  Calls that fill host statistics synchronise that stream.
 *  - Device memory is allocated only by the create calls (mhd_ens_mesh,
 *    mhd_ens_shared_create, mhd_ens_ctx_create, mhd_ens_group_create) and by
 *    the explicit tuning calls (mhd_ens_prepare, mhd_ens_ctx_prepare,
 *    mhd_ens_autotune, mhd_ens_set_plan), which build the data of the kernel
 *    plans they choose.  Solves, steps, assemblies and SpMMs never allocate
 *    (mhd_ens_alloc_stats counts the library's allocations; HIP graph
 *    instantiation by mhd_ens_step in graph mode is the runtime's own).
 *    Context creation prepares the plans for J_max; a solve or step with a J
 *    no tuning call prepared runs the default kernel plans (same results).
 */
#ifndef MHD_ENS_H
#define MHD_ENS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int mhd_status;
#define MHD_OK        0
#define MHD_EINVAL   (-1)   /* invalid argument (null pointer, bad size, bad enum)   */
#define MHD_ENOMEM   (-2)   /* device or host allocation failed                      */
#define MHD_EHIP     (-3)   /* a HIP runtime call failed (message names it)          */
#define MHD_ENOCONV  (-4)   /* solver hit maxit: best iterate written, stats filled  */
#define MHD_ESHAPE   (-5)   /* J larger than the handle was created for, or mesh mismatch */

typedef enum { MHD_FP64 = 0, MHD_FP32_IR = 1 } mhd_precision;
typedef enum { MHD_MESH_UNIT_SQUARE = 0, MHD_MESH_STEP_CHANNEL = 1 } mhd_mesh_kind;
typedef enum { MHD_ELEMENT_TAYLOR_HOOD = 0, MHD_ELEMENT_SCOTT_VOGELIUS = 1 } mhd_element;
typedef enum { MHD_V_PROBLEM = 0, MHD_W_PROBLEM = 1 } mhd_which;

typedef void* mhd_stream_t;            /* a hipStream_t */
typedef struct mhd_mesh_s*   mhd_mesh;
typedef struct mhd_shared_s* mhd_shared;
typedef struct mhd_ctx_s*    mhd_ctx;

/* Mesh description (paper, Section 4: regular triangulations; every square
 * cell is cut by its rising diagonal).
 *   MHD_MESH_UNIT_SQUARE: [0,1]^2 with nx = ny = N cells per side.
 *   MHD_MESH_STEP_CHANNEL: [0,30]x[0,10] minus [0,1]x[0,1], h = 1/m with
 *     nx = m (cells per unit length); outflow x = 30.
 * natural_outflow: 1 = do-nothing condition on x = 30 (step channel only),
 *   0 = Dirichlet on the whole boundary.  With a fully Dirichlet boundary the
 *   pressure is pinned (identity row) because it is determined only up to a
 *   constant (Section 2, Q = L^2_0): Taylor-Hood at the vertex (0,0) (the
 *   first vertex), Scott-Vogelius at pressure unknown 0.
 * element (Section 2: any inf-sup stable pair; the experiments of Section 4
 *   use Scott-Vogelius):
 *   MHD_ELEMENT_TAYLOR_HOOD: continuous P2 velocity, continuous P1 pressure
 *     on the triangulation above.
 *   MHD_ELEMENT_SCOTT_VOGELIUS: continuous P2 velocity, discontinuous P1
 *     pressure on its barycentric (Alfeld) refinement: each triangle
 *     (p0, p1, p2) with barycentre g (cells in row-major order, lower
 *     (v00, v10, v11) before upper (v00, v11, v01)) becomes the elements
 *     (p0, p1, g), (p1, p2, g), (p2, p0, g).  P2 nodes are the points of the
 *     (6 nx + 1) x (6 ny + 1) grid of sixth steps used by some element, in
 *     row-major order; pressure unknown 3 e + k belongs to vertex k of
 *     element e (nP1 = 3 n_el).  The velocity divergence then lies in the
 *     pressure space, so discrete solutions are divergence-free pointwise.
 *     Kernel plans with row tiles (tile != 0) are defined for Taylor-Hood
 *     meshes only (MHD_EINVAL). */
typedef struct {
    int kind;
    int nx;
    int natural_outflow;
    int element;
} mhd_mesh_desc;

typedef struct {
    int64_t n_el, nP2, nP1, n_u, n;     /* n_u = 2 nP2, n = n_u + nP1            */
    int64_t nnz_A, nnz_B;               /* scalar P2-P2 pattern, P1-P2 pattern   */
    int64_t nnz;                        /* nonzeros of the full saddle-point CSR */
    int64_t n_bd, n_dir;                /* boundary P2 nodes, Dirichlet P2 nodes */
    int32_t pin;                        /* pinned pressure node, -1 if none      */
    int32_t mg_levels;                  /* pressure multigrid levels             */
} mhd_mesh_info;

/* Host-only: counts of a mesh without creating it (no device needed). */
mhd_status mhd_ens_mesh_counts(const mhd_mesh_desc* d, mhd_mesh_info* info);

/* Builds the mesh, the CSR patterns of the saddle-point operator, the
 * element-to-slot maps and the pressure multigrid hierarchy, and uploads
 * them to the current device.  info (host) may be NULL. */
mhd_status mhd_ens_mesh(const mhd_mesh_desc* d, mhd_mesh* out, mhd_mesh_info* info);

/* (Section 4: the problem data -- initial values, forcing f_{1,j}, f_{2,j},
 * boundary values -- are given as functions of x and enter the scheme as
 * their values at the P2 nodes.)  Host copies of what a caller needs to
 * evaluate them: xy_p2 (nP2*2 doubles, may be NULL), dir_nodes (n_dir int32:
 * the Dirichlet P2 nodes in the order bc arrays use, may be NULL). */
mhd_status mhd_ens_mesh_coords(mhd_mesh m, double* xy_p2, int32_t* dir_nodes);

/* (Section 2: the finite element spaces are defined element by element.)
 * Host copy of the element connectivity, tri (host, n_el*6 int32): the P2
 * nodes of element e are tri[6e..6e+5] in the order (v0, v1, v2, m01, m12,
 * m20), vertices counter-clockwise, m_ab the midpoint of edge ab.  The
 * pressure unknowns of element e are vertex ids of the unrefined grid
 * (Taylor-Hood, P1 numbering) or 3e, 3e+1, 3e+2 (Scott-Vogelius). */
mhd_status mhd_ens_mesh_elements(mhd_mesh m, int32_t* tri);

/* Releases a mesh and everything mhd_ens_mesh built for it (Section 2's
 * finite element spaces on that triangulation).  Handles created from it
 * must be freed first.  NULL is accepted. */
mhd_status mhd_ens_mesh_free(mhd_mesh m);

/* Coefficients of one subproblem (Algorithm 1): time step dt, eddy tuning
 * mu (nu_T = mu dt l^2), mean viscosity nu_bar and diffusivity num_bar
 * ((nu_bar + num_bar)/2 multiplies the implicit Laplacian), convective form:
 * 0 = skew-symmetric b*(u,v,w) = (b(u,v,w) - b(u,w,v))/2, 1 = b(u,v,w) as
 * written in Section 2. */
typedef struct {
    double dt, mu, nu_bar, num_bar;
    int convective;
} mhd_coeffs;

/* Shared-matrix handle: the CSR values of one subproblem's saddle-point
 * matrix S = [[A (x) I_2, B^T], [B, D_p]] (FP64 master + FP32 shadow) and the
 * solver workspace for up to J_max right-hand sides and a Krylov restart
 * length `restart`. */
mhd_status mhd_ens_shared_create(mhd_mesh m, int J_max, int restart, mhd_shared* out);
mhd_status mhd_ens_shared_free(mhd_shared A);

/* (Algorithm 1, left-hand sides of (weaknew1)/(weaknew2)) Assembles
 *   A = M/dt + b*(<z>, ., .) + (nu_bar+num_bar)/2 K + K[2 mu dt l_z^2]
 * from the OTHER variable's members z_other (device, (nP2,2,J) FP64):
 * computes the ensemble mean <z> and l_z^2 = max_j |z_j - <z>|^2 at the 7
 * quadrature points of every element, then the element matrices, gathered
 * into the CSR values deterministically (no atomics).  Dirichlet rows
 * become identity rows; the pinned pressure row becomes an identity row. */
mhd_status mhd_ens_assemble_shared(mhd_mesh m, const mhd_coeffs* c, const double* z_other,
                                   int J, mhd_shared A, mhd_stream_t s);

/* (Algorithm 1, the one left-hand side of each subproblem; Section 2's mixed
 * form with the divergence constraint) Borrowed device views of the
 * assembled operator (valid until the next assemble or free).  Scalar P2 block A: rowptr_A (nP2+1), col_A (nnz_A),
 * val_A (nnz_A, FP64).  B^T: rowptr_Bt (nP2+1), col_Bt (P1 ids), val_Bt
 * (2 per entry: x then y component).  B: rowptr_B (nP1+1), col_B (P2 ids),
 * val_B (2 per entry).  D_p: (nP1) pressure diagonal (1 at the pin, else 0). */
typedef struct {
    const int32_t *rowptr_A, *col_A, *rowptr_Bt, *col_Bt, *rowptr_B, *col_B;
    const double *val_A, *val_Bt, *val_B, *diag_p;
    const float* val_A32;
    int64_t nP2, nP1, nnz_A, nnz_Bt, nnz_B;
} mhd_csr_view;
mhd_status mhd_ens_shared_csr(mhd_shared A, mhd_csr_view* view);

/* (Algorithm 1, right-hand sides of (weaknew1)/(weaknew2)) For which =
 * MHD_V_PROBLEM (self = v, other = w, forcing f_1) or MHD_W_PROBLEM
 * (self = w, other = v, forcing f_2), for every member j:
 *   b_j = M (self_j/dt + f_j) - b*(other_j - <other>, self_j, .)
 *         - (nu_j - num_j)/2 K other_j - (nu_j' + num_j')/2 K self_j
 * on velocity rows; Dirichlet rows take bc_vals; pressure rows 0.
 *   self_n, other_n: device (nP2,2,J) FP64 at t^n
 *   nu, nu_m:        device (J) FP64 member viscosities / diffusivities
 *   forcing:         device (nP2,2,J) FP64 nodal f at t^{n+1}, or NULL (= 0)
 *   bc_vals:         device (n_dir,2,J) FP64 Dirichlet values at t^{n+1},
 *                    in mhd_ens_mesh_coords' dir_nodes order
 *   rhs:             device (n,J) output, every row written: double for
 *                    precision MHD_FP64, float for MHD_FP32_IR (the same
 *                    FP64 arithmetic, rounded once when stored)
 * The forcing functional (f, chi) is taken as M times the nodal interpolant.
 * One kernel pass over the elements (no element buffer), deterministic. */
mhd_status mhd_ens_assemble_rhs(mhd_mesh m, const mhd_coeffs* c, int which, int J,
                                const double* self_n, const double* other_n,
                                const double* nu, const double* nu_m,
                                const double* forcing, const double* bc_vals,
                                void* rhs, int precision, mhd_stream_t s);

/* For callers that cannot allocate device memory (code under the caller's own
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * right-hand sides as mhd_ens_assemble_rhs, same arguments, bitwise the same
 * result, but the scratch it needs (2 J member coefficients and the 2 nP2
 * values of the other variable's ensemble mean, 256-byte aligned) lives in a
 * fixed 32 MiB device array of the library instead of the mesh handle.  The
 * call allocates nothing.  Each GPU holds its own copy of that array for the
 * life of the process; calls on one GPU share it and it keeps the last call's
 * contents (every value is written before it is read), so calls that overlap
 * on one GPU (concurrent streams or threads) race.  MHD_ESHAPE if
 * 2 J (rounded up to 32) + 2 nP2 exceeds 4,194,304 doubles, i.e. nP2 above
 * 2,093,056 at J = 4096. */
mhd_status mhd_ens_assemble_rhs_noalloc(mhd_mesh m, const mhd_coeffs* c, int which, int J,
                                        const double* self_n, const double* other_n,
                                        const double* nu, const double* nu_m,
                                        const double* forcing, const double* bc_vals,
                                        void* rhs, int precision, mhd_stream_t s);

/* Solver options.  precision: MHD_FP64 (all Krylov work in FP64) or
 * MHD_FP32_IR (FP32 SpMM/preconditioner/Krylov vectors inside FP64 iterative
 * refinement: r = b - S x in FP64, S d = r in FP32, x += d).  rtol: target
 * per member ||b_j - S x_j||_2 / ||b_j||_2.  inner_rtol: reduction asked of
 * each inner Krylov cycle.  maxit: total inner iterations.  restart: Krylov
 * length per cycle (<= the handle's restart). */
typedef struct {
    int precision;
    double rtol;
    double inner_rtol;
    int maxit;
    int restart;
    int jacobi_sweeps;        /* velocity-block smoothing sweeps in the preconditioner */
    int check_every;          /* inner iterations between convergence checks (>= 1)    */
    int cgs_passes;           /* classical Gram-Schmidt: 1 or 2 passes with the new
                                 vector's norm taken directly; 3 = one pass with the
                                 norm from the dot products (|w|^2 - |h|^2) and the
                                 vector stored normalised in the same update (fewer
                                 launches; in FP32 the difference cancels once the
                                 vector nearly lies in the basis's span, which is
                                 counted in mhd_solve_stats.norm_clamps); 0 = 1 for
                                 FP32 inner solves, 2 for FP64                        */
    int fixed_cycles;         /* > 0: fixed schedule of fixed_cycles refinement cycles of
                                 `restart` inner iterations each, with no host
                                 synchronisation (graph-capturable); rtol, inner_rtol,
                                 maxit and check_every are then ignored and the stats
                                 report max_relres = -1, converged = -1              */
    double jacobi_omega;      /* damping of the velocity-block Jacobi sweeps, in (0, 1.5];
                                 0 = the default 0.6.  A developed flow makes the spectrum
                                 of D^-1 A complex, and damping 0.85 then diverges; 0.6
                                 with two V-cycles (mg_cycles) stays convergent         */
    int mg_unfused;           /* 0 (default): on each multigrid level above the coarsest
                                 the residual and its restriction run as one precomputed
                                 sparse operator, and so do the prolongation and the first
                                 post-smoothing sweep (4 launches per level instead of 6);
                                 1: one kernel per sweep, residual and transfer (the same
                                 arithmetic up to rounding)                              */
    int mg_cycles;            /* V-cycles per application of the Schur part: 0 or 1 = one,
                                 2 = two (the second on the first one's residual), a
                                 closer approximation of (B D^-1 B^T)^-1 for flows where
                                 the outer iteration is sensitive to it                */
    int block_krylov;         /* 1: block GMRES, one Krylov space shared by the J columns
                                 (block Gram-Schmidt with a second pass, pivoted Cholesky
                                 QR of each new block that deflates dependent directions,
                                 block least squares on the host); adaptive schedule only,
                                 J in {16, 32, 64, 128}.  0 (default): one Arnoldi process
                                 per member over the shared SpMM                        */
    int mg_post;              /* extra damped Jacobi post-smoothing sweeps on the finest
                                 pressure level of each V-cycle (0 to 8; default 0)    */
    int keep_converged;       /* adaptive schedule, per-member solver: 0 (default) = once
                                 some members meet rtol at a refinement cycle, the
                                 others continue as a compacted block of fewer columns
                                 (every kernel then streams only those), the converged
                                 iterates are left as they are; 1 = all J columns stay
                                 in every cycle                                        */
} mhd_solver_opts;

typedef struct {
    int iters;                /* total inner Krylov iterations                        */
    int cycles;               /* outer refinement / restart cycles                    */
    double max_relres;        /* max over members of the final relative residual
                                 ||b_j - S x_j||_2 / ||b_j||_2 (NaN if a residual is not
                                 finite); with a fixed schedule computed after the solve
                                 when stats are requested                              */
    int converged;            /* 1 if every member reached rtol, 0 if not, -1 for a
                                 fixed schedule (no target)                            */
    int nonfinite;            /* members whose final residual is NaN or Inf (the call
                                 then returns MHD_ENOCONV)                              */
    double* relres;           /* host (J) or NULL, set by the caller: each member's final
                                 relative residual                                     */
    int32_t* member_iters;    /* host (J) or NULL, set by the caller: inner iterations
                                 after which member j's residual first met rtol (all
                                 members run one shared Krylov schedule, so the total
                                 if never, and the total for a fixed schedule)         */
    int min_block_rank;       /* block GMRES: the smallest rank of a basis block after
                                 deflation; J for the per-member solver                */
    int norm_clamps;          /* cgs_passes = 3: new basis vectors of nonzero w whose
                                 |w|^2 - |h|^2 was not positive, so that their norm was
                                 taken as 0 (the member's cycle ends there), summed over
                                 members and iterations of the call (-1: not read back) */
    int compacted;            /* adaptive per-member solver: the number of members that
                                 continued as a compacted block once the others had met
                                 rtol (0: no compaction)                                */
} mhd_solve_stats;

/* (Section 1: A [x_1|...|x_J] = [b_1|...|b_J]) Solves S X = B for the J
 * member columns with the assembled shared matrix: right-preconditioned
 * restarted GMRES with one Arnoldi process per member, one SpMM over all J
 * columns per iteration, block-triangular preconditioner (damped Jacobi
 * sweeps on A; Schur complement approximated by B D^-1 B^T, D the diagonal of
 * M/dt + nu_c K, inverted by a Galerkin multigrid V-cycle on the nested P1
 * grids).  rhs (n,J) FP64 device; x (n,J) FP64 device: initial
 * guess in, solution out.  st (host) may be NULL; if non-NULL the stream is
 * synchronised (with a fixed schedule the final residuals are then computed,
 * outside graph capture).  Returns MHD_ENOCONV (x = best iterate) if maxit is
 * hit or a residual is not finite.  Allocates nothing and tunes nothing: the
 * node-row kernels run the plans mhd_ens_prepare chose for this J. */
mhd_status mhd_ens_solve(mhd_shared A, const double* rhs, double* x, int J,
                         const mhd_solver_opts* o, mhd_solve_stats* st, mhd_stream_t s);

/* Full-step context: owns both subproblems' shared matrices, right-hand
 * sides and solver workspace for up to J_max members. */
typedef struct {
    mhd_coeffs coeffs;        /* nu_bar/num_bar are recomputed from nu, nu_m each step */
    mhd_solver_opts solver;
    int J_max;
    int adjoint;              /* 1: also allocate the adjoint-step workspace */
    int graph;                /* 1: capture the step's device work into a HIP graph on the
                                 first call (per argument set and stream) and replay it
                                 afterwards; needs solver.fixed_cycles > 0 and a non-null
                                 stream */
    int serial;               /* 0 (default): with a fixed schedule the w-subproblem runs on
                                 a second stream of the context, concurrently with the
                                 v-subproblem (both read time level n only); 1: both on the
                                 caller's stream, one after the other */
} mhd_ctx_desc;
mhd_status mhd_ens_ctx_create(mhd_mesh m, const mhd_ctx_desc* d, mhd_ctx* out);
mhd_status mhd_ens_ctx_free(mhd_ctx ctx);

typedef struct {
    const double *nu, *nu_m;      /* host (J) member parameters (read at call time)        */
    const double *f1, *f2;        /* device (nP2,2,J) forcing at t^{n+1}, or NULL          */
    const double *g_v, *g_w;      /* device (n_dir,2,J) Dirichlet data at t^{n+1}          */
    int J;
} mhd_step_inputs;

/* Warning bits of a step (Section 3.1: the stability and convergence theorems
 * assume alpha_j = nu_bar + num_bar - |nu_j - nu_m,j| - |nu_j' + nu_m,j'| > 0
 * for every member and mu > 1/2; the scheme still runs without them). */
#define MHD_WARN_ALPHA      1   /* some alpha_j <= 0                                   */
#define MHD_WARN_MU         2   /* mu <= 1/2                                           */
#define MHD_WARN_NONFINITE  4   /* a final residual is NaN or Inf (step returns ENOCONV) */

typedef struct {
    mhd_solve_stats v, w;         /* per subproblem; set v.relres etc. for per-member arrays */
    double energy;                /* E_h^{n+1} = (||<v>||^2 + ||<w>||^2)/2 (Section 4.2)   */
    int warnings;                 /* MHD_WARN_* bits                                       */
    double min_alpha;             /* min_j alpha_j of this step's parameters               */
} mhd_step_stats;

/* (Algorithm 1, one step n -> n+1 for all members) V, W: device (nP2,2,J)
 * FP64, in: t^n, out: t^{n+1}.  Q, R: device (nP1,J) FP64, in: pressure of
 * t^n (initial guess), out: pressures of t^{n+1} (zero mean when the pressure
 * is pinned).  st (host) may be NULL (then no synchronisation); if non-NULL
 * the stream is synchronised and, with a fixed schedule, the final residuals
 * of both subproblems are computed.  Returns MHD_ENOCONV if a solve hit maxit
 * or a residual is not finite.  Allocates nothing. */
mhd_status mhd_ens_step(mhd_ctx ctx, double* V, double* W, double* Q, double* R,
                        const mhd_step_inputs* in, mhd_step_stats* st, mhd_stream_t s);

/* (Section 1: the shared matrix A applied to [x_1|...|x_J]) y = S x for an
 * (n,J) block with the assembled operator of A: the SpMM the Krylov solver
 * performs once per iteration.  precision MHD_FP64: x, y double; MHD_FP32_IR:
 * x, y float with the FP32 shadow values.  x and y must not overlap. */
mhd_status mhd_ens_spmm(mhd_shared A, const void* x, void* y, int J, int precision, mhd_stream_t s);

/* Kernel autotuner for the node-row operators.  A solve of a given precision
 * launches four such operators per Krylov iteration: the saddle-point SpMM,
 * the first and the following velocity-block Jacobi sweeps of the
 * preconditioner, and the FP64 residual r = b - S x.  For each one the tuner
 * times every candidate launch shape on the handle's own workspace.  It keeps
 * the fastest in a process-wide table keyed by (mesh, J, word size).
 * mhd_ens_prepare and context creation tune missing entries; solves and steps
 * use the table as it stands (or a default plan where this handle lacks a
 * plan's data).  This call re-tunes unconditionally.  Candidates:
 *   gather kernels (each wavefront reads its rows' node values from memory):
 *     vec   = members per lane per load: 1, 2, 4 for FP32 and 1, 2 for FP64,
 *             with J a multiple of 32 vec;
 *     group = units (mesh nodes) per wavefront: 1, 2, 4 with batched gathers,
 *             or 0 for one unit per wavefront with per-entry CSR loads;
 *     deep  = 1: pipelined gathers (group 1, 2, 4 or 8): the next row's
 *             entries load while the current row computes, and all of a
 *             row's member loads are in flight at once (rows of at most 24
 *             entries, B^T rows of at most 8);
 *     deep  = 2: paired rows (group 4 or 8): the two halves of a wavefront
 *             compute two rows at once with 16-byte member loads (J a
 *             multiple of 64 for FP32, 32 for FP64; a row's entries in
 *             chunks of 32); vec is then 16 / word size;
 *   LDS-staged kernels (J a multiple of 32; each workgroup first copies the
 *   node values of a square tile of rows, and its halo, into LDS):
 *     tile  = tile edge in half-steps of the mesh: 8, 12 or 16, where the
 *             staged values fit the device's LDS per workgroup;
 *     waves = wavefronts per workgroup: 4 or 8;
 *     deep  = 3: the tile's CSR entries are staged into LDS as well, so a
 *             row is computed from LDS only (deep = 0: entries by scalar
 *             loads from memory);
 *   row-per-lane tiles (FP32 SpMM and Jacobi sweeps, not the FP64 residual):
 *     deep  = 6: each workgroup stages the values of M members of every node
 *             a rectangle of rows reads, then every lane computes one row,
 *             reading its entries as packed (LDS offset, value) records;
 *     tile  = tx * 100 + ty, the rectangle in half-steps (1616, 3208 or
 *             1608) with M = 16 members per workgroup (J a multiple of 16),
 *             or the same plus 10000 (11616, 13208, 11608) with M = 8 (J a
 *             multiple of 8); vec is reported as 4, group and waves as 0.
 * Every candidate performs the same arithmetic in the same order, so results
 * do not depend on the choice.  Tuning a handle builds the tilings and packed
 * entry arrays of every candidate on first use (device memory held until the
 * mesh or handle is freed); assemblies refresh the A values of the row-per-lane
 * tilings a plan uses.
 *   out:   host array of cap entries, or NULL; receives every timed candidate
 *   count: host, or NULL; receives the number of entries written
 * Synchronises the stream. */
typedef struct {
    int32_t op;               /* MHD_TUNE_*                                   */
    int32_t word;             /* 4 (FP32) or 8 (FP64)                         */
    int32_t J;
    int32_t vec;              /* members per lane                             */
    int32_t group;            /* gather kernels; 0 for LDS-staged entries     */
    int32_t deep;
    int32_t tile;             /* LDS-staged kernels; 0 for gather entries     */
    int32_t waves;
    float us;                 /* mean launch time in microseconds; -1 if the
                                 device refused the launch shape              */
    int32_t chosen;           /* 1 for the plan kept                          */
} mhd_tune_entry;
enum { MHD_TUNE_SADDLE = 0, MHD_TUNE_RESIDUAL = 1, MHD_TUNE_JACOBI_FIRST = 2, MHD_TUNE_JACOBI = 3 };
mhd_status mhd_ens_autotune(mhd_shared A, int J, int precision, mhd_tune_entry* out, int cap, int* count,
                            mhd_stream_t s);

/* Pins the launch plan of one operator (MHD_TUNE_*) for this handle's mesh, J
 * and precision (MHD_TUNE_RESIDUAL is always FP64), replacing the tuned one in
 * the process-wide table, for example to benchmark one shape.
 *   vec, group, deep: the gather kernels as in mhd_ens_autotune; vec = 0
 *               selects the generic kernels (any J);
 *   tile, waves: tile 0, or 8, 12, 16 with waves 4 or 8 for the LDS-staged
 *               kernels, with deep 0 or 3 (where the tiling is not usable,
 *               e.g. an unaligned block, the gather kernels run instead);
 *               with deep 6 a row-per-lane tile code as in mhd_ens_autotune
 *               (FP32 SpMM and Jacobi operators only; waves ignored).
 * Graphs captured earlier keep the kernels they hold.  MHD_EINVAL for a shape
 * this mesh, J or device does not admit.  Builds the tiling on first use
 * (synchronous host-to-device copies). */
mhd_status mhd_ens_set_plan(mhd_shared A, int J, int precision, int op, int vec, int group, int deep, int tile,
                            int waves);

/* The launch plan one operator (MHD_TUNE_*) currently runs with for this
 * handle's mesh, J and precision, in the autotuner's report form: the tuned or
 * pinned table entry (chosen = 1, us = its tuned time or 0 if pinned) or the
 * default plan used when the table has none (chosen = 0, us = -1).  Host only:
 * no device work, no synchronisation.  out: host, one entry. */
mhd_status mhd_ens_get_plan(mhd_shared A, int J, int precision, int op, mhd_tune_entry* out);

/* (Section 1: one matrix for all J members, so its kernels are tuned once per
 * shape) Prepares a shared-matrix handle for solves with J columns in the
 * given precision: tunes the node-row operators whose plans the process-wide
 * table lacks (as mhd_ens_autotune, without re-tuning) and builds this
 * handle's tilings and packed entries for the chosen plans.  Allocates device
 * memory and synchronises the stream; not under graph capture. */
mhd_status mhd_ens_prepare(mhd_shared A, int J, int precision, mhd_stream_t s);

/* mhd_ens_prepare for both subproblem handles of a context, at the context's
 * precision (context creation already did it for J_max). */
mhd_status mhd_ens_ctx_prepare(mhd_ctx ctx, int J, mhd_stream_t s);

/* Diagnostics: number and total bytes of the device allocations this library
 * has made since it was loaded (host, either may be NULL). */
mhd_status mhd_ens_alloc_stats(int64_t* count, int64_t* bytes);

/* Diagnostics: while enabled, every saddle-point SpMM launch of this library
 * (inside mhd_ens_solve / mhd_ens_step and mhd_ens_spmm, outside graph
 * capture) is timed by a pair of HIP events that its dispatch records at the
 * kernel's start and end.  mhd_ens_timer_read synchronises those
 * events and returns the summed kernel milliseconds and the launch count
 * since the last enable; nbytes_fp32 / nbytes_fp64 receive the summed
 * launch sizes (units of n*J) per precision.  Enabling resets the counters. */
mhd_status mhd_ens_timer_enable(int on);
mhd_status mhd_ens_timer_read(double* ms, int64_t* launches, double* nJ_fp32, double* nJ_fp64);
/* Diagnostics: which operator the timer times, MHD_TUNE_SADDLE (the SpMM, the
 * default) or MHD_TUNE_JACOBI (the velocity Jacobi sweeps that update the
 * previous iterate; the first one or two sweeps of each preconditioner
 * application are other kernels); MHD_EINVAL otherwise. */
mhd_status mhd_ens_timer_op(int op);

/* ------------------------------------------------------------------------
 * Discrete adjoint of Algorithm 1 for an ensemble-mean objective.  The
 * context must have been created with desc.adjoint = 1 and the
 * skew-symmetric trilinear form.  Adjoint states are (nP2,2,J) FP64 blocks:
 * lambda_V = dPhi / dV (per member, velocity nodes and components).
 * ---------------------------------------------------------------------- */
typedef struct {
    const double *nu, *nu_m;      /* host (J) member parameters                           */
    const double* fhat;           /* device (nP2,2) forcing shape f_{1,j} = f_{2,j} = a_j fhat,
                                     or NULL (no forcing-amplitude gradient)              */
    int J;
} mhd_adjoint_inputs;

/* (Section 4.2, E_h) Terminal adjoint of Phi = E_h = (||<v>||^2 + ||<w>||^2)/2
 * at the state V, W: lambda_V_j = (1/J) M <v>, lambda_W_j = (1/J) M <w>. */
mhd_status mhd_ens_adjoint_terminal(mhd_ctx ctx, const double* V, const double* W, double* lamV, double* lamW,
                                    int J, mhd_stream_t s);

/* (Algorithm 1, transposed) One reverse step n+1 -> n: re-assembles the shared
 * matrices of level n from V_n, W_n, solves S_v^T mu_v = [lamV_np1; 0] and
 * S_w^T mu_w = [lamW_np1; 0] (same solver and preconditioner on the transposed
 * operator, J columns), and writes lamV_n, lamW_n including the couplings
 * through the ensemble means and the eddy-viscosity maximum.  grad (device,
 * (J,3) row-major: d/dnu_j, d/dnu_m,j, d/da_j) is accumulated, may be NULL.
 * lamV_n may alias lamV_np1 (and lamW_n lamW_np1).  st (host) may be NULL. */
mhd_status mhd_ens_adjoint_step(mhd_ctx ctx, const double* V_n, const double* W_n, const double* V_np1,
                                const double* W_np1, const double* lamV_np1, const double* lamW_np1,
                                double* lamV_n, double* lamW_n, const mhd_adjoint_inputs* in, double* grad,
                                mhd_step_stats* st, mhd_stream_t s);

/* (Section 1, v = u + sqrt(s) B, w = u - sqrt(s) B) Gradients w.r.t. initial
 * mode coefficients: modes (device, (nm,nP2,2)) are the nodal mode fields,
 * coefficients m < nm scale u, m >= nm scale B.  grad_ic (device (J, 2 nm)) is
 * overwritten: d/dc_{j,m} = <phi_m, lamV0_j + lamW0_j>, d/dc_{j,nm+m} =
 * sqrt(s) <phi_m, lamV0_j - lamW0_j>.  nm <= 4. */
mhd_status mhd_ens_adjoint_ic(mhd_ctx ctx, const double* lamV0, const double* lamW0, const double* modes, int nm,
                              double s_coupling, double* grad_ic, int J, mhd_stream_t s);

/* One launch for several ensembles: the device work of one step of every
 * context in the group (each with its own mesh, J and fixed solver schedule)
 * is captured into a single HIP graph with one parallel branch per ensemble
 * (forked onto the group's own streams) and replayed by every later call with
 * the same arguments.  Arrays are per context (n of each); in[i] as for
 * mhd_ens_step.  The stream must be non-null.  Contexts of one group must not
 * be stepped concurrently elsewhere. */
typedef struct mhd_group_s* mhd_group;
mhd_status mhd_ens_group_create(int n, const mhd_ctx* ctxs, mhd_group* out);
mhd_status mhd_ens_group_step(mhd_group g, double* const* V, double* const* W, double* const* Q, double* const* R,
                              const mhd_step_inputs* in, mhd_stream_t s);
mhd_status mhd_ens_group_free(mhd_group g);

/* Last error message of the calling thread ("" if none). */
const char* mhd_ens_last_error(void);

/* Library version string. */
const char* mhd_ens_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MHD_ENS_H */
