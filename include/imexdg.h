/*
 * imexdg.h - C-ABI of the MI355X rotating IMEX-DG hot path.
 *
 * The library evaluates the matrix-free DG operators of a rotating,
 * compressible Euler solver (gravity, f-plane Coriolis) and advances it with
 * the second-order IMEX additive Runge-Kutta scheme of Sec. 3 of the paper:
 * explicit advective residual, implicit acoustic pressure Schur complement
 * solved by GMRES inside the R1 / R2 Picard iterations, with
 * (A + R)^{-1} = (I + beta J)^{-1} A^{-1} applied pointwise (Sec. 3.1).
 *
 * Conventions shared by every call:
 *  - All floating-point data are IEEE binary64 unless stated otherwise.
 *  - A field is an array [E][Np] with Np = (r+1)^3 nodal values per element;
 *    multi-field arrays are field-major, e.g. the conserved state is
 *    [5][E][Np] = (rho, rho*u, rho*v, rho*w, rho*E).
 *  - Nodes are the tensor Gauss-Legendre points of each element (the nodal
 *    basis of Sec. 3); node index i + n*(j + n*k), n = r+1, x index fastest.
 *  - Elements: base cells numbered bz + nz*(bx + nx*by) (vertical fastest);
 *    a refined base cell is replaced by its leaves, depth first, children
 *    numbered cz + 2*(cx + 2*cy).
 *  - "Dual" vectors are weak-form integrals against the basis functions
 *    (e.g. S p); "nodal" vectors hold values at the nodes (tendencies
 *    f = M^{-1} T, states).
 *  - Device pointers are caller-owned device memory (on the device current
 *    when the solver was created) and must not alias unless stated. Work is
 *    queued on the solver's HIP stream; a call that returns host values
 *    synchronises that stream.
 *  - Every function returns IMX_OK (0) or an error code and never aborts or
 *    prints. A call on a solver or a server that fails leaves its description
 *    in that object (imx_solver_last_error, imx_server_last_error); calls with
 *    no object yet (mesh and solver creation) leave it in imx_last_error(),
 *    which describes the last failure on the calling thread.
 *  - The library keeps no global mutable state besides that per-thread error
 *    text: objects own everything else.
 */
#ifndef IMEXDG_H
#define IMEXDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IMX_OK = 0,
    IMX_EINVAL = 1,      /* invalid argument or unsupported configuration */
    IMX_ENOMEM = 2,      /* workspace too small / host allocation failed */
    IMX_EHIP = 3,        /* HIP runtime error */
    IMX_ENOCONV = 4,     /* Picard or GMRES iteration cap reached without convergence */
    IMX_ENONFINITE = 5,  /* NaN or Inf detected */
    IMX_EREJECT = 6,     /* server: request can never fit the budget */
    IMX_ESTATE = 7       /* call not valid in the object's current state */
} imx_status;

enum { IMX_R1 = 1, IMX_R2 = 2 };            /* fixed-point treatment of R u and M_g u */
enum { IMX_FP64 = 0, IMX_MIXED = 1 };       /* arithmetic of the Krylov inner loop */
enum { IMX_FLAT = 0, IMX_BELL = 1, IMX_GAUSS = 2 };

typedef struct imx_mesh imx_mesh;
typedef struct imx_solver imx_solver;

/* Box [0,Lx]x[0,Ly]x[0,Lz] with nx*ny*nz base hexahedra of degree `degree`
 * (1..4). Periodic in x / y when flagged, slip walls otherwise and always at
 * z = 0 and z = Lz. terrain != IMX_FLAT deforms the box with the Gal-Chen
 * map z = h + zeta (Lz - h) / Lz over the surface
 *   bell:     h = h0 / (1 + d^2/a^2)       (Sec. 4.3)
 *   gaussian: h = h0 exp(-d^2/a^2)
 * with d the (minimum-image, in periodic directions) horizontal distance to
 * (xc, yc); the map is represented by its degree-r interpolant at the
 * Gauss-Lobatto points of each base cell. ref_boxes holds n_ref boxes
 * {x0,x1,y0,y1,z0,z1}: box i refines every level-i leaf that overlaps it with
 * positive volume (static 2:1 refinement, hanging faces, Sec. 4.3). */
typedef struct {
    double Lx, Ly, Lz;
    int nx, ny, nz, degree;
    int periodic_x, periodic_y;
    int terrain;
    double h0, a, xc, yc;
    int n_ref;
    const double* ref_boxes;     /* host, n_ref*6 doubles, read during the call */
} imx_mesh_desc;

/* Physical constants (Sec. 2, Sec. 4) and the optional Rayleigh sponge of
 * Sec. 4.3 (eq. damping), relaxing the momentum towards rho * sponge_u in the
 * explicit (non-stiff) part; sponge_lambda = 0 switches it off. Its
 * coefficient at a node is the largest of the top layer's
 * lambda_z = sponge_lambda sin^2(pi/2 (z - zB)/(zT - zB)) for z >= zB and of
 * the lateral layers' profiles of the same form over the first and the last
 * sponge_xw of [0, Lx] and sponge_yw of [0, Ly] (0 = no lateral layer),
 * rising from 0 at a layer's inner edge to sponge_lambda at the domain
 * boundary (Lx, Ly: the mesh's extents). imx_solver_create fails with
 * IMX_EINVAL if a width is negative, the two layers of a direction
 * overlap, or a sponge is asked for (sponge_lambda != 0) with
 * sponge_lambda negative or not finite or with sponge_zT <= sponge_zB.
 * slice != 0 selects the vertical-slice equations (Sec. 2, eq.
 * vertical_slice: d/dy = 0, v prognostic) on a mesh with one periodic
 * element in y, no refinement and flat ground: every step ends with the L2
 * projection of the state onto fields constant in y (each y-line of nodes
 * replaced by its Gauss-weighted mean; element integrals and the mass are
 * unchanged). imx_solver_create fails with IMX_EINVAL on another mesh. */
typedef struct {
    double gamma, R, g, f;
    double sponge_zB, sponge_zT, sponge_lambda;
    double sponge_u[3];
    double sponge_xw, sponge_yw;
    int slice;
} imx_phys;

/* Solver settings. GMRES(gmres_restart) on the M-preconditioned pressure
 * Schur system in the L2(M) inner product stops when its residual falls to
 * gmres_tol times the norm of the right-hand side, after gmres_max
 * iterations (per solve), or on breakdown; the Picard loop stops when the
 * relative variation of (u, p) (velocity weighted by the acoustic impedance)
 * is below picard_tol or after picard_max iterations. fixed_iterations != 0
 * runs exactly picard_max Picard and gmres_max GMRES iterations (parity
 * mode). precision IMX_MIXED runs the Krylov inner loop in binary32 inside an
 * outer binary64 defect correction that stops at gmres_tol; inner_tol is the
 * relative residual reduction asked of each binary32 inner solve. */
typedef struct {
    double dt;
    int scheme;                  /* IMX_R1 or IMX_R2 */
    int precision;               /* IMX_FP64 or IMX_MIXED */
    double picard_tol;
    int picard_max;
    double gmres_tol;
    int gmres_restart;           /* 1..32 */
    int gmres_max;
    int fixed_iterations;
    double inner_tol;
} imx_numerics;

typedef struct {
    int picard_iters;
    int gmres_iters;             /* total Krylov iterations (all precisions) */
    double gmres_relres;         /* last true relative residual */
    double picard_variation;     /* last relative Picard variation */
} imx_solve_stats;

typedef struct {
    int steps;
    int picard_iters;
    int gmres_iters;
    double mass;                 /* total mass after the last step (binary64) */
} imx_step_stats;

/* ---------------------------------------------------------------- mesh */
/* Builds the mesh and its geometry on the host. Errors: IMX_EINVAL for bad
 * sizes, unbalanced refinement or inverted elements, and on terrain-following
 * meshes when the compact per-element form of the metric (from which the
 * Krylov passes form it) does not reproduce the mapped geometry to 1e-12 of
 * its largest entry. */
imx_status imx_mesh_create(const imx_mesh_desc* desc, imx_mesh** out);
/* The same call under the name of the box-mesh constructor (every mesh of the
 * library is such a box, optionally refined and terrain-following). */
imx_status imx_mesh_create_box(const imx_mesh_desc* desc, imx_mesh** out);
/* Number of elements, nodes per element, number of coarse hanging faces and
 * whether the geometry is deformed (per-point Jacobians). */
imx_status imx_mesh_info(const imx_mesh* mesh, int64_t* n_elem, int* nodes_per_elem,
                         int64_t* n_hanging_faces, int* deformed);
/* Physical coordinates of every node, host array [3][E][Np] owned by the caller. */
imx_status imx_mesh_node_coords(const imx_mesh* mesh, double* xyz_host);
/* Diagonal of the mass matrix (quadrature weight times det J) at every node,
 * host array [E][Np]. */
imx_status imx_mesh_mass_diag(const imx_mesh* mesh, double* m_host);
void imx_mesh_destroy(imx_mesh* mesh);

/* -------------------------------------------------------------- solver */
/* Creates a solver for `mesh` (which must outlive it) on HIP stream
 * `hip_stream` (NULL = default stream) of the current device. No device
 * memory is allocated: query the workspace size and bind caller memory.
 * IMX_EINVAL on invalid settings (checked before any device call),
 * IMX_EHIP when no HIP device is current. */
imx_status imx_solver_create(const imx_mesh* mesh, const imx_phys* phys, const imx_numerics* num,
                             void* hip_stream, imx_solver** out);
imx_status imx_solver_workspace_bytes(const imx_solver* s, size_t* bytes);
/* Binds `bytes` of caller-owned device memory (>= the queried size, 256-byte
 * aligned) as the solver's workspace and uploads tables and geometry. The
 * memory must stay valid until imx_solver_destroy. */
imx_status imx_solver_bind_workspace(imx_solver* s, void* dev_ptr, size_t bytes);
/* Changes dt / tolerances / scheme / precision of a bound solver. */
imx_status imx_solver_set_numerics(imx_solver* s, const imx_numerics* num);
/* Replay of the Krylov loop from HIP graphs (default off). Each chunk of up to
 * 8 GMRES columns (matrix-vector product, Gram-Schmidt pass, Givens step per
 * column; Sec. 3, the pressure system's GMRES) is a fixed launch sequence: it
 * is captured once per solver and argument set on a private stream of the
 * solver and then replayed on the solver's stream with one launch. Results
 * are bitwise those of direct launches. enable = 0 launches every kernel
 * directly and frees the captured graphs. Kernel timing (imx_solver_timing)
 * always launches directly. For callers that drive many small solvers from
 * few host threads; on a single MI355X the replay measured the same step
 * times as direct launches (the time between dependent kernels is spent on
 * the device, not in the launch calls). */
imx_status imx_solver_set_graphs(imx_solver* s, int enable);

/* Rayleigh damping layers (Sec. 4.3, eq. damping): by default they relax the
 * momentum towards rho * sponge_u (the mass stays exactly conserved). With a
 * target state q_target_dev (device, [5][E][Np] conserved (rho, rho u, rho E),
 * caller-owned, retained: it must stay valid and unchanged until the next call
 * with another pointer or NULL) they relax the whole conserved state towards
 * it instead; the density part then changes the mass inside the layers. The
 * section states the damping profile and lambda * dt but not the variables it
 * acts on; both readings are offered. NULL restores the default. Takes effect
 * from the next explicit evaluation; IMX_EINVAL for a null solver. */
imx_status imx_solver_set_sponge_target(imx_solver* s, const double* q_target_dev);

/* Copies the conserved state y = (rho, rho u, rho E) of Sec. 2 as nodal values
 * [5][E][Np] (device, caller-owned, not retained) into / out of the solver's
 * resident copy y^n that imx_step advances (Sec. 3: y^n -> y^{n+1}).
 * Asynchronous on the solver's stream; IMX_ESTATE before a workspace is
 * bound, IMX_EINVAL for a null pointer. */
imx_status imx_set_state(imx_solver* s, const double* q_dev);
imx_status imx_get_state(const imx_solver* s, double* q_dev);

/* Explicit tendencies of Sec. 3 as nodal vectors f = M^{-1} T at state q:
 * fNS [5][E][Np] (advection with Rusanov fluxes, sponge) and fS [4][E][Np]
 * (momentum and energy: pressure with centred flux, enthalpy flux with
 * Rusanov dissipation on rho e, gravity, Coriolis). Face values are the
 * traces of the nodal (rho, u, p), the variables on whose traces the stage
 * operators act, so fS at a converged stage is the stage's own operator. */
imx_status imx_explicit_residual(imx_solver* s, const double* q_dev, double* fNS_dev, double* fS_dev);

/* Fixes the stage coefficients of the implicit operators for the implicit
 * diagonal coefficient a_ll = (2 - sqrt(2))/2 of the tableau: stage density
 * rho_l [E][Np], lagged pressure p^k [E][Np] and lagged velocity u^k
 * [3][E][Np] (all nodal, device, copied). */
imx_status imx_implicit_setup(imx_solver* s, const double* rho_l_dev, const double* p_lag_dev,
                              const double* u_lag_dev);
/* Dual vector S p of the pressure Schur complement of the current setup:
 * R2: [D - (C^k + M_g)(A + R)^{-1} B] p, R1: [D - C^k A^{-1} B] p (Sec. 3). */
imx_status imx_schur_apply(imx_solver* s, const double* p_dev, double* out_dev);
/* One implicit stage solve (Picard + GMRES) for the stage density rho_l:
 * F = f - f_g [3][E][Np] and G0 = g without the lagged implicit Rusanov term
 * [E][Np] are dual vectors; p0 / u0 the initial iterate (nodal). On return
 * p [E][Np] and u [3][E][Np] hold the last iterate. IMX_ENOCONV if the
 * Picard loop hit picard_max without convergence (not in parity mode). */
imx_status imx_implicit_solve(imx_solver* s, const double* rho_l_dev, const double* F_dev,
                              const double* G0_dev, const double* p0_dev, const double* u0_dev,
                              double* p_dev, double* u_dev, imx_solve_stats* stats);
/* Advances the bound state by nsteps IMEX-ARK2 steps (Sec. 3). A step that
 * fails (IMX_ENOCONV, IMX_ENONFINITE) leaves the state of the last completed
 * step in place. */
imx_status imx_step(imx_solver* s, int nsteps, imx_step_stats* stats);
/* Total mass sum_K int_K rho of the bound state with the elements'
 * Gauss-Legendre rule (the discrete mass that the DG scheme of Sec. 3
 * conserves: the density equation is in flux form and b = b~ preserves linear
 * invariants), accumulated in binary64 in a fixed order; *mass (host)
 * receives it (NaN if the state holds one). Synchronises the stream. */
imx_status imx_total_mass(imx_solver* s, double* mass);
/* Allocation-free form of imx_total_mass, for callers that cannot allocate
 * device memory or synchronise (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). Writes the mass sum_K int_K rho of
 * the caller's state q_dev [5][E][Np] (device, caller-owned, this solver's
 * mesh) to out_dev[0] and the number of NaN or Inf values among its 5 fields
 * to out_dev[1] (device, caller-owned, 2 doubles), asynchronously on the
 * solver's stream: no synchronisation and no host copy. Same kernels and
 * summation order as imx_total_mass, so the same bits for the same state.
 * The partial sums go to a static device array of 4096 x 2 doubles (64 KiB)
 * that every GPU the library runs on holds until the process ends; the
 * reduction never uses more than 4096 workgroups, so every mesh a solver
 * accepts fits. All calls on one GPU share that array: calls that overlap on
 * one GPU (different streams or threads) race. Allocates nothing.
 * IMX_ESTATE before a workspace is bound, IMX_EINVAL for a null pointer or
 * when the solver's device is not the current device. */
imx_status imx_total_mass_noalloc(const imx_solver* s, const double* q_dev, double* out_dev);
/* Geostrophic imbalance of the bound state (eq. egeo, Sec. 4.2, planetary-
 * scale test): the domain mean int |(1/rho) dp/dx - f v| dV / int dV, with
 * dp/dx the derivative of each element's own pressure polynomial at its
 * nodes and the elements' Gauss-Legendre rule. On a vertical slice (one
 * element in y) it is the paper's mean over x and z. *egeo (host) receives the
 * value; synchronises. IMX_EINVAL for a null pointer. */
imx_status imx_geo_imbalance(imx_solver* s, double* egeo);
void imx_solver_destroy(imx_solver* s);
/* Description of the last failure of a call on this solver ("" if none);
 * the text stays valid until the next failing call on it or its destruction. */
const char* imx_solver_last_error(const imx_solver* s);

/* ------------------------------------------------------- adaptivity */
/* Dynamic adaptivity: the refinement of Sec. 4.3 (nested 2:1 boxes around
 * the hill, static in the paper) changed during a run. Transfers nodal
 * fields [nfields][E][Np] from mesh `from` to mesh `to`, two refinements of
 * the same box, base grid, degree and terrain whose leaves differ by at most
 * two levels: a leaf present in both is copied; a new leaf inside an old,
 * coarser one takes the old polynomial at its nodes (exact: the restriction
 * of a polynomial of degree r is one); a new leaf covering old, finer leaves
 * takes the L2 projection of the old fields onto its polynomials with the
 * mass-matrix quadrature of Sec. 3 (W detJ at the Gauss-Legendre nodes), so
 * the integral of every field (mass, momentum, energy for the conserved
 * state) is kept in both directions, and on affine elements coarsening
 * undoes refinement. q_from_dev / q_to_dev: device, caller-owned, not
 * aliased. ws_dev: caller-owned device workspace of at least the queried
 * bytes (256-byte aligned) holding the leaf map, W detJ of both meshes and
 * the interpolation tables; it is written on `hip_stream` (NULL = default
 * stream) and may be reused once the stream has passed the transfer. The
 * host part (the leaf map) synchronises the stream once before the kernel
 * is queued; the kernel itself runs asynchronously. IMX_EINVAL if the meshes
 * are not two refinements of one grid or differ by more than two levels,
 * IMX_ENOMEM if the workspace is too small. */
imx_status imx_transfer_workspace_bytes(const imx_mesh* from, const imx_mesh* to, size_t* bytes);
imx_status imx_transfer_state(const imx_mesh* from, const imx_mesh* to, void* ws_dev, size_t ws_bytes,
                              const double* q_from_dev, double* q_to_dev, int nfields, void* hip_stream);

/* ------------------------------------------------------------ timing */
/* Kernel classes timed by imx_solver_timing. */
enum {
    IMX_K_EXPLICIT = 0,   /* explicit residual */
    IMX_K_PASS1 = 1,      /* Schur pass 1: w = (I+beta J)^{-1} A^{-1} (F - B p), face fluxes */
    IMX_K_PASS2 = 2,      /* Schur pass 2: D p - (C^k + M_g) w */
    IMX_K_LAMBDA = 3,     /* Picard refresh of the lagged energy terms */
    IMX_K_DOTS = 4,       /* GMRES M-weighted multi-dot products */
    IMX_K_ORTHO = 5,      /* GMRES Gram-Schmidt update (+ dots or norm) */
    IMX_K_LINCOMB = 6,    /* GMRES solution update */
    IMX_K_STAGE = 7,      /* ARK2 stage combinations */
    IMX_K_REDUCE = 8,     /* small reductions (norms, mass, Picard variation) */
    IMX_K_COUNT = 9
};
/* enable != 0: clears the counters and brackets every subsequent kernel
 * launch of the solver with a pair of HIP events on its stream; enable = 0
 * stops recording. */
imx_status imx_solver_timing(imx_solver* s, int enable);
/* Accumulated device time (ms), algorithmic bytes (every field a kernel reads
 * or writes counted once, geometry included, neighbour re-reads and internal
 * face buffers excluded) and launch count of kernel class `kind` since timing
 * was enabled. Synchronises the stream. */
imx_status imx_solver_timing_report(imx_solver* s, int kind, double* total_ms, double* bytes,
                                    int64_t* launches);

/* ------------------------------------------------------------ serving */
/* Serving form of the method (not a construct of the paper, which integrates
 * one state at a time): many independent integrations of Sec. 3 (ARK2 steps
 * of their own meshes and states), each exactly as imx_step would advance it
 * alone.
 * Ensemble server: integrations of different meshes, degrees and physics
 * share one device memory pool (the HBM budget). Requests wait in arrival
 * order; imx_server_tick admits every waiting request whose workspace fits
 * the free pool while fewer than max_running members run, and reaps members
 * that have finished (their memory returns to the pool). Each running member
 * owns a HIP stream and a host worker thread that advances it step by step,
 * so members admitted at different times overlap on the device. A member's
 * result does not depend on what runs beside it (no shared buffers, fixed
 * reduction orders). */
typedef struct imx_server imx_server;

typedef struct {
    int steps_done;
    int status;                  /* imx_status of the member's last step */
    double p50_step_ms, p99_step_ms, mean_step_ms;
    double queue_ms;             /* submit -> admission */
    double run_ms;               /* admission -> last step done */
    int64_t gmres_iters;
} imx_member_stats;

typedef struct {
    int64_t submitted, admitted, completed, rejected, running, waiting;
    size_t pool_bytes, pool_bytes_in_use, pool_bytes_peak;
    double p50_step_ms, p99_step_ms;   /* over every member step so far */
    double dof_updates;                /* sum over members of 5 E Np x steps done */
    double busy_seconds;               /* first admission -> last completion */
} imx_server_stats;

/* pool_dev: caller-owned device memory of pool_bytes (256-byte aligned) on the
 * current device; it must outlive the server. */
imx_status imx_server_create(void* pool_dev, size_t pool_bytes, int max_running, imx_server** out);
/* Queues nsteps IMEX-ARK2 steps of a member starting from q0_host [5][E][Np]
 * (copied). IMX_EREJECT if its workspace can never fit the pool. */
imx_status imx_server_submit(imx_server* sv, const imx_mesh_desc* mesh, const imx_phys* phys,
                             const imx_numerics* num, const double* q0_host, int nsteps, uint64_t* id);
/* Reaps finished members and admits waiting ones; returns the counts. */
imx_status imx_server_tick(imx_server* sv, int* n_running, int* n_waiting);
/* Final state [5][E][Np] (host) and statistics of a finished member;
 * IMX_ESTATE while it has not finished, IMX_EINVAL for an unknown id. */
imx_status imx_server_result(imx_server* sv, uint64_t id, double* q_host, imx_member_stats* stats);
imx_status imx_server_query(imx_server* sv, imx_server_stats* stats);
/* Members admitted after this call replay the chunks of their Krylov loop
 * from HIP graphs (enable != 0; see imx_solver_set_graphs) or launch every
 * kernel directly (0, the default). Results are bitwise the same either way. */
imx_status imx_server_set_graphs(imx_server* sv, int enable);
/* Waits for running members, then destroys the server. */
void imx_server_destroy(imx_server* sv);
/* Description of the last failure of a call on this server ("" if none);
 * valid until the next failing call on it or its destruction. A member's own
 * failure is reported through imx_server_result. */
const char* imx_server_last_error(const imx_server* sv);

/* Description of the last error raised on the calling thread (by any call). */
const char* imx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
