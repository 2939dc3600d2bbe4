/*
 * sgp.h -- C ABI of libsgp: support-graph (maximum-spanning-tree)
 * preconditioned conjugate gradients for the friction equation Gamma v = F of
 * off-lattice cell-based models, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Steinman & Buttenschoen, "Support Graph Preconditioners for
 * Off-Lattice Cell-Based Models", arXiv 2410.04512.  The call chain follows
 * the paper's simulation step (Section 2, Steps 1-4):
 *
 *   sgp_collide        Steps 1-2   which cells touch (collision graph)
 *   sgp_assemble_gamma Step 3      friction blocks, Gamma as 3x3-block CSR
 *   sgp_build_tree     Section 3.1 maximum spanning forest, rooted
 *   sgp_factor_tree    Section 3.3 block LDL^T of the forest's Laplacian P
 *   sgp_pcg_solve      Section 1.1 + Appendix B.1: PCG with z = P^{-1} r
 *
 * Conventions shared by every entry point
 *  - Every int-returning call returns an sgp_status (0 = success, negative =
 *    error).  No C++ exception crosses this boundary.  sgp_last_error(ctx)
 *    gives a human-readable message for the last failing call on ctx.
 *  - Pointers named as "device" must point to device memory of the GPU that
 *    was current when the context was created; "host" pointers to host memory.
 *    Caller-owned buffers stay owned by the caller; the library never frees
 *    them and never keeps them after the call returns.
 *  - Handles (sgp_graph, sgp_bsr, sgp_tree, sgp_prec) are library-owned and
 *    are released with their *_free function.  A handle keeps its device
 *    buffers between calls and only grows them, so repeated calls of the same
 *    size allocate nothing.
 *  - All work is ordered on the context's stream (borrowed from the caller).
 *    Calls that must report a data-dependent size synchronise that stream;
 *    each such call says so.
 *  - Vectors of cell quantities are [n][3] row-major FP64 (x, y, z per cell).
 *  - One context per host thread; a context is not thread-safe.
 *  - Layouts of exported arrays are the canonical order: edges (i, j), i < j,
 *    lexicographic; neighbour rows ascending; tree edges ascending.
 */
#ifndef SGP_H
#define SGP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGP_OK = 0,
    SGP_EINVAL = -1,      /* bad argument (null pointer, negative size, coincident centres) */
    SGP_ENOMEM = -2,      /* device allocation failed */
    SGP_EHIP = -3,        /* a HIP runtime call failed */
    SGP_ECAPACITY = -4,   /* a cell has more than max_deg contacts */
    SGP_ENOTSPD = -5,     /* a 3x3 pivot block is not symmetric positive definite */
    SGP_ENOCONV = -6,     /* max_iter reached before the tolerance */
    SGP_EBREAKDOWN = -7,  /* CG breakdown: p.Gamma p <= 0 or not finite */
    SGP_ENONFINITE = -8,  /* NaN or Inf in an input or an iterate */
    SGP_ESTALE = -9       /* a recorded step cannot replay these inputs (record it again), or
                             Gamma's 3x3 blocks are asked for after its graph was collided again */
} sgp_status;

typedef struct sgp_ctx_ *sgp_ctx;
typedef struct sgp_graph_ *sgp_graph;
typedef struct sgp_bsr_ *sgp_bsr;
typedef struct sgp_tree_ *sgp_tree;
typedef struct sgp_prec_ *sgp_prec;
typedef struct sgp_mpnn_ *sgp_mpnn;
typedef struct sgp_step_ *sgp_step;

/* ---------------------------------------------------------------- context */

/* Create a context on the current HIP device that orders its work on
 * `hip_stream` (a hipStream_t; NULL = the default stream).  The stream is
 * borrowed: the caller keeps it alive until sgp_destroy. */
int sgp_create(sgp_ctx *out, void *hip_stream);
void sgp_destroy(sgp_ctx ctx);
/* Message of the last failing call on ctx ("" if none).  Owned by ctx. */
const char *sgp_last_error(sgp_ctx ctx);
/* Change the stream subsequent calls are ordered on. */
int sgp_set_stream(sgp_ctx ctx, void *hip_stream);

/* ------------------------------------------------- Steps 1-2: collide */

int sgp_graph_create(sgp_ctx ctx, sgp_graph *out);
void sgp_graph_free(sgp_graph g);

/* Collision graph of n spheres (Section 2, Steps 1-2).  pos [n][3] and
 * radius [n] are device FP64.  Cells i < j touch iff d_ij < R_i + R_j with
 * d_ij = sqrt((dx*dx + dy*dy) + dz*dz), dx = x_j - x_i (IEEE, no fused
 * multiply-add); the overlap w_ij = (R_i + R_j) - d_ij stands in for the
 * contact area A_ij and u_ij = (r_j - r_i)/d_ij is the unit contact vector.
 * max_deg bounds the contacts of any one cell (SGP_ECAPACITY beyond it).
 * Coincident centres in contact give SGP_EINVAL; non-finite positions
 * SGP_ENONFINITE.  Synchronises the stream once (edge count). */
int sgp_collide(sgp_ctx ctx, int64_t n, const double *pos, const double *radius,
                int32_t max_deg, sgp_graph g);

/* Same, for n_inst independent cell clusters stored back to back: cluster k
 * owns cells [offsets[k], offsets[k+1]) (offsets: host int64 [n_inst+1],
 * offsets[0] = 0).  Cells of different clusters never touch, wherever they
 * are.  The result is the disjoint union of the clusters' graphs; edge ids of
 * cluster k follow those of cluster k-1. */
int sgp_collide_batched(sgp_ctx ctx, int64_t n_inst, const int64_t *offsets,
                        const double *pos, const double *radius, int32_t max_deg, sgp_graph g);

/* What collide stores as a contact's w (the contact area A_ij of eq.
 * cell_cell_friction), for the collides that follow on this context:
 *  SGP_CONTACT_OVERLAP  w = R_i + R_j - d_ij, the overlap (default);
 *  SGP_CONTACT_HERTZ    the contact area of the Hertz model that the paper's
 *                       benchmark cells use (Section 5.1; the paper names the
 *                       model, not its formula): two spheres pressed together
 *                       by the overlap delta touch in a disc of radius
 *                       sqrt(R* delta), R* = R_i R_j / (R_i + R_j), so
 *                       w = pi R* delta, evaluated as
 *                       (pi * ((R_i * R_j) / (R_i + R_j))) * delta.
 * The contact test, u and the edge numbering do not change.  Unknown models
 * give SGP_EINVAL. */
enum { SGP_CONTACT_OVERLAP = 0, SGP_CONTACT_HERTZ = 1 };
int sgp_set_contact_model(sgp_ctx ctx, int32_t model);

/* Sizes: n cells, m contacts.  Host outputs; either may be NULL. */
int sgp_graph_size(sgp_graph g, int64_t *n, int64_t *m);

/* Copy the graph into caller buffers (device pointers; NULL = skip):
 * rowptr [n+1], col [2m] (neighbour rows ascending), ei, ej [m] (edges
 * (i, j), i < j, lexicographic), w [m], u [m][3]. */
int sgp_graph_export(sgp_ctx ctx, sgp_graph g, int32_t *rowptr, int32_t *col,
                     int32_t *ei, int32_t *ej, double *w, double *u);

/* ---------------------------------------- Step 3: friction matrix Gamma */

int sgp_bsr_create(sgp_ctx ctx, sgp_bsr *out);
void sgp_bsr_free(sgp_bsr A);

/* Gamma as a 3x3-block CSR matrix (eq. cell_cell_friction and the block
 * Laplacian definition of Section 2): for every contact e = (i, j),
 * W_e = w_e (g_par u u^T + g_perp (I - u u^T)), Gamma_ij = Gamma_ji = -W_e;
 * Gamma_ii = g_med I + the W_e of cell i's contacts added in ascending
 * neighbour order.  Row i holds its neighbours and itself, columns ascending.
 * g_par, g_perp > 0 and g_med >= 0, else SGP_EINVAL.  Stored in the form the
 * product reads (tune key spmv_form): the contacts' v = sqrt(w) u with the
 * diagonal blocks, and the 3x3 blocks themselves only for the block-CSR
 * product (spmv_form 0; assembled on first use when that key changes after
 * the assembly, which needs g not collided again since: SGP_ESTALE
 * otherwise).  sgp_bsr_export always rebuilds the blocks from g. */
int sgp_assemble_gamma(sgp_ctx ctx, sgp_graph g, double g_par, double g_perp, double g_med,
                       sgp_bsr A);

/* Sizes of the matrix: n block rows, nnzb stored blocks (n + 2m). */
int sgp_bsr_size(sgp_bsr A, int64_t *n, int64_t *nnzb);

/* Copy out (device pointers; NULL = skip): rowptr [n+1], bcol [nnzb],
 * val [nnzb][3][3] row-major blocks. */
int sgp_bsr_export(sgp_ctx ctx, sgp_bsr A, int32_t *rowptr, int32_t *bcol, double *val);

/* y = Gamma x (device [n][3] FP64; x and y must not overlap). */
int sgp_spmv(sgp_ctx ctx, sgp_bsr A, const double *x, double *y);

/* ----------------------------- Section 3.1: maximum spanning forest */

int sgp_tree_create(sgp_ctx ctx, sgp_tree *out);
void sgp_tree_free(sgp_tree T);

/* Maximum spanning forest of the collision graph weighted by w_e (the
 * smallest eigenvalue of W_e is g_perp w_e or g_par w_e, so the order by w_e
 * is the paper's order by lambda_min, Section 3.1), ties broken by the
 * smaller edge id, so the forest is unique and equals Prim's.  Each tree is
 * rooted at its smallest cell id; parent and hop depth are computed.
 * Synchronises the stream. */
int sgp_build_tree(sgp_ctx ctx, sgp_graph g, sgp_tree T);

/* The local-MST forest of Section 6 (Discussion): the cells are cut into
 * clusters by a spatial subdivision and every cluster keeps a maximum
 * spanning forest of its own contacts; contacts between clusters are left
 * out of the preconditioner (still a subgraph of the collision graph, so the
 * support bound lambda_min(P^{-1} Gamma) >= 1 of Section 4 holds) and no
 * tree path leaves a cluster.  Clusters: the cells of every instance of g in
 * the Z-order of a uniform grid, cut into runs of cluster_size (the last run
 * of an instance may be shorter); grid cubes of side 2 max R (1 if every
 * radius is 0) anchored at the bounding box's minimum corner, cell coordinates
 * floor((x - lo) / h) in FP64, Z-order = the Morton code interleaving the
 * bits of (c_x, c_y, c_z) from the lowest (x lowest), ties by cell id; cluster
 * ids numbered instance by instance in that order.  pos, radius: the device
 * arrays g was built from.  The forest is the maximum spanning forest of the
 * graph without its edges between clusters (same order and ties as
 * sgp_build_tree), each tree rooted at its smallest cell id.  sgp_factor_tree
 * on such a forest (CONTRACT schedule) groups every elimination step by
 * component, so each sweep of the apply is one launch.  More than 1024 grid
 * cells along an axis, or Z-order keys with the instance over 32 bits, give
 * SGP_EINVAL.  Synchronises the stream. */
int sgp_build_forest(sgp_ctx ctx, sgp_graph g, const double *pos, const double *radius,
                     int32_t cluster_size, sgp_tree T);

/* The cluster of every cell (device int32 [n], caller numbering; NULL =
 * skip) and the number of clusters (host, NULL = skip) of a forest from
 * sgp_build_forest (0 clusters and nothing copied for sgp_build_tree). */
int sgp_tree_clusters(sgp_ctx ctx, sgp_tree T, int32_t *cluster, int64_t *n_clusters);

/* n_tree_edges = n - (number of trees); n_roots; max_depth (host outputs,
 * NULL = skip). */
int sgp_tree_size(sgp_tree T, int64_t *n_tree_edges, int64_t *n_roots, int32_t *max_depth);

/* Copy out (device pointers, NULL = skip): tree_edge [n_tree_edges] edge ids
 * ascending; parent [n] (-1 at roots); depth [n] (0 at roots). */
int sgp_tree_export(sgp_ctx ctx, sgp_tree T, int32_t *tree_edge, int32_t *parent, int32_t *depth);

/* --------------------------------- Section 3.3: factor the support tree */

int sgp_prec_create(sgp_ctx ctx, sgp_prec *out);
void sgp_prec_free(sgp_prec M);

/* Elimination schedules for the tree factorisation.  Any order that removes
 * a vertex only after the vertices it connects to below it gives the exact
 * LDL^T of P without fill (Lemma nofill):
 *  SGP_SCHED_LEVEL     decreasing depth, one parallel step per level
 *                      (Alg. 2's own order);
 *  SGP_SCHED_CONTRACT  leaves and an independent set of one-child chain
 *                      vertices are removed together in each step (rake and
 *                      compress); a removed chain vertex joins its parent and
 *                      child by a new 3x3 block, so the factor is the exact
 *                      LDL^T of P in that order with O(log n) steps. */
enum { SGP_SCHED_LEVEL = 0, SGP_SCHED_CONTRACT = 1 };

/* Factor the block Laplacian P of the forest (self-loops g_med I included,
 * Section 3.1): P_ii = g_med I + W_e of the tree edges at i (ascending edge
 * id), P_{p(i),i} = -W_{e(i)}.  Pivot blocks are inverted in FP64 through a
 * 3x3 Cholesky factor; a non-positive pivot gives SGP_ENOTSPD.
 * Synchronises the stream. */
int sgp_factor_tree(sgp_ctx ctx, sgp_graph g, sgp_tree T, double g_par, double g_perp,
                    double g_med, int32_t schedule, sgp_prec M);

/* Vaidya's augmented maximum spanning tree (Section 3.1) with the nested
 * solve of Sections 3 and 5.  The tree (a spanning tree from sgp_build_tree,
 * not a local forest) is factored as by sgp_factor_tree; then it is cut into
 * pieces: walking the forest children first, a vertex weighs 1 plus the
 * weights of its children that were not cut off, and a vertex of weight
 * >= ceil(n / parts) is cut off from its parent and heads a piece (parts <= 0:
 * ceil(n^(1/4)), the paper's choice of t).  For every pair of pieces joined
 * by a contact, the heaviest such contact (ties: the smaller edge id) is
 * added back; P' is the block Laplacian of the tree and the added contacts
 * plus g_med I.  sgp_pcg_solve with M then runs flexible CG (Notay; one
 * direction kept: alpha = p.r / p.q, beta = -z.q / p.q) whose
 * preconditioner is CG on P' z = r from zero, preconditioned by the tree, to
 * ||r_inner|| <= inner_rtol ||r|| (0 < inner_rtol < 1; the paper: 0.1).  One
 * FP64 system to rtol only (SGP_EINVAL for batches, FP32 refinement or fixed
 * iteration counts); info.iters counts the outer iterations,
 * info.inner_iters the inner ones in all.  sgp_prec_apply on such an M
 * applies its tree.  Synchronises. */
int sgp_factor_augmented(sgp_ctx ctx, sgp_graph g, sgp_tree T, double g_par, double g_perp,
                         double g_med, int32_t schedule, int32_t parts, double inner_rtol, sgp_prec M);

/* The pieces and added contacts of an augmented tree: their counts (host,
 * NULL = skip), the head of every cell's piece (device int32 [n], caller
 * numbering, NULL = skip) and the added edge ids ascending (device int32
 * [added], NULL = skip). */
int sgp_prec_augmented(sgp_ctx ctx, sgp_prec M, int64_t *pieces, int64_t *added, int32_t *piece,
                       int32_t *added_edges);

/* Block-Jacobi preconditioner M = blockdiag(Gamma_ii) (comparison method of
 * Section 5). */
int sgp_make_jacobi(sgp_ctx ctx, sgp_bsr A, sgp_prec M);

/* Number of parallel elimination steps of a tree preconditioner (host). */
int sgp_prec_steps(sgp_prec M, int32_t *steps);
/* Shape of a tree factor's elimination schedule (host outputs, each may be
 * NULL): the number of steps, the first step run by the one-workgroup tail
 * (== steps when there is none), the number of leading light steps, and the
 * number of vertices of every step (step_sizes: `steps` entries). */
int sgp_prec_info(sgp_prec M, int32_t *steps, int32_t *tail_step, int32_t *light_steps, int32_t *step_sizes);

/* z = M^{-1} r (device [n][3] FP64; r and z must not overlap).  For the tree
 * this is ForwardSolve, DiagSolve and BackwardSolve of Appendix B.1. */
int sgp_prec_apply(sgp_ctx ctx, sgp_prec M, const double *r, double *z);

/* The same apply as sgp_prec_apply, same kernels and bitwise the same z, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): it calls no
 * hipMalloc, hipFree or other allocating routine.  Its scratch (r and z in
 * the library's internal order) is a static device array of 48 MiB per GPU,
 * reserved when the library's code object is loaded and held until the
 * process ends; its address is taken at sgp_create.  Systems of more than
 * 1,048,576 cells (2^20) give SGP_EINVAL, with nothing launched.  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, contexts or host threads) race and must be ordered by the caller.
 * r and z: device [n][3] FP64, caller numbering, must not overlap. */
int sgp_prec_apply_noalloc(sgp_ctx ctx, sgp_prec M, const double *r, double *z);

/* -------------------------------------------- Section 1.1: the solve */

enum { SGP_PREC_F64 = 0, SGP_PREC_F32_IR = 1 };
/* Stopping rule: the recurrence residual, or an upper bound of the relative
 * energy-norm error ||v - v_k||_Gamma / ||v||_Gamma (Gauss-Radau quadrature
 * over CG's own coefficients with a node mu <= lambda_min(P^-1 Gamma): the
 * error estimates Section 5 monitors CG with, the lower eigenvalue bound of
 * Section 4 supplying mu).  With x0 = 0, ||v||^2 = S_k + eps_k for S_k =
 * sum_{j<k} alpha_j rho_j (rho_j = r_j'z_j), and eps_k <= phi_k rho_k with
 * phi_0 = 1/mu, phi_{k+1} = (phi_k - alpha_k) / (mu (phi_k - alpha_k) +
 * beta_{k+1}); the solve stops when phi_k rho_k / (S_k + phi_k rho_k) <= rtol^2. */
enum { SGP_STOP_RESIDUAL = 0, SGP_STOP_ERROR = 1 };

typedef struct {
    double rtol;          /* stop when ||r_k|| / ||F|| <= rtol (recurrence residual), or see stop */
    int32_t max_iter;     /* iteration cap (inner iterations in total for IR) */
    int32_t fixed_iters;  /* > 0: run exactly this many iterations, ignore rtol */
    int32_t use_x0;       /* 1: v holds the initial guess on entry; 0: start from 0 */
    int32_t precision;    /* SGP_PREC_F64, or SGP_PREC_F32_IR: FP32 inner PCG inside FP64 refinement */
    double inner_rtol;    /* IR only: relative tolerance of each inner FP32 solve */
    int32_t max_outer;    /* IR only: cap on refinement steps */
    int32_t check_every;  /* CG iterations per chunk between possible convergence reads (0 = the knob) */
    int32_t stop;         /* SGP_STOP_RESIDUAL, or SGP_STOP_ERROR: rtol bounds the relative energy-norm
                             error (FP64 from x0 = 0 only; not with the augmented tree) */
    int32_t reserved;     /* 0 */
    double mu;            /* SGP_STOP_ERROR: the Gauss-Radau node, a lower bound of lambda_min(P^-1
                             Gamma); <= 0: 1 for a tree or forest preconditioner (Section 4),
                             g_med without one, required (> 0) with block Jacobi */
} sgp_solve_opts;

typedef struct {
    int32_t status;       /* sgp_status of the solve */
    int32_t iters;        /* CG iterations (all inner iterations for IR) */
    int32_t outer_iters;  /* IR refinement steps (0 for plain PCG) */
    int32_t inner_iters;  /* augmented tree: inner CG iterations in all (0 otherwise) */
    double relres_rec;    /* ||r_k|| / ||F|| of the recurrence (FP64 residual for IR) */
    double relres_true;   /* ||F - Gamma v|| / ||F|| recomputed at the end */
    double err_bound;     /* SGP_STOP_ERROR: the final bound of the relative energy-norm error (else 0) */
} sgp_solve_info;

/* Solve Gamma v = F by preconditioned CG (left form of Section 1.1's split
 * preconditioning; Saad, Alg. 9.1).  M = NULL means no preconditioner.  F and
 * v are device [n][3] FP64; v holds x0 on entry if opts->use_x0 and the
 * solution on return (the last iterate if the status is SGP_ENOCONV).
 * ||F|| = 0 gives v = 0 with 0 iterations.  info is a host pointer and is
 * filled on every return; the call synchronises the stream. */
int sgp_pcg_solve(sgp_ctx ctx, sgp_bsr A, sgp_prec M, const double *F, double *v,
                  const sgp_solve_opts *opts, sgp_solve_info *info);

/* Independent solves of the block-diagonal system built from a batched
 * collision graph: cluster k owns rows [offsets[k], offsets[k+1]) (host
 * int64 [n_inst+1]).  Every cluster runs its own CG (own step lengths and
 * stopping test) while all clusters share each kernel launch.  info is a
 * host array [n_inst]. */
int sgp_pcg_solve_batched(sgp_ctx ctx, sgp_bsr A, sgp_prec M, int64_t n_inst,
                          const int64_t *offsets, const double *F, double *v,
                          const sgp_solve_opts *opts, sgp_solve_info *info);

/* ||F - Gamma x|| / ||F|| in FP64 (host output; F, x device [n][3]).
 * Synchronises.  Used to pick the better of two initial guesses. */
int sgp_residual_norm(sgp_ctx ctx, sgp_bsr A, const double *F, const double *x, double *relres);

/* ------------------------------- a whole batched step as one hipGraph */

/* The batched step collide -> assemble_gamma -> (build_tree -> factor_tree
 * | make_jacobi) -> pcg_solve_batched, recorded once and then replayed as a
 * single hipGraph launch: no host round trip inside the step.
 *
 * A step owns a context and graph, matrix, tree and preconditioner handles
 * of its own (created by sgp_step_create on the caller's device), so the
 * buffers its graph points to are never grown or freed by other calls; the
 * caller's context lends its stream and its launch-shape knobs and contact
 * model (copied at recording).
 *
 * sgp_step_record_batched runs the step eagerly with these arguments (the
 * same meaning as in the single calls; prec: SGP_STEP_NONE, SGP_STEP_JACOBI
 * or SGP_STEP_TREE; schedule as for sgp_factor_tree) and keeps every value
 * the host reads back on the way (bounding box, edge count, the rounds of the
 * spanning tree and of the elimination schedule, the schedule's step sizes,
 * the CG's convergence polls) and every host table it uploads.  It then runs
 * the same host code again under stream capture, with each of those values
 * taken from the recording and checked on the device against the live value,
 * and instantiates the graph.  v receives the velocities, info (host,
 * [n_inst]) the solve results.  Synchronises.
 *
 * The step keeps the device pointers pos, radius, F and v: they must stay
 * allocated until the step is freed or recorded again.
 *
 * sgp_step_replay launches the graph on the context's stream.  A replay is
 * valid only for the recorded inputs: before launching, a 64-bit device-side
 * hash of pos, radius, F (and v when opts->use_x0) is compared with the
 * recorded one, and changed inputs give SGP_ESTALE without launching
 * anything (the launch sizes, buffer sizes and iteration count of the graph
 * are the recorded data's; other data could index past buffers sized for the
 * recorded contacts).  After the graph, a flag set by the device-side
 * comparisons is read back (SGP_ESTALE if any differed).  v receives the
 * velocities, info the solve results (bitwise those of the recorded run).
 * Synchronises once for the hash and once for the flag. */
enum { SGP_STEP_NONE = 0, SGP_STEP_JACOBI = 1, SGP_STEP_TREE = 2 };
int sgp_step_create(sgp_ctx ctx, sgp_step *out);
void sgp_step_free(sgp_step S);
int sgp_step_record_batched(sgp_ctx ctx, sgp_step S, int64_t n_inst, const int64_t *offsets,
                            const double *pos, const double *radius, int32_t max_deg, double g_par,
                            double g_perp, double g_med, int32_t prec, int32_t schedule, const double *F,
                            double *v, const sgp_solve_opts *opts, sgp_solve_info *info);
int sgp_step_replay(sgp_ctx ctx, sgp_step S, sgp_solve_info *info);
/* Recorded host-visible values and their total bytes (host outputs, NULL = skip). */
int sgp_step_size(sgp_step S, int64_t *values, int64_t *bytes);

/* ------------------------------------- Section 2, Steps 2 and 5 (dynamics) */

/* F_i = noise_i + sum over contacts j of k_rep w_ij (r_i - r_j) / d_ij: pairwise
 * repulsion along the line of centres plus a caller-drawn active force.
 * noise, F device [n][3]. */
int sgp_forces(sgp_ctx ctx, sgp_graph g, double k_rep, const double *noise, double *F);

/* Forward Euler, Step 5: pos += dt v (device [n][3]). */
int sgp_euler(sgp_ctx ctx, int64_t n, double dt, const double *v, double *pos);

/* ------------------------------- learned warm start (not in the paper) */

/* A message-passing network over the collision graph that maps (F, v_prev)
 * to a velocity guess for the CG (the CG to the same tolerance still decides;
 * v_prev is the fallback, see sgp_mpnn_warm_start).  Hidden width 64, three
 * layers:
 *   x_i = [F_i/sF, v_prev,i/sV]; e_p = [w_ij/sW, (r_i - r_j)/d_ij] for the
 *   neighbour entry p = (i, j);  h = relu(x W_in + b_in);
 *   per layer: m_p = relu(h_i W_a + b_m + h_j W_b + e_p W_c),
 *              a_i = sum over i's entries of m_p,  h = h + relu([h, a] W_u + b_u);
 *   v_hat = sV (h W_out + b_out).
 * Parameters: one flat FP32 vector in the order W_in(6x64) b_in(64), then per
 * layer W_a(64x64) W_b(64x64) W_c(4x64) b_m(64) W_u(128x64) b_u(64), then
 * W_out(64x3) b_out(3), all row-major.  Products run on BF16 MFMA with FP32
 * accumulation.  Two losses:
 *   Gamma given (energy):  (v_hat' G v_hat - 2 v_hat' F + v' F) / (v' F), which
 *       is ||v_hat - v||^2_G / ||v||^2_G when G v = F: the error norm that
 *       CG's convergence depends on; its gradient needs only G v_hat - F;
 *   Gamma NULL (MSE):      mean over i, components of (v_hat/sV - v/sV)^2.
 * Gamma must be the matrix assembled from the same graph g. */
int sgp_mpnn_param_count(int64_t *count);
int sgp_mpnn_create(sgp_ctx ctx, sgp_mpnn *out);
void sgp_mpnn_free(sgp_mpnn M);
/* theta: device FP32 [param_count]; copied.  Resets the Adam state.  The
 * scales must be positive. */
int sgp_mpnn_set_params(sgp_ctx ctx, sgp_mpnn M, const float *theta, double sF, double sV, double sW);
int sgp_mpnn_get_params(sgp_ctx ctx, sgp_mpnn M, float *theta);
/* v_hat [n][3] FP64 (device) from F, v_prev [n][3] FP64 (device) on graph g. */
int sgp_mpnn_forward(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, const double *F, const double *vprev,
                     double *vhat);
/* Loss and its gradient in the parameter layout (device FP32) against the
 * solved velocity v; Gamma selects the loss (above, may be NULL); loss is a
 * host pointer (may be NULL).  Synchronises. */
int sgp_mpnn_grad(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, sgp_bsr Gamma, const double *F, const double *vprev,
                  const double *v, float *grad, double *loss);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) at learning rate lr on one
 * sample; loss as above.  Synchronises. */
int sgp_mpnn_train_step(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, sgp_bsr Gamma, const double *F,
                        const double *vprev, const double *v, double lr, double *loss);
/* Initial guess for the CG: of v_prev, the network's v_hat and zero, the
 * one of lowest energy 0.5 x' Gamma x - x' F (the lower energy is the
 * smaller Gamma-norm error; zero has energy 0), preferring them in that
 * order on ties.  x0 device [n][3], may alias vprev.  used_net (host, may be
 * NULL): 0 = v_prev, 1 = the network's guess, 2 = zero; energy_net,
 * energy_prev: host outputs (may be NULL).  Synchronises. */
int sgp_mpnn_warm_start(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, sgp_bsr Gamma, const double *F,
                        const double *vprev, double *x0, int32_t *used_net, double *energy_net,
                        double *energy_prev);

/* Launch-shape knobs of this context (chosen by the autotuner):
 *  "check_every"  CG iterations per chunk (1..1024, default 2).  The host
 *                 reads the convergence state after whole chunks only: after
 *                 every chunk at first, then, from the decay of the slowest
 *                 cluster's residual so far, after as many chunks as half
 *                 the iterations it still needs; iterations issued past
 *                 convergence are no-ops on the device
 *  "tail_max"     the largest number of tree vertices whose last elimination
 *                 steps run as one LDS-resident workgroup in the tree sweeps
 *                 (0..65536, 0 disables, default 2200; used by factors built
 *                 afterwards)
 *  "graph"        1: each chunk of check_every CG iterations is captured once
 *                 per solve into a hipGraph and replayed (default 0)
 *  "spmv_waves"   waves per workgroup of the product: 2, 4 or 8 (default 4)
 *  "spmv_form"    how the CG forms Gamma p: 0 from the stored 3x3 blocks,
 *                 1 from the contacts, D_i p_i - sum_j W_ij p_j with
 *                 W_ij p = g_perp (v.v) p + (g_par - g_perp)(v.p) v for the
 *                 contact's v = sqrt(w) u (w u u^T = v v^T; default 1; fewer
 *                 bytes per product; sgp_spmv uses it too)
 *  "light_height" CONTRACT schedule: the first light_height rounds remove
 *                 leaves only; the subtrees they remove are swept by one
 *                 workgroup each, in one launch per sweep (0..1024, 0 = plain
 *                 rake-and-compress, default 0; used by factors built
 *                 afterwards)
 *  "light_cap"    vertices of such subtrees packed into one workgroup
 *                 (1..2^20, default 512); also the packing of the mid
 *                 steps' components (CONTRACT without light steps: the
 *                 steps between the first two and the tail, from the first
 *                 with at most 2^17 vertices left, are swept one workgroup
 *                 per group of components, in one launch per sweep)
 *  "fuse_step0"   1: in sgp_pcg_solve* with a tree preconditioner whose
 *                 first elimination step runs as launches of its own, that
 *                 step's forward substitution runs inside the CG's
 *                 r -= alpha q pass and its backward substitution inside the
 *                 r.z pass, on the rows each block of those passes holds
 *                 (default 1; 0: separate launches)
 *  "mid_lds"      1: the mid elimination steps (swept one workgroup per group
 *                 of components) keep the group's push slots and x in LDS
 *                 and load every constant once per launch (default 1; 0:
 *                 through global memory, step by step); bitwise the same
 *                 results
 *  "small_solve"  1: sgp_pcg_solve of one FP64 system of at most 1024 cells
 *                 with a tree preconditioner whose elimination lies wholly in
 *                 the one-workgroup tail (tail_max >= n) runs every PCG
 *                 iteration inside one workgroup, in one launch (at most
 *                 20,000 iterations; default 1; 0: a launch per kernel).  Same
 *                 product and sweeps; the dot products are summed in another
 *                 order, so results agree to CG's rounding
 *  "tail_side"    1: in sgp_pcg_solve*, while the one-workgroup tail of the
 *                 tree sweeps runs, extra workgroups of its launch do the
 *                 CG's x += alpha p (the rest of the chip would idle), and
 *                 the later vector pass only updates p (default 1; 0: x and
 *                 p in that pass)
 *  "prefetch"     1: the launch before the one-workgroup tail of the tree
 *                 sweeps also loads the tail's constants, from the XCD that
 *                 runs the tail, and the tail launch's other workgroups load
 *                 the backward mid steps' constants, so that those launches'
 *                 start-up loads hit in the caches (default 1; 0: off)
 * Unknown keys or values out of range give SGP_EINVAL.  check_every,
 * graph, fuse_step0, mid_lds, tail_side and prefetch leave every result bitwise
 * unchanged, and so does tail_max as long as the tail does not reach the first elimination
 * step (that step forms its couplings from the contacts' (w, u) when it runs
 * as its own launch, from the stored blocks inside the tail: the same values
 * up to rounding); spmv_waves changes only the summation order of the p.q
 * dot product; small_solve only that of the dot products; spmv_form,
 * light_height and light_cap change the order of roundings, so results
 * agree to rounding. */
int sgp_tune(sgp_ctx ctx, const char *key, int32_t value);
/* Current value of a knob (host output). */
int sgp_tune_get(sgp_ctx ctx, const char *key, int32_t *value);

/* Per-launch timing of the CG's product: when enabled, one product per
 * chunk of check_every CG iterations launched by sgp_pcg_solve* (the third
 * of the chunk, or its last if shorter) is bracketed by HIP events on the
 * context's stream -- an event pair around every product would itself cost
 * time.  A single solve's products issued after its last iteration return at
 * once and are not counted.  sgp_kernel_stats returns the summed duration
 * (ms) and the number of timed launches since timing was enabled (enabling
 * resets them).  Graph replay is off while timing is on. */
int sgp_kernel_timing(sgp_ctx ctx, int32_t enable);
int sgp_kernel_stats(sgp_ctx ctx, double *total_ms, int64_t *launches);

/* Duration of the last call of each phase on this context, measured with HIP
 * events on its stream, in milliseconds:
 * [0] collide, [1] assemble, [2] build_tree, [3] factor, [4] solve.
 * The phases record their events without waiting for them; this call waits
 * for the last recorded phase ends that were not read yet. */
int sgp_phase_times(sgp_ctx ctx, double *ms5);

#ifdef __cplusplus
}
#endif
#endif /* SGP_H */
