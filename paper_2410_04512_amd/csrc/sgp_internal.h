// Internal declarations of libsgp (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "sgp.h"

// ---------------------------------------------------------------- buffers

// Grow-only device buffer.  Contents are not preserved across growth.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Per-context scalar block for the PCG drivers and reductions (device).
struct PcgScalars {
    double rho, alpha, beta, pq, rr, rz, nF2, tol2, relres2;
    int32_t iter, done, status, fixed, max_iter, stop;
    // SGP_STOP_ERROR: the Gauss-Radau node mu, phi_k, S_k and phi_k rho_k
    double mu, phi, gs, gbound;
};

// The solve's stop flag, or 0 without a solve.  The address is selected
// rather than branched on, so the load can be issued early and awaited late,
// together with a kernel's first round of loads.
static __device__ int32_t k_never_done = 0;   // never written
__device__ inline int32_t done_flag(const PcgScalars *s)
{
    return *(s ? &s->done : &k_never_done);
}

// A compiler-only fence (no instruction): memory accesses written before it
// stay before it, so a branch after it cannot pull the loads above it into
// one of its arms and make them wait for the branch condition.
__device__ inline void keep_loads_above() { __asm__ __volatile__("" ::: "memory"); }

// A recorded pipeline step (sgp_step_*): every value the host read back
// during an eager run, and every block of host data it uploaded, in order.
// While a step is captured into a hipGraph the same host code runs again;
// each readback then returns the recorded value at once and enqueues a
// device-side comparison of the live value with it instead (a mismatch sets
// `flag`: the data no longer has the recorded structure), and each upload
// copies the recorded block from `arena` (device) so the graph holds no
// pointer to host memory.
enum { PLAN_OFF = 0, PLAN_RECORD = 1, PLAN_CAPTURE = 2 };
struct StepPlan {
    std::vector<uint8_t> bytes;   // recorded values back to back
    std::vector<size_t> off, len;
    std::vector<uint8_t> kind;    // 0: read back by the host, 1: uploaded by the host
    size_t pos = 0;               // next entry while capturing
    DevBuf arena;                 // device copy of `bytes`
    DevBuf flag;                  // int32: 1 once a live value differed from the recorded one
};

struct sgp_ctx_ {
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    unsigned *tickets = nullptr;   // device counters for last-block reductions (kept at 0 between uses)
    int n_tickets = 0;
    void *pinned = nullptr;        // small pinned host block for readbacks
    hipEvent_t poll_ev = nullptr;  // the CG's poll readback (created on first use)
    DevBuf ws[24];                 // scratch workspaces (by role index)
    hipEvent_t ev[12] = {};
    float phase_ms[5] = {0, 0, 0, 0, 0};
    bool phase_pending[5] = {false, false, false, false, false};   // end recorded, time not read yet
    // per-launch timing of the CG's matrix product (events on ctx->stream)
    int ktiming = 0;
    std::vector<hipEvent_t> kev;   // pairs (start, stop)
    hipEvent_t kt_start = nullptr, kt_stop = nullptr;   // the pair the next product launch carries
    bool kt_used = false;          // a launch took that pair
    std::vector<int32_t> kev_iter; // CG iteration index (from 0) of each pair's launch
    int kev_used = 0;
    double ktime_ms = 0.0;
    int64_t klaunches = 0;
    // launch-shape knobs (sgp_tune); none changes a result beyond rounding order
    int check_every = 2;           // CG iterations per chunk (the host polls after whole chunks)
    int tail_max = 2200;           // vertices at most left for the one-workgroup tail of the tree sweeps
    int use_graph = 0;             // replay a captured chunk of CG iterations as one hipGraph
    int spmv_waves = 4;            // waves per workgroup of the block-CSR product (2, 4 or 8)
    int spmv_form = 1;             // product from the 3x3 blocks (0) or from the contacts' (w, u) (1)
    int fuse_step0 = 1;            // CG: first elimination step inside the vector passes around the sweeps
    int small_solve = 1;           // one-workgroup PCG for small single systems (small.hip)
    int mid_lds = 1;               // tree sweeps: the mid steps' slots and x in LDS (factor.hip)
    int tail_side = 1;             // CG: x += alpha p by extra workgroups of the one-workgroup tail launch
    int prefetch = 1;              // tree sweeps: the tail's and the backward mid steps' constants loaded ahead
    int light_height = 0;          // rake rounds whose subtrees the sweeps handle one workgroup each (0: off)
    int light_cap = 512;           // vertices of such subtrees packed into one workgroup
    hipStream_t cap_stream = nullptr;   // private stream for graph capture (created on first use)
    int contact_model = SGP_CONTACT_OVERLAP;   // what collide stores as a contact's w
    int plan_mode = PLAN_OFF;      // recording or capturing a step (sgp_step_*)
    StepPlan *plan = nullptr;
};

// event pair around one timed launch of CG iteration `iter` (no-op unless
// timing is on)
int ktimer_begin(sgp_ctx ctx, int32_t iter);
int ktimer_end(sgp_ctx ctx);
// synchronises: adds the finished pairs to the totals, except those of
// iterations >= iters_done (launched after convergence, which return at once)
int ktimer_flush(sgp_ctx ctx, int32_t iters_done);

// workspace slots (shared scratch of a context; each call may reuse them)
enum {
    WS_KEY_A, WS_KEY_B, WS_VAL_A, WS_VAL_B, WS_HIST, WS_TILES, WS_SLOTS, WS_DEG, WS_TMP0, WS_TMP1,
    WS_TMP2, WS_TMP3, WS_TMP4, WS_TMP5, WS_TMP6, WS_TMP7, WS_PART, WS_SCAL, WS_TMP8, WS_TMP9,
    WS_PAIR,   // a few words gathered for one readback
    WS_COUNT
};

// The graph is kept in the caller's numbering (canonical edge ids).  perm/inv
// give the library's internal vertex order -- the cell-list order of the last
// collide (cluster-major, then cell, then id) -- in which Gamma, the CG
// vectors and the tree sweeps' gathers are laid out for locality:
// internal i <-> caller perm[i], caller u <-> internal inv[u].
struct sgp_graph_ {
    int64_t n = 0, m = 0, n_inst = 1;
    uint64_t version = 0;   // changes whenever a collide rewrites the graph
    DevBuf rowptr, col, ent_edge, ei, ej, wu, inst_off, inst_of;
    DevBuf w;   // the contacts' w alone (dense, for passes that read only w)
    DevBuf perm, inv;
    std::vector<int64_t> h_inst_off;
};

// Gamma in block CSR: rowptr/bcol as usual; the symmetric blocks keep their 6
// distinct entries in 64-block groups (see spmv.hip for the layout).
struct sgp_bsr_ {
    int64_t n = 0, nnzb = 0;
    uint64_t gen = 0;   // new at every assembly (next_gen)
    DevBuf rowptr, bcol, val, val32, diagpos;   // internal order; bcol, val, diagpos only once have_blocks
    bool have_blocks = false;                   // the 3x3 blocks assembled (bsr_blocks)
    bool have_val32 = false;                    // their FP32 copy
    uint64_t src_version = 0;                   // the graph's version at assembly
    DevBuf perm, inv;                           // copy of the graph's order
    sgp_graph src = nullptr;                    // graph it was assembled from (canonical export)
    double gpar = 0, gperp = 0, gmed = 0;
    DevBuf wrow;          // first row of every product wave
    // edge form of the same matrix (internal order): the off-diagonal entries
    // of row i are rowptr[i] - i + c (c < degree; the diagonal block is the
    // last of every block row); per entry its column and v = sqrt(w) u in
    // 64-entry groups of EDGE_PLANES planes; the diagonal blocks as 64-row
    // groups of 6 planes
    DevBuf ecol, ew, dg, ew32, dg32, ewrow;
    int64_t enwaves = 0;
    int64_t nwaves = 0;
    bool have32 = false;
};

inline int64_t sym_group_size(int64_t nnzb) { return ((nnzb + 63) / 64) * 384; }   // values incl. padding
// the edge form keeps per entry v = sqrt(w) u of its contact (w = v.v), in
// 64-entry groups of EDGE_PLANES planes
constexpr int EDGE_PLANES = 3;
inline int64_t edge_group_size(int64_t ne) { return ((ne + 63) / 64) * 64 * EDGE_PLANES; }   // v incl. padding

struct sgp_tree_ {
    int64_t n = 0, nt = 0, n_roots = 0;
    int32_t max_depth = 0;
    DevBuf tree_edge, parent, pedge, depth, comp;
    DevBuf tptr, tadj, tadje;   // forest incidence: rows of tree neighbours, ascending edge id
    // local forest (sgp_build_forest): cells per cluster (0: a spanning
    // forest of the whole graph), the cluster of every cell (caller numbering)
    int32_t cluster_size = 0;
    int64_t n_clusters = 0;
    DevBuf cluster;
};

// clusters of the local forest: Z-order runs of K cells per instance (collide.hip)
int forest_partition(sgp_ctx ctx, sgp_graph g, const double *pos, const double *radius, int32_t K,
                     int32_t *cluster, int64_t *n_clusters);

enum { PREC_NONE = 0, PREC_JACOBI = 1, PREC_TREE = 2 };

struct sgp_prec_ {
    int kind = PREC_NONE;
    uint64_t gen = 0;   // new at every factorisation (next_gen)
    // the one-workgroup solve's copy of a matrix's entries (small.hip), for
    // the matrix of generation small_a_gen and this factor's generation
    DevBuf small_ell;
    uint64_t small_a_gen = 0, small_m_gen = 0;
    int32_t small_deg = 0;
    int64_t n = 0;
    int schedule = 0;
    int32_t steps = 0;
    std::vector<int32_t> h_step_ptr;   // [steps+1] elimination-index ranges of each step
    DevBuf elim, pos, up, in_ptr, in_src, F, Dinv, y;   // tree (F: [n][2][9], Dinv: [n][6])
    DevBuf elim_int;                                    // elim in the internal order
    DevBuf perm, inv;                                   // copy of the graph's internal order
    DevBuf tout, cs;                                    // push slots: in-list position of (q,k); slot values [n_in][3]
    DevBuf step_ptr;                                    // device copy of h_step_ptr
    int32_t light_steps = 0, light_nwg = 0;             // steps < light_steps: subtrees, one workgroup each
    DevBuf light_ptr;                                   // [light_steps * light_nwg + 1] first q of (step, workgroup)
    int32_t mid_step0 = 0, mid_steps = 0, mid_nwg = 0;  // steps mid_step0.. +mid_steps: components, one workgroup each
    DevBuf mid_ptr;                                     // [mid_steps * mid_nwg + 1] first q of (step, workgroup)
    DevBuf mid_tab;                                     // tables of the LDS mid sweeps (factor.hip, MidTab)
    bool mid_lds_built = false, mid_lds = false;        // built, and every group fits the LDS sweeps
    int32_t tail_step = 0;                              // steps >= tail_step run in one workgroup
    int32_t tail_nt = 0, tail_ni = 0;                   // tail vertices, tail-internal push slots
    DevBuf tail_iptr, tail_tslot;                       // per tail target: first internal slot; per (q,k): its slot
    DevBuf tail_b;                                      // [tail_nt][3] right-hand sides entering the tail
    // the first step's couplings as the contacts' (w, u) (nothing has been
    // eliminated before it, so each is -W_e of a tree edge): planes
    // [2][n_wu0][4], read by the first step of the sweeps instead of F
    DevBuf wu0, wu032;
    int64_t n_wu0 = 0;
    bool step0_sorted = false;   // positions 0..n_wu0-1 ascend in the internal order
    double gpar = 0, gperp = 0, gmed = 0;
    DevBuf F32, Dinv32, y32, cs32;                      // FP32 copies for the refinement inner solve
    bool have32 = false;
    DevBuf jdinv;                                       // Jacobi: [n][6]
    // augmented tree (sgp_factor_augmented): the tree factor above is the
    // inner preconditioner; P' = its tree's Laplacian plus the added contacts
    int aug = 0;
    double inner_rtol = 0.1;
    int32_t aug_parts = 0;
    int64_t aug_pieces = 0, aug_added = 0;
    DevBuf aug_piece, aug_list;                         // head of every cell's piece; added edge ids ascending
    DevBuf aug_tptr, aug_tadj, aug_twu;                 // tree rows (caller numbering): neighbour (internal), (w, u)
    DevBuf aug_ptr, aug_adj, aug_wu;                    // added-contact rows, the same
};

// the augmented tree's flexible CG (augment.hip); F and x in the internal order
int solve_augmented(sgp_ctx ctx, sgp_bsr A, sgp_prec M, const double *F, double *x, const sgp_solve_opts *o,
                    sgp_solve_info *info);

// ---------------------------------------------------------------- errors

int set_err(sgp_ctx ctx, int code, const char *fmt, ...);

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e__ = (expr);                                                            \
        if (e__ != hipSuccess)                                                              \
            return set_err((ctx), SGP_EHIP, "%s failed: %s (%s:%d)", #expr,                 \
                           hipGetErrorString(e__), __FILE__, __LINE__);                     \
    } while (0)

#define LAUNCH_CHECK(ctx) HIP_TRY(ctx, hipGetLastError())

#define SGP_TRY(expr)              \
    do {                           \
        int s__ = (expr);          \
        if (s__ != SGP_OK) return s__; \
    } while (0)

int ensure(sgp_ctx ctx, DevBuf &b, size_t bytes);
template <class T>
inline int ensure_t(sgp_ctx ctx, DevBuf &b, size_t count, T **out)
{
    int s = ensure(ctx, b, count * sizeof(T) + 64);
    *out = (T *)b.p;
    return s;
}
void release(DevBuf &b);
int readback(sgp_ctx ctx, void *host, const void *dev, size_t bytes);   // synchronises
// host -> device copy of a small block of host data (ordered on the stream)
int upload(sgp_ctx ctx, void *dev, const void *host, size_t bytes);

// end of phase k (0 collide, 1 assemble, 2 build_tree, 3 factor, 4 solve):
// its events are ev[2k], ev[2k+1]; the time is read when it is asked for, so
// the host does not wait for the phase here
inline void phase_begin(sgp_ctx ctx, int k)
{
    if (ctx && ctx->ev[2 * k] && ctx->plan_mode != PLAN_CAPTURE) (void)hipEventRecord(ctx->ev[2 * k], ctx->stream);
}
inline void phase_end(sgp_ctx ctx, int k)
{
    if (!ctx->ev[2 * k + 1] || ctx->plan_mode == PLAN_CAPTURE) return;
    (void)hipEventRecord(ctx->ev[2 * k + 1], ctx->stream);
    ctx->phase_pending[k] = true;
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads) ? (unsigned)((n + threads - 1) / threads) : 1u; }

// ---------------------------------------------------------------- primitives (util.hip)

// out[0..n] = exclusive prefix sum of in[0..n-1]; out[n] = total.  in may alias out.
int scan_exclusive(sgp_ctx ctx, const int32_t *in, int32_t *out, int64_t n);
// Stable LSD radix sort of (key, val) pairs on the low key_bits bits.  tmp buffers of n.
int radix_sort_pairs(sgp_ctx ctx, uint32_t *keys, int32_t *vals, uint32_t *ktmp, int32_t *vtmp,
                     int64_t n, int key_bits);
int fill_i32(sgp_ctx ctx, int32_t *p, int32_t v, int64_t n);
int fill_f64(sgp_ctx ctx, double *p, double v, int64_t n);
int iota_i32(sgp_ctx ctx, int32_t *p, int64_t n);

// The CG's x += alpha p, handed to the tree sweeps: while the tail's single
// workgroup runs its chain of dependent steps, the rest of the chip idles, so
// extra workgroups of the same launch stream this update meanwhile.  The
// rows are the CG's vector blocks (row0, row1, cluster per block); a block
// is updated while its cluster's done mark is 0, as in the CG's own pass.
constexpr int SIDE_BLOCK_VALUES = 1024;   // values of one vector block at most
struct SideX {
    void *x;               // T[3 n], internal order
    const void *p;         // T[3 n]
    const int32_t *row0, *row1, *inst;
    const PcgScalars *S;
    int32_t nb;            // vector blocks
    int32_t nwg;           // extra workgroups
    bool ran;              // set by the sweeps when the update was launched
    // filled by the sweeps (knob prefetch): after the update, the same
    // workgroups load the backward mid steps' constants ahead, from the XCD
    // that will sweep them (mid_L = 0: none)
    const int32_t *mid_wptr, *mid_lup;
    int32_t mid_L, mid_nwg, mid_Q0, never;
    int32_t wait;          // sleep ~7 us before either job (the tail's constants not prefetched)
};

// shared by several translation units
// r, z in the internal order (used by the CG)
int prec_apply_f64(sgp_ctx ctx, sgp_prec M, const double *r, double *z, PcgScalars *s, bool skip0 = false,
                   SideX *side = nullptr);
int permute_rows(sgp_ctx ctx, const int32_t *idx, const double *src, double *dst, int64_t n, int scatter);
int copy_order(sgp_ctx ctx, DevBuf &dperm, DevBuf &dinv, const DevBuf &sperm, const DevBuf &sinv, int64_t n);
int prec_apply_f32(sgp_ctx ctx, sgp_prec M, const float *r, float *z, PcgScalars *s, bool skip0 = false,
                   SideX *side = nullptr);
int32_t prec_step0_launch(sgp_prec M);
// Gamma's 3x3 blocks (block-CSR product), assembled on first use
int bsr_blocks(sgp_ctx ctx, sgp_bsr A);
// a number no earlier call returned (generations of matrices and factors)
uint64_t next_gen();
// the whole PCG of one small system in one workgroup (small.hip)
bool small_solve_fits(sgp_ctx ctx, sgp_bsr A, sgp_prec M);
int solve_small(sgp_ctx ctx, sgp_bsr A, sgp_prec M, const double *F, double *x, const sgp_solve_opts *o,
                PcgScalars *S);
// cells at most for sgp_prec_apply_noalloc (its static scratch holds two
// [n][3] FP64 vectors: 48 MiB per device)
constexpr int64_t NOALLOC_MAX_CELLS = (int64_t)1 << 20;
// device address of that scratch on the context's device, taken once per device
int noalloc_scratch_init(sgp_ctx ctx);
int prec_make32(sgp_ctx ctx, sgp_prec M);
int tail_setup_attr(sgp_ctx ctx);
int bsr_make32(sgp_ctx ctx, sgp_bsr A);
int bsr_prepare(sgp_ctx ctx, sgp_bsr A);
int spmv_blocks(sgp_ctx ctx, sgp_bsr A);
uint64_t next_graph_version();   // process-wide, strictly increasing
int spmv_f64(sgp_ctx ctx, sgp_bsr A, const double *x, double *y, const PcgScalars *S, double *part, int mode);
int spmv_f32(sgp_ctx ctx, sgp_bsr A, const float *x, float *y, const PcgScalars *S, double *part, int mode);

// ---------------------------------------------------------------- device helpers

#define SGP_DEV __device__ __forceinline__

constexpr int RED_BLOCKS = 512;     // fixed grid of the deterministic reductions
constexpr int RED_THREADS = 256;

// Workgroup barrier that orders LDS only: waits for the wave's LDS accesses,
// not for its global loads, so loads whose results are not needed yet stay
// in flight across it.  For code whose threads exchange data through LDS
// alone (global memory written before it is not read after it by others).
SGP_DEV void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wave-level counterpart of lds_barrier: orders the LDS accesses of the
// lanes of one wave (for steps that only one wave works on).
SGP_DEV void lds_wave_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Sum over a 256-thread block in a fixed order; result valid in thread 0.
SGP_DEV double block_sum_256(double v, double *sh)
{
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) sh[t] = sh[t] + sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Last-block detection for the two-stage reductions: every block writes its
// partial, then takes a ticket; the block holding the last ticket sees all
// partials (device-scope release/acquire through the fences) and resets the
// counter for the next use.
SGP_DEV bool last_block(unsigned *ticket, unsigned nblocks, int *sh_flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned t = atomicAdd(ticket, 1u);
        *sh_flag = (t == nblocks - 1);
        if (*sh_flag) {
            __threadfence();
            *ticket = 0u;
        }
    }
    __syncthreads();
    return *sh_flag != 0;
}

// Fixed-order sum of n partials by one 256-thread block; result in thread 0.
SGP_DEV double sum_partials(const double *part, int n, double *sh)
{
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) v = v + part[k];
    return block_sum_256(v, sh);
}

// XCD-aware block order.  The dispatcher deals workgroups round-robin to the
// 8 XCDs (each with its own L2), so workgroup b runs on XCD b % 8.  Mapping b
// to the logical block below gives every XCD one contiguous run of logical
// blocks, so the neighbours a run gathers stay in that XCD's L2 instead of
// being fetched by all eight.  A bijection of [0, nb) for any nb.
constexpr int NUM_XCD = 8;
SGP_DEV int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t q = nb / NUM_XCD, r = nb % NUM_XCD;
    const int64_t x = b % NUM_XCD, i = b / NUM_XCD;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// --- 3x3 blocks: full row-major [9]; symmetric packed [6] = (00,01,02,11,12,22)

SGP_DEV void sym_unpack(const double *s, double *f)
{
    f[0] = s[0]; f[1] = s[1]; f[2] = s[2];
    f[3] = s[1]; f[4] = s[3]; f[5] = s[4];
    f[6] = s[2]; f[7] = s[4]; f[8] = s[5];
}

// Inverse of an SPD 3x3 block through its Cholesky factor C (D = C C^T);
// returns false on a non-positive or non-finite pivot.  Result packed sym.
SGP_DEV bool spd_inverse3(const double *D, double *inv6)
{
    double c00 = D[0];
    if (!(c00 > 0.0) || !isfinite(c00)) return false;
    c00 = sqrt(c00);
    double c10 = D[3] / c00, c20 = D[6] / c00;
    double c11 = D[4] - c10 * c10;
    if (!(c11 > 0.0) || !isfinite(c11)) return false;
    c11 = sqrt(c11);
    double c21 = (D[7] - c20 * c10) / c11;
    double c22 = D[8] - c20 * c20 - c21 * c21;
    if (!(c22 > 0.0) || !isfinite(c22)) return false;
    c22 = sqrt(c22);
    // inverse of C (lower triangular)
    double i00 = 1.0 / c00, i11 = 1.0 / c11, i22 = 1.0 / c22;
    double i10 = -c10 * i00 * i11;
    double i21 = -c21 * i11 * i22;
    double i20 = -(c20 * i00 + c21 * i10) * i22;
    // D^{-1} = C^{-T} C^{-1}
    inv6[0] = i00 * i00 + i10 * i10 + i20 * i20;
    inv6[1] = i10 * i11 + i20 * i21;
    inv6[2] = i20 * i22;
    inv6[3] = i11 * i11 + i21 * i21;
    inv6[4] = i21 * i22;
    inv6[5] = i22 * i22;
    return true;
}

template <class T>
SGP_DEV void sym_mv(const T *s, T x0, T x1, T x2, T &y0, T &y1, T &y2)
{
    y0 = s[0] * x0 + s[1] * x1 + s[2] * x2;
    y1 = s[1] * x0 + s[3] * x1 + s[4] * x2;
    y2 = s[2] * x0 + s[4] * x1 + s[5] * x2;
}

// -W p for the block W = w (g_perp I + (g_par - g_perp) u u^T) of contact
// e = (w, u): the coupling of a first-step vertex, from 4 values instead of 9
template <class T>
SGP_DEV void neg_w_mv(const T *e, T gpar, T gperp, T p0, T p1, T p2, T &o0, T &o1, T &o2)
{
    const T w = e[0], u0 = e[1], u1 = e[2], u2 = e[3];
    const T c = (gpar - gperp) * ((u0 * p0 + u1 * p1) + u2 * p2);
    o0 = -(w * (gperp * p0 + c * u0));
    o1 = -(w * (gperp * p1 + c * u1));
    o2 = -(w * (gperp * p2 + c * u2));
}

// The pivot solve of a first-step vertex with at most one tree edge (a leaf,
// or a lone vertex: w = 0): its pivot is P_qq = g_med I + W_e =
// c I + d u u^T with c = g_med + w g_perp, d = w (g_par - g_perp), whose
// inverse is I / c - d / (c (c + d)) u u^T (|u| = 1), so it needs no stored
// inverse; a compressed vertex (two tree edges) uses its stored one.
template <class T>
SGP_DEV void leaf_pivot_solve(const T *e, T gpar, T gperp, T gmed, T b0, T b1, T b2, T &o0, T &o1, T &o2)
{
    const T w = e[0], u0 = e[1], u1 = e[2], u2 = e[3];
    const T c = gmed + w * gperp, cd = gmed + w * gpar;
    const T beta = (w * (gpar - gperp)) / (c * cd);
    const T ub = beta * ((u0 * b0 + u1 * b1) + u2 * b2);
    o0 = b0 / c - ub * u0;
    o1 = b1 / c - ub * u1;
    o2 = b2 / c - ub * u2;
}

// W_e p of the block W_e = w (g_perp I + (g_par - g_perp) u u^T) of a
// contact stored as v = sqrt(w) u: W_e p = g_perp (v.v) p + (g_par - g_perp)
// (v.p) v (eq. cell_cell_friction with w = v.v and w u u^T = v v^T)
template <class T>
SGP_DEV void edge_wp(T v0, T v1, T v2, T x0, T x1, T x2, T gpar, T gperp, T &o0, T &o1, T &o2)
{
    const T ww = gperp * ((v0 * v0 + v1 * v1) + v2 * v2);
    const T c = (gpar - gperp) * ((v0 * x0 + v1 * x1) + v2 * x2);
    o0 = ww * x0 + c * v0;
    o1 = ww * x1 + c * v1;
    o2 = ww * x2 + c * v2;
}

// c = a * b (full 3x3)
SGP_DEV void mm3(const double *a, const double *b, double *c)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            c[3 * i + j] = a[3 * i + 0] * b[0 + j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}
