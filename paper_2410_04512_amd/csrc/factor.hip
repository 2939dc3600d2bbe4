// Section 3.3 (Alg. 2, TreeLDLT) and Appendix B.1 (tree solves) on the GPU.
//
// The factorisation is driven by an elimination schedule: a partition of the
// vertices into steps such that every vertex is eliminated after the
// vertices it is connected to from below.  Each vertex v records the (at most
// two) vertices it is still connected to when eliminated -- up0 (toward the
// root) and, for a chain vertex removed by compress, up1 (its one child).
// With the vertices renumbered in elimination order q, P = L D L^T where row
// q of L^T has the blocks L_{up_k(q), q} = A_{up_k, q} D_q^{-1}.  We store
//    Dinv[q]   = D_q^{-1}            (symmetric, packed 6)
//    F[k][q]   = A_{up_k(q), q}      (full 3x3, the coupling at elimination; two
//                                   planes of n blocks, so the many vertices
//                                   with one up-link never fetch a second block)
// and solve P x = b as
//    forward   y_q = D_q^{-1} (b_q - sum_{(u,k): up_k(u) = q} F[u][k] y_u)
//    backward  x_q = y_q - D_q^{-1} sum_k F[q][k]^T x_{up_k(q)}
// which is ForwardSolve, DiagSolve and BackwardSolve of Appendix B.1 with
// the pivot solve folded into each sweep.  The forward sweep pushes: once y_u
// is known, u writes F[u][k] y_u into the slot its target reads (the target's
// in-list entries are contiguous), so a target sums a run of slots in a fixed
// order instead of chasing source indices.
//
// Schedules:
//  LEVEL     step = max depth - depth: Alg. 2's order (decreasing distance
//            to the root); up0 = parent.  One step per tree level.
//  CONTRACT  rake and compress (tree contraction): in one step every current
//            leaf is eliminated into its parent, and an independent set of
//            one-child vertices whose child is not a leaf is eliminated,
//            joining parent and child by the Schur block
//            A'_{p,c} = -A_{p,v} D_v^{-1} A_{v,c}.  The forest stays a forest
//            (no fill beyond one block per removed chain vertex) and the
//            number of steps is O(log n) instead of the tree depth.
#include "sgp_internal.h"

#include <algorithm>
#include <climits>
#include <mutex>

// ---------------------------------------------------------------- W and P_ii

SGP_DEV void friction_block_dev(double w, double ux, double uy, double uz, double gpar, double gperp,
                                double *W)
{
    const double u[3] = {ux, uy, uz};
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double uu = u[a] * u[b];
            double id = (a == b) ? 1.0 : 0.0;
            W[3 * a + b] = w * (gpar * uu + gperp * (id - uu));
        }
}

// P_vv = g_med I + sum of W_e over the tree edges at v, ascending edge id;
// E_v = A_{parent(v), v} = -W_{pedge(v)} (zero at roots).
__global__ void k_tree_blocks(int64_t n, const int32_t *tptr, const int32_t *tadje, const int32_t *pedge,
                              const double4 *wu, double gpar, double gperp, double gmed, double *Pd,
                              double *E)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    // the parent edge's (w, u) is loaded before the first store (a load
    // behind a store waits for it)
    const int32_t e = pedge[v];
    const double4 qe = wu[e >= 0 ? e : 0];
    double P[9];
    for (int t = 0; t < 9; t++) P[t] = (t % 4 == 0) ? gmed : 0.0;
    for (int32_t k = tptr[v]; k < tptr[v + 1]; k++) {
        double4 q = wu[tadje[k]];
        double W[9];
        friction_block_dev(q.x, q.y, q.z, q.w, gpar, gperp, W);
        for (int t = 0; t < 9; t++) P[t] = P[t] + W[t];
    }
    for (int t = 0; t < 9; t++) Pd[9 * v + t] = P[t];
    if (e >= 0) {
        const double4 q = qe;
        double W[9];
        friction_block_dev(q.x, q.y, q.z, q.w, gpar, gperp, W);
        for (int t = 0; t < 9; t++) E[9 * v + t] = -W[t];
    } else {
        for (int t = 0; t < 9; t++) E[9 * v + t] = 0.0;
    }
}

// ---------------------------------------------------------------- schedules

// (w, u) of the first step's couplings: plane 0 the edge to the up-link
// (the tree parent), plane 1 for a compressed vertex the edge from its child
__global__ void k_step0_wu(int32_t q1, const int32_t *elim, const int32_t *upq, const int32_t *pedge,
                           const double4 *wu, double4 *out)
{
    const int32_t q = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= q1) return;
    const int32_t pe = pedge[elim[q]];
    out[q] = pe >= 0 ? wu[pe] : make_double4(0.0, 0.0, 0.0, 0.0);
    const int32_t qb = upq[2 * q + 1];
    out[q1 + q] = qb >= 0 ? wu[pedge[elim[qb]]] : make_double4(0.0, 0.0, 0.0, 0.0);
}

__global__ void k_sched_level(int64_t n, const int32_t *depth, const int32_t *parent, int32_t maxd,
                              int32_t *stepv, int32_t *up0, int32_t *up1)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    stepv[v] = maxd - depth[v];
    up0[v] = parent[v];
    up1[v] = -1;
}

__global__ void k_contract_init(int64_t n, const int32_t *parent, int32_t *par, int32_t *nch, int32_t *xch,
                                int32_t *stepv)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t p = parent[v];
    par[v] = p;
    stepv[v] = -1;
    if (p >= 0) {
        atomicAdd(&nch[p], 1);
        atomicXor(&xch[p], (int32_t)v);
    }
}

SGP_DEV uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// priority of v in step s: a hash, ties by id (a strict order)
SGP_DEV bool beats(int32_t a, int32_t b, int32_t s)
{
    uint32_t ha = mix32((uint32_t)a * 0x9e3779b1u ^ (uint32_t)s * 0x85ebca77u);
    uint32_t hb = mix32((uint32_t)b * 0x9e3779b1u ^ (uint32_t)s * 0x85ebca77u);
    return ha != hb ? ha > hb : a > b;
}

__global__ void k_contract_select(int64_t n, int32_t s, const int32_t *par, const int32_t *nch,
                                  const int32_t *xch, int32_t *stepv, int32_t *up0, int32_t *up1)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || stepv[v] >= 0) return;
    int32_t p = par[v], c0 = nch[v];
    if (c0 == 0) {   // leaf (rake) or a lone root (final)
        stepv[v] = s;
        up0[v] = p;
        up1[v] = -1;
        return;
    }
    if (c0 != 1 || p < 0) return;
    int32_t c = xch[v];
    if (nch[c] == 0) return;   // its child is a leaf: it is raked first
    bool unary_p = nch[p] == 1 && par[p] >= 0;
    bool unary_c = nch[c] == 1 && par[c] >= 0;
    if (unary_p && !beats((int32_t)v, p, s)) return;
    if (unary_c && !beats((int32_t)v, c, s)) return;
    stepv[v] = s;
    up0[v] = p;
    up1[v] = c;
}

__global__ void k_contract_apply(int64_t n, int32_t s, const int32_t *stepv, const int32_t *up0,
                                 const int32_t *up1, int32_t *par, int32_t *nch, int32_t *xch)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || stepv[v] != s) return;
    int32_t p = up0[v], c = up1[v];
    if (c >= 0) {
        par[c] = p;
        atomicXor(&xch[p], (int32_t)v ^ c);
    } else if (p >= 0) {
        atomicSub(&nch[p], 1);
        atomicXor(&xch[p], (int32_t)v);
    }
}

// Progress of the schedule without a counter that every vertex increments
// (atomics on one address serialise): per block the vertices still
// unscheduled and the largest step given so far, then one block combines.
constexpr int SCHED_STAT_BLOCKS = 1024;

__global__ __launch_bounds__(256) void k_sched_stats(int64_t n, const int32_t *stepv, int32_t *part)
{
    __shared__ int32_t sa[4], sm[4];
    int32_t alive = 0, mx = -1;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        const int32_t st = stepv[v];
        alive += st < 0;
        mx = st > mx ? st : mx;
    }
    for (int o = 32; o > 0; o >>= 1) {
        alive += __shfl_xor(alive, o, 64);
        const int32_t m2 = __shfl_xor(mx, o, 64);
        mx = m2 > mx ? m2 : mx;
    }
    if ((threadIdx.x & 63) == 0) {
        sa[threadIdx.x >> 6] = alive;
        sm[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa[0] + sa[1] + sa[2] + sa[3];
        int32_t m = sm[0];
        for (int k = 1; k < 4; k++) m = sm[k] > m ? sm[k] : m;
        part[2 * blockIdx.x + 1] = m;
    }
}

// out[0]: vertices unscheduled, out[1]: largest step given (-1: none)
__global__ __launch_bounds__(256) void k_sched_final(int nb, const int32_t *part, int32_t *out)
{
    __shared__ int32_t sa[256], sm[256];
    int32_t alive = 0, mx = -1;
    for (int b = threadIdx.x; b < nb; b += 256) {
        alive += part[2 * b];
        mx = part[2 * b + 1] > mx ? part[2 * b + 1] : mx;
    }
    sa[threadIdx.x] = alive;
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            sa[threadIdx.x] += sa[threadIdx.x + st];
            sm[threadIdx.x] = sm[threadIdx.x + st] > sm[threadIdx.x] ? sm[threadIdx.x + st] : sm[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sa[0];
        out[1] = sm[0];
    }
}

// The first round's changes, pulled by every surviving vertex from its
// children in the tree (the same sums as k_contract_apply's atomics: XOR and
// counts commute, so the state is identical bit for bit).  Before round 0 the
// children of p are exactly its tree neighbours whose parent is p.
__global__ void k_contract_pull0(int64_t n, const int32_t *parent, const int32_t *tptr, const int32_t *tadj,
                                 const int32_t *stepv, const int32_t *up0, const int32_t *up1, int32_t *par,
                                 int32_t *nch, int32_t *xch)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || stepv[p] == 0) return;
    int32_t nc = nch[p], xc = xch[p];
    for (int32_t t = tptr[p]; t < tptr[p + 1]; t++) {
        const int32_t v = tadj[t];
        if (parent[v] != (int32_t)p || stepv[v] != 0) continue;
        const int32_t c = up1[v];
        if (c < 0) {
            nc -= 1;
            xc ^= v;
        } else {
            xc ^= v ^ c;
        }
    }
    nch[p] = nc;
    xch[p] = xc;
    const int32_t pp = par[p];
    if (pp >= 0 && stepv[pp] == 0 && up1[pp] == (int32_t)p) par[p] = up0[pp];
}

// ---- light subtrees (CONTRACT with a rake-only start)
//
// The first rounds eliminate only leaves (rake), so after H rounds the
// eliminated vertices are exactly those of height < H: whole subtrees hanging
// off the remaining tree.  Each such subtree is handed to one workgroup of the
// sweeps (several subtrees per workgroup, packed in the internal order up to
// light_cap vertices), which walks the H steps with a barrier between them:
// one launch per sweep instead of H.

__global__ void k_rake_select(int64_t n, int32_t s, const int32_t *par, const int32_t *nch, int32_t *stepv,
                              int32_t *up0, int32_t *up1)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || stepv[v] >= 0 || nch[v] != 0) return;
    stepv[v] = s;
    up0[v] = par[v];
    up1[v] = -1;
}

// jr[v]: v's parent if v and its parent are light, v itself for the root of a
// light subtree, -1 for a vertex that is not light
__global__ void k_light_init(int64_t n, const int32_t *parent, const int32_t *stepv, int32_t *jr)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (stepv[v] < 0) {
        jr[v] = -1;
        return;
    }
    const int32_t p = parent[v];
    jr[v] = (p >= 0 && stepv[p] >= 0) ? p : (int32_t)v;
}

__global__ void k_light_jump(int64_t n, const int32_t *a, int32_t *b)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t j = a[v];
    b[v] = j >= 0 ? a[j] : -1;
}

__global__ void k_light_count(int64_t n, const int32_t *jr, int32_t *cnt)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (jr[v] >= 0) atomicAdd(&cnt[jr[v]], 1);
}

// subtree sizes of the light roots, walked in the internal order
__global__ void k_light_vals(int64_t n, const int32_t *perm, const int32_t *jr, const int32_t *cnt, int32_t *val)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = perm[i];
    val[i] = jr[v] == v ? cnt[v] : 0;
}

// workgroup of a light root: its first vertex's rank among all light vertices / cap
__global__ void k_light_rootwg(int64_t n, const int32_t *perm, const int32_t *jr, const int32_t *start, int32_t cap,
                               int32_t *wgr)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = perm[i];
    if (jr[v] == v) wgr[v] = start[i] / cap;
}

__global__ void k_light_wg(int64_t n, const int32_t *jr, const int32_t *wgr, int32_t *wgv)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    wgv[v] = jr[v] >= 0 ? wgr[jr[v]] : 0;
}

// first q of every (light step, workgroup) key below lim; keys sorted
__global__ void k_light_ptr(int64_t n, const uint32_t *key, int64_t lim, int32_t *wptr)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q > n) return;
    const int64_t lo = q == 0 ? -1 : (int64_t)key[q - 1];
    int64_t hi = q == n ? lim : (int64_t)key[q];
    if (hi > lim) hi = lim;
    for (int64_t k = lo + 1; k <= hi; k++) wptr[k] = (int32_t)q;
}

// ---- mid steps grouped by component (CONTRACT without light steps)
//
// The steps between the first, large ones and the tail hold few vertices
// each, and their vertices, joined by their up-links, fall apart into small
// components (the pieces of the tree hanging below the tail's vertices: tens
// of vertices each).  Every push and every read of x between steps stays
// inside a component or goes to the tail, so each component is handed to one
// workgroup of the sweeps (packed in the internal order up to light_cap
// vertices), which walks those steps with a barrier between them, with the
// kernels of the light subtrees: one launch per sweep instead of one per step.

// vertices per step (S <= HIST_MAX_STEPS): per-block LDS counts, part[b * S + s]
constexpr int HIST_MAX_STEPS = 256;

__global__ __launch_bounds__(256) void k_step_hist(int64_t n, const int32_t *stepv, int32_t S, int32_t *part)
{
    __shared__ int32_t h[HIST_MAX_STEPS];
    for (int s = threadIdx.x; s < S; s += 256) h[s] = 0;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        const int32_t st = stepv[v];
        if (st >= 0 && st < S) atomicAdd(&h[st], 1);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < S; s += 256) part[(int64_t)blockIdx.x * S + s] = h[s];
}

// out[s] = sum over the nb blocks' counts of step s: one workgroup per step
__global__ __launch_bounds__(256) void k_step_hist_sum(int nb, int32_t S, const int32_t *part, int32_t *out)
{
    __shared__ int32_t sw[4];
    const int32_t s = blockIdx.x;
    int32_t c = 0;
    for (int b = threadIdx.x; b < nb; b += 256) c += part[(int64_t)b * S + s];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) out[s] = sw[0] + sw[1] + sw[2] + sw[3];
}

// jr[v] = v for a vertex of steps m0..m1-1, -1 otherwise
__global__ void k_mid_init(int64_t n, const int32_t *stepv, int32_t m0, int32_t m1, int32_t *jr)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) jr[v] = stepv[v] >= m0 && stepv[v] < m1 ? (int32_t)v : -1;
}

// one round of hooking along the up-links between mid vertices: where the
// two ends carry different labels, the larger label (a vertex of the
// component) takes the smaller one as its label.  Labels only decrease and
// stay members of the component, so with the jumps below they converge to
// its smallest vertex; flag: a link still joined two labels
__global__ void k_mid_link(int64_t n, const int32_t *up0, const int32_t *up1, int32_t *jr, int32_t *flag)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t a = jr[v];
    if (a < 0) return;
    const int32_t u[2] = {up0[v], up1[v]};
    for (int k = 0; k < 2; k++) {
        if (u[k] < 0) continue;
        const int32_t b = jr[u[k]];
        if (b < 0 || b == a) continue;
        if (b < a)
            atomicMin(&jr[a], b);
        else
            atomicMin(&jr[b], a);
        flag[0] = 1;
    }
}

// jr[v] = jr[jr[v]]: a label's own label is no larger
__global__ void k_mid_jump(int64_t n, int32_t *jr)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t a = jr[v];
    if (a >= 0) jr[v] = jr[a];
}

// first q of every (step, workgroup) key in [lo, hi], at wptr[key - lo]; keys sorted
__global__ void k_mid_ptr(int64_t n, const uint32_t *key, int64_t lo, int64_t hi, int32_t *wptr)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q > n) return;
    int64_t a = q == 0 ? lo - 1 : (int64_t)key[q - 1];
    int64_t b = q == n ? hi : (int64_t)key[q];
    if (a < lo - 1) a = lo - 1;
    if (b > hi) b = hi;
    for (int64_t k = a + 1; k <= b; k++) wptr[k - lo] = (int32_t)q;
}

// step boundaries from the keys sorted by step: sptr[s] = first q of step s
__global__ void k_step_bounds(int64_t n, const uint32_t *skey, uint32_t div, int32_t S, int32_t *sptr)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q > n) return;
    int32_t lo = q == 0 ? -1 : (int32_t)(skey[q - 1] / div);
    int32_t hi = q == n ? S : (int32_t)(skey[q] / div);
    for (int32_t s = lo + 1; s <= hi; s++) sptr[s] = (int32_t)q;
}

// keys walked in the internal order: within a step, vertices end up in the
// internal (spatial) order, which keeps the sweeps' gathers local
__global__ void k_stepkeys(int64_t n, const int32_t *stepv, const int32_t *wgv, uint32_t nwg, const int32_t *perm,
                           uint32_t *key, int32_t *val)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t v = perm[i];
    key[i] = (uint32_t)stepv[v] * nwg + (wgv ? (uint32_t)wgv[v] : 0u);
    val[i] = v;
}

__global__ void k_map_ids(int64_t n, const int32_t *ids, const int32_t *inv, int32_t *out)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = inv[ids[q]];
}

__global__ void k_step0_sorted(int32_t q1, const int32_t *elim, int32_t *flag)
{
    const int32_t q = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q > 0 && q < q1 && elim[q] <= elim[q - 1]) flag[0] = 1;
}

__global__ void k_invperm(int64_t n, const int32_t *elim, int32_t *pos)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) pos[elim[q]] = (int32_t)q;
}

// up links in elimination numbering, and the in-list entries (target, source slot)
__global__ void k_uplinks(int64_t n, const int32_t *elim, const int32_t *pos, const int32_t *up0,
                          const int32_t *up1, int32_t *upq, uint32_t *ikey, int32_t *ival, int32_t *icnt)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int32_t v = elim[q];
    int32_t a = up0[v], b = up1[v];
    int32_t qa = a >= 0 ? pos[a] : -1, qb = b >= 0 ? pos[b] : -1;
    upq[2 * q] = qa;
    upq[2 * q + 1] = qb;
    ikey[2 * q] = qa >= 0 ? (uint32_t)qa : (uint32_t)n;
    ival[2 * q] = (int32_t)(2 * q);
    ikey[2 * q + 1] = qb >= 0 ? (uint32_t)qb : (uint32_t)n;
    ival[2 * q + 1] = (int32_t)(2 * q + 1);
    if (qa >= 0) atomicAdd(&icnt[qa], 1);
    if (qb >= 0) atomicAdd(&icnt[qb], 1);
}

// ---------------------------------------------------------------- numeric factor

// One elimination step: pivots of the step's vertices, their couplings F and
// their Schur contributions C[slot] (symmetric packed) to the vertices above.
__global__ void k_factor_step(int32_t q0, int32_t q1, const int32_t *elim, const int32_t *upq,
                              const int32_t *in_ptr, const int32_t *in_src, const double *Pd, double *E,
                              double *C, double *F, int64_t fs, double *Dinv, int32_t *status)
{
    int32_t q = q0 + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= q1) return;
    int32_t v = elim[q];
    double D[9];
    for (int t = 0; t < 9; t++) D[t] = Pd[9 * (int64_t)v + t];
    for (int32_t t = in_ptr[q]; t < in_ptr[q + 1]; t++) {
        const double *c = C + 6 * (int64_t)in_src[t];
        D[0] = D[0] - c[0]; D[1] = D[1] - c[1]; D[2] = D[2] - c[2];
        D[3] = D[3] - c[1]; D[4] = D[4] - c[3]; D[5] = D[5] - c[4];
        D[6] = D[6] - c[2]; D[7] = D[7] - c[4]; D[8] = D[8] - c[5];
    }
    double inv[6];
    if (!spd_inverse3(D, inv)) {
        atomicOr(status, 1);
        for (int t = 0; t < 6; t++) inv[t] = 0.0;
    }
    for (int t = 0; t < 6; t++) Dinv[6 * (int64_t)q + t] = inv[t];
    double Di[9];
    sym_unpack(inv, Di);
    int32_t qa = upq[2 * q], qb = upq[2 * q + 1];
    double T0[9];
    if (qa >= 0) {
        double E0[9];
        for (int t = 0; t < 9; t++) E0[t] = E[9 * (int64_t)q + t];   // A_{p,v}
        for (int t = 0; t < 9; t++) F[9 * (int64_t)q + t] = E0[t];
        mm3(E0, Di, T0);                                                // A_{p,v} D^{-1}
        double *c = C + 6 * (2 * (int64_t)q);
        // A_{p,v} D^{-1} A_{v,p}: upper triangle of T0 E0^T
        c[0] = T0[0] * E0[0] + T0[1] * E0[1] + T0[2] * E0[2];
        c[1] = T0[0] * E0[3] + T0[1] * E0[4] + T0[2] * E0[5];
        c[2] = T0[0] * E0[6] + T0[1] * E0[7] + T0[2] * E0[8];
        c[3] = T0[3] * E0[3] + T0[4] * E0[4] + T0[5] * E0[5];
        c[4] = T0[3] * E0[6] + T0[4] * E0[7] + T0[5] * E0[8];
        c[5] = T0[6] * E0[6] + T0[7] * E0[7] + T0[8] * E0[8];
    }
    if (qb >= 0) {
        double E1[9], E1t[9], T1[9];
        for (int t = 0; t < 9; t++) E1[t] = E[9 * (int64_t)qb + t];   // A_{v,c}
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) E1t[3 * a + b] = E1[3 * b + a];
        for (int t = 0; t < 9; t++) F[fs + 9 * (int64_t)q + t] = E1t[t];   // A_{c,v}
        mm3(E1t, Di, T1);                                                   // A_{c,v} D^{-1}
        double *c = C + 6 * (2 * (int64_t)q + 1);
        // A_{c,v} D^{-1} A_{v,c}: upper triangle of T1 E1
        c[0] = T1[0] * E1[0] + T1[1] * E1[3] + T1[2] * E1[6];
        c[1] = T1[0] * E1[1] + T1[1] * E1[4] + T1[2] * E1[7];
        c[2] = T1[0] * E1[2] + T1[1] * E1[5] + T1[2] * E1[8];
        c[3] = T1[3] * E1[1] + T1[4] * E1[4] + T1[5] * E1[7];
        c[4] = T1[3] * E1[2] + T1[4] * E1[5] + T1[5] * E1[8];
        c[5] = T1[6] * E1[2] + T1[7] * E1[5] + T1[8] * E1[8];
        // new coupling of parent and child: -A_{p,v} D^{-1} A_{v,c}
        double Nw[9];
        mm3(T0, E1, Nw);
        for (int t = 0; t < 9; t++) E[9 * (int64_t)qb + t] = -Nw[t];
    }
}

__global__ void k_slot_of(const int32_t *n_in, const int32_t *in_src, int32_t *tout)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < *n_in) tout[in_src[t]] = (int32_t)t;
}

// E is stored per vertex id for the initial blocks; the factor works in
// elimination numbering: permute once.
// One thread per entry (9 n of them): the stores are contiguous and a block's
// 9 loads are one 72-byte run (one thread per block had made every store
// instruction write 64 lanes 72 bytes apart: 220 us at 1M).
__global__ void k_permute9(int64_t n, const int32_t *elim, const double *src, double *dst)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 9 * n) return;
    const int64_t q = e / 9, t = e - 9 * q;
    dst[e] = src[9 * (int64_t)elim[q] + t];
}

// ---------------------------------------------------------------- sweeps


// b -= the slots t..te-1, in slot order; slots are independent loads:
// fetched four at a time.  (Issuing up to 12 slots' loads at once was
// measured too: the small steps got slower, ~7.5 instead of ~6.3 us.)
template <class T>
SGP_DEV void sum_slots(int32_t t, int32_t te, const T *cs, T &b0, T &b1, T &b2)
{
    for (; t + 4 <= te; t += 4) {
        const T *c = cs + 3 * (int64_t)t;
        T c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5];
        T c6 = c[6], c7 = c[7], c8 = c[8], c9 = c[9], c10 = c[10], c11 = c[11];
        b0 = b0 - c0; b1 = b1 - c1; b2 = b2 - c2;
        b0 = b0 - c3; b1 = b1 - c4; b2 = b2 - c5;
        b0 = b0 - c6; b1 = b1 - c7; b2 = b2 - c8;
        b0 = b0 - c9; b1 = b1 - c10; b2 = b2 - c11;
    }
    for (; t < te; t++) {
        const T *c = cs + 3 * (int64_t)t;
        b0 = b0 - c[0]; b1 = b1 - c[1]; b2 = b2 - c[2];
    }
}

// The same sum with the first chunk of four slots and the last one to three
// loaded together, ahead of any wait, and unconditionally (indices clamped
// into [t, max(te - 1, t)]; the slot array holds a spare slot past its end):
// a load in a branch makes the compiler wait for every earlier load there.
// Chunks between them are loaded four at a time.  Faster for the tail's
// pre-sums (many slots per vertex: 5.1 -> 4.8 us), slower in the step
// kernels (~6.2 -> ~7.2 us per small step: larger code, fewer vertices with
// many slots), which keep sum_slots.
template <class T>
SGP_DEV void sum_slots_early(int32_t t, int32_t te, const T *cs, T &b0, T &b1, T &b2)
{
    const int32_t n = te - t, full = n & ~3, last = te > t ? te - 1 : t;
    T h[12], r[9];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const T *c = cs + 3 * (int64_t)min(t + k, last);
        h[3 * k] = c[0];
        h[3 * k + 1] = c[1];
        h[3 * k + 2] = c[2];
    }
#pragma unroll
    for (int u = 0; u < 3; u++) {
        const T *c = cs + 3 * (int64_t)min(t + full + u, last);
        r[3 * u] = c[0];
        r[3 * u + 1] = c[1];
        r[3 * u + 2] = c[2];
    }
    keep_loads_above();
    if (full >= 4) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            b0 = b0 - h[3 * k];
            b1 = b1 - h[3 * k + 1];
            b2 = b2 - h[3 * k + 2];
        }
    }
    for (int32_t m = t + 4; m < t + full; m += 4) {
        const T *c = cs + 3 * (int64_t)m;
        T c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5];
        T c6 = c[6], c7 = c[7], c8 = c[8], c9 = c[9], c10 = c[10], c11 = c[11];
        b0 = b0 - c0; b1 = b1 - c1; b2 = b2 - c2;
        b0 = b0 - c3; b1 = b1 - c4; b2 = b2 - c5;
        b0 = b0 - c6; b1 = b1 - c7; b2 = b2 - c8;
        b0 = b0 - c9; b1 = b1 - c10; b2 = b2 - c11;
    }
#pragma unroll
    for (int u = 0; u < 3; u++) {
        const bool on = u < n - full;
        b0 = on ? b0 - r[3 * u] : b0;
        b1 = on ? b1 - r[3 * u + 1] : b1;
        b2 = on ? b2 - r[3 * u + 2] : b2;
    }
}

// forward substitution of one vertex q (pivot solve folded in), then the
// push of its contributions to the vertices above it.  The loads come in
// rounds: what depends on q alone (ids, the pivot, the first coupling
// plane), then what those ids address (r, the slots, and the second plane
// for a vertex with a second link).  Every load precedes every store in the
// source, so the compiler need not order a coupling's load after a push that
// might alias it.  A finished solve (s->done) skips the stores only, so its
// flag is awaited together with the loads.
template <class T>
SGP_DEV void fwd_vertex(int32_t q, const int32_t *elim, const int32_t *in_ptr, const int32_t *tout, const T *F,
                        int64_t fs, const T *Dinv, const T *r, T *y, T *cs, const PcgScalars *s)
{
    const int32_t dn = done_flag(s);
    const int64_t v = elim[q];
    const int32_t t = in_ptr[q];
    const int32_t te = in_ptr[q + 1];
    const int32_t to0 = tout[2 * q], to1 = tout[2 * q + 1];
    T d[6], f0[9], f1[9];
    for (int k = 0; k < 6; k++) d[k] = Dinv[6 * (int64_t)q + k];
    for (int k = 0; k < 9; k++) f0[k] = F[9 * (int64_t)q + k];
    T b0 = r[3 * v], b1 = r[3 * v + 1], b2 = r[3 * v + 2];
    if (to1 >= 0)
        for (int k = 0; k < 9; k++) f1[k] = F[fs + 9 * (int64_t)q + k];
    sum_slots<T>(t, te, cs, b0, b1, b2);
    keep_loads_above();
    if (dn) return;
    T o0, o1, o2;
    sym_mv(d, b0, b1, b2, o0, o1, o2);
    y[3 * (int64_t)q] = o0;
    y[3 * (int64_t)q + 1] = o1;
    y[3 * (int64_t)q + 2] = o2;
    if (to0 >= 0) {
        T *c = cs + 3 * (int64_t)to0;
        c[0] = f0[0] * o0 + f0[1] * o1 + f0[2] * o2;
        c[1] = f0[3] * o0 + f0[4] * o1 + f0[5] * o2;
        c[2] = f0[6] * o0 + f0[7] * o1 + f0[8] * o2;
    }
    if (to1 >= 0) {
        T *c = cs + 3 * (int64_t)to1;
        c[0] = f1[0] * o0 + f1[1] * o1 + f1[2] * o2;
        c[1] = f1[3] * o0 + f1[4] * o1 + f1[5] * o2;
        c[2] = f1[6] * o0 + f1[7] * o1 + f1[8] * o2;
    }
}

// backward substitution of one vertex q; y holds x for the vertices above.
// Two rounds of loads: ids, pivot, own y and the first coupling plane; then
// x of both up-links (a missing link reads the vertex's own y and is masked)
// and, for a second link, the second plane.  x_q is kept in y only for the
// vertices below that read it (keep_x: vertices with in-slots; none in the
// first elimination step).
template <class T>
SGP_DEV void bwd_vertex(int32_t q, const int32_t *elim, const int32_t *upq, const T *F, int64_t fs, const T *Dinv,
                        T *y, T *z, const PcgScalars *s, bool keep_x = true)
{
    const int32_t dn = done_flag(s);
    const int32_t w0 = upq[2 * q], w1 = upq[2 * q + 1];
    const int64_t v = elim[q];
    T d[6], f0[9], f1[9];
    for (int k = 0; k < 6; k++) d[k] = Dinv[6 * (int64_t)q + k];
    for (int k = 0; k < 9; k++) f0[k] = F[9 * (int64_t)q + k];
    const T y0 = y[3 * (int64_t)q], y1 = y[3 * (int64_t)q + 1], y2 = y[3 * (int64_t)q + 2];
    const int64_t u0 = w0 >= 0 ? w0 : q, u1 = w1 >= 0 ? w1 : q;
    const T p0 = y[3 * u0], p1 = y[3 * u0 + 1], p2 = y[3 * u0 + 2];
    const T x0 = y[3 * u1], x1 = y[3 * u1 + 1], x2 = y[3 * u1 + 2];
    if (w1 >= 0)
        for (int k = 0; k < 9; k++) f1[k] = F[fs + 9 * (int64_t)q + k];
    keep_loads_above();
    if (dn) return;
    T a0 = 0, a1 = 0, a2 = 0;
    if (w0 >= 0) {
        a0 = a0 + (f0[0] * p0 + f0[3] * p1 + f0[6] * p2);
        a1 = a1 + (f0[1] * p0 + f0[4] * p1 + f0[7] * p2);
        a2 = a2 + (f0[2] * p0 + f0[5] * p1 + f0[8] * p2);
    }
    if (w1 >= 0) {
        a0 = a0 + (f1[0] * x0 + f1[3] * x1 + f1[6] * x2);
        a1 = a1 + (f1[1] * x0 + f1[4] * x1 + f1[7] * x2);
        a2 = a2 + (f1[2] * x0 + f1[5] * x1 + f1[8] * x2);
    }
    T e0, e1, e2;
    sym_mv(d, a0, a1, a2, e0, e1, e2);
    const T n0 = y0 - e0, n1 = y1 - e1, n2 = y2 - e2;
    if (keep_x) {
        y[3 * (int64_t)q] = n0;
        y[3 * (int64_t)q + 1] = n1;
        y[3 * (int64_t)q + 2] = n2;
    }
    z[3 * v] = n0;
    z[3 * v + 1] = n1;
    z[3 * v + 2] = n2;
}

// The first elimination step, couplings from (w, u) (planes of ws values):
// forward, its vertices have no in-slots, so y = P_qq^{-1} r and the pushes
// follow; backward, x = y - P_qq^{-1} (sum over up-links of W x) and only z
// is written (no vertex reads a first-step x).
template <class T>
__global__ void k_fwd_step0(int32_t q1, const int32_t *elim, const int32_t *tout, const T *wu, int64_t ws,
                            T gpar, T gperp, T gmed, const T *Dinv, const T *r, T *y, T *cs, const PcgScalars *s)
{
    const int32_t q = (int32_t)(xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x);
    if (q >= q1) return;
    const int32_t dn = done_flag(s);
    const int64_t v = elim[q];
    const int32_t to0 = tout[2 * q], to1 = tout[2 * q + 1];
    T d[6], e0[4], e1[4];
    for (int k = 0; k < 4; k++) e0[k] = wu[4 * (int64_t)q + k];
    const T b0 = r[3 * v], b1 = r[3 * v + 1], b2 = r[3 * v + 2];
    if (to1 >= 0) {
        for (int k = 0; k < 4; k++) e1[k] = wu[ws + 4 * (int64_t)q + k];
        for (int k = 0; k < 6; k++) d[k] = Dinv[6 * (int64_t)q + k];
    }
    keep_loads_above();
    if (dn) return;
    T o0, o1, o2;
    if (to1 >= 0)
        sym_mv(d, b0, b1, b2, o0, o1, o2);
    else
        leaf_pivot_solve(e0, gpar, gperp, gmed, b0, b1, b2, o0, o1, o2);
    y[3 * (int64_t)q] = o0;
    y[3 * (int64_t)q + 1] = o1;
    y[3 * (int64_t)q + 2] = o2;
    if (to0 >= 0) {
        T *c = cs + 3 * (int64_t)to0;
        neg_w_mv(e0, gpar, gperp, o0, o1, o2, c[0], c[1], c[2]);
    }
    if (to1 >= 0) {
        T *c = cs + 3 * (int64_t)to1;
        neg_w_mv(e1, gpar, gperp, o0, o1, o2, c[0], c[1], c[2]);
    }
}

template <class T>
__global__ void k_bwd_step0(int32_t q1, const int32_t *elim, const int32_t *upq, const T *wu, int64_t ws, T gpar,
                            T gperp, T gmed, const T *Dinv, const T *y, T *z, const PcgScalars *s)
{
    const int32_t q = (int32_t)(xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x);
    if (q >= q1) return;
    const int32_t dn = done_flag(s);
    const int32_t w0 = upq[2 * q], w1 = upq[2 * q + 1];
    const int64_t v = elim[q];
    T d[6], e0[4], e1[4];
    for (int k = 0; k < 4; k++) e0[k] = wu[4 * (int64_t)q + k];
    const T y0 = y[3 * (int64_t)q], y1 = y[3 * (int64_t)q + 1], y2 = y[3 * (int64_t)q + 2];
    const int64_t u0 = w0 >= 0 ? w0 : q, u1 = w1 >= 0 ? w1 : q;
    const T p0 = y[3 * u0], p1 = y[3 * u0 + 1], p2 = y[3 * u0 + 2];
    const T x0 = y[3 * u1], x1 = y[3 * u1 + 1], x2 = y[3 * u1 + 2];
    if (w1 >= 0) {
        for (int k = 0; k < 4; k++) e1[k] = wu[ws + 4 * (int64_t)q + k];
        for (int k = 0; k < 6; k++) d[k] = Dinv[6 * (int64_t)q + k];
    }
    keep_loads_above();
    if (dn) return;
    T a0 = 0, a1 = 0, a2 = 0;
    if (w0 >= 0) {
        T c0, c1, c2;
        neg_w_mv(e0, gpar, gperp, p0, p1, p2, c0, c1, c2);
        a0 = a0 + c0;
        a1 = a1 + c1;
        a2 = a2 + c2;
    }
    if (w1 >= 0) {
        T c0, c1, c2;
        neg_w_mv(e1, gpar, gperp, x0, x1, x2, c0, c1, c2);
        a0 = a0 + c0;
        a1 = a1 + c1;
        a2 = a2 + c2;
    }
    T e0_, e1_, e2_;
    if (w1 >= 0)
        sym_mv(d, a0, a1, a2, e0_, e1_, e2_);
    else
        leaf_pivot_solve(e0, gpar, gperp, gmed, a0, a1, a2, e0_, e1_, e2_);
    z[3 * v] = y0 - e0_;
    z[3 * v + 1] = y1 - e1_;
    z[3 * v + 2] = y2 - e2_;
}

template <class T>
__global__ __launch_bounds__(256) void k_fwd_step(int32_t q0, int32_t q1, const int32_t *elim,
                                                  const int32_t *in_ptr, const int32_t *tout, const T *F, int64_t fs,
                                                  const T *Dinv, const T *r, T *y, T *cs, const PcgScalars *s)
{
    int32_t q = q0 + (int32_t)(xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x);
    if (q < q1) fwd_vertex<T>(q, elim, in_ptr, tout, F, fs, Dinv, r, y, cs, s);
}

// keep_x = false for the first elimination step (its vertices have no
// in-slots, so no vertex reads their x)
template <class T>
__global__ __launch_bounds__(256) void k_bwd_step(int32_t q0, int32_t q1, const int32_t *elim, const int32_t *upq,
                                                  const T *F, int64_t fs, const T *Dinv, T *y, T *z,
                                                  const PcgScalars *s, int keep_x)
{
    int32_t q = q0 + (int32_t)(xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x);
    if (q < q1) bwd_vertex<T>(q, elim, upq, F, fs, Dinv, y, z, s, keep_x != 0);
}

// The light steps of both sweeps: workgroup w owns the light subtrees packed
// into it and walks steps 0..L-1 (forward) or L-1..0 (backward) over its own
// vertices, wptr[s * nwg + w] .. wptr[s * nwg + w + 1], with a barrier between
// steps.  A light vertex's pushes go to its parent, which is in the same
// workgroup (read after the barrier) or above the light steps (read by a
// later launch); backward, a light vertex reads x of its parent the same way.
template <class T>
__global__ __launch_bounds__(256) void k_fwd_light(int32_t L, int32_t nwg, const int32_t *wptr, const int32_t *elim,
                                                   const int32_t *in_ptr, const int32_t *tout, const T *F,
                                                   int64_t fs, const T *Dinv, const T *r, T *y, T *cs,
                                                   const PcgScalars *s)
{
    if (s && s->done) return;
    const int32_t w = (int32_t)xcd_block(blockIdx.x, gridDim.x);
    for (int32_t k = 0; k < L; k++) {
        const int32_t q1 = wptr[(int64_t)k * nwg + w + 1];
        for (int32_t q = wptr[(int64_t)k * nwg + w] + (int32_t)threadIdx.x; q < q1; q += 256)
            fwd_vertex<T>(q, elim, in_ptr, tout, F, fs, Dinv, r, y, cs, nullptr);
        __syncthreads();
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_bwd_light(int32_t L, int32_t nwg, const int32_t *wptr, const int32_t *elim,
                                                   const int32_t *upq, const T *F, int64_t fs, const T *Dinv,
                                                   T *y, T *z, const PcgScalars *s)
{
    if (s && s->done) return;
    const int32_t w = (int32_t)xcd_block(blockIdx.x, gridDim.x);
    for (int32_t k = L - 1; k >= 0; k--) {
        const int32_t q1 = wptr[(int64_t)k * nwg + w + 1];
        for (int32_t q = wptr[(int64_t)k * nwg + w] + (int32_t)threadIdx.x; q < q1; q += 256)
            bwd_vertex<T>(q, elim, upq, F, fs, Dinv, y, z, nullptr);
        __syncthreads();
    }
}

// The last, small steps of both sweeps in one workgroup.  The tail vertices
// q >= Qt (elimination order) and the pushes between them live in LDS:
//   sv[q - Qt]   the right-hand side, then y_q, then x_q (in place)
//   slot[i]      the contribution of a tail source to a tail target; the
//                internal in-entries of a target are the last ones of its
//                in-list, so its slots form one range iptr[q-Qt]..iptr[q-Qt+1]
// Contributions from vertices eliminated before the tail are summed first,
// for all tail vertices in parallel.  A barrier separates two steps; all
// up-links of tail vertices point into the tail, so the backward steps read
// x only from LDS.  x is also written to y (global) for the earlier steps.
// Threads exchange data through LDS only (global reads are of inputs this
// kernel never writes, global writes are never read back here), so the steps
// are separated by LDS-only barriers: the next step's prefetched loads stay
// in flight across them.
constexpr int TAIL_THREADS = 512;
constexpr int TAIL_WINDOW = 2 * TAIL_THREADS;   // tail vertices whose constants stay in registers
constexpr int TAIL_SLOTS = 4;   // LDS reads of in-slots issued together
constexpr int TAIL_LDS_BYTES = 160 * 1024;

// LDS of the tail: right-hand sides and internal push slots (3 values each),
// and the step bounds of its steps
static size_t tail_lds_bytes(size_t elem, int64_t nt, int64_t ni, int64_t nsteps)
{
    return 3 * elem * (size_t)(nt + ni) + 4 * (size_t)(nsteps + 1);
}

// tail vertices at most: every vertex pushes to at most two others and a step
// holds at least one vertex, so 3 * 8 * 3 nt + 4 (nt + 1) bytes always suffice
constexpr int TAIL_MAX_VERTICES = (TAIL_LDS_BYTES - 4) / 76;
constexpr int TAIL_DEFAULT_VERTICES = 2200;   // the tail_max knob's default
// right-hand-side values a tail thread loads: 3 per vertex, up to the most
// vertices the tail holds
constexpr int TAIL_RHS_PER_THREAD = (3 * TAIL_MAX_VERTICES + TAIL_THREADS - 1) / TAIL_THREADS;
constexpr int64_t MID_MAX_VERTICES = 1 << 17;   // vertices left at the first mid step at most

// The tail's constants (pivots, both coupling planes, push slots, up-links,
// ids, in-slot bounds of its nt vertices) loaded ahead, from the XCD that
// runs the tail's single workgroup, so that its start-up loads hit in the
// caches.  Workgroup i of a launch runs on XCD i mod 8; the tail launch's
// first workgroup is the tail, so the prefetching workgroups are the
// TAIL_PF_WG / 8 of this launch with blockIdx = 0 mod 8, 64 threads each, a
// thread's loads all issued before any is used.  Their sum is stored only if
// `never` (0) says so, which keeps the loads.  1M cells: the tail launch
// 33.8 -> 28.0 us (29.0 us with the same loads spread over all XCDs); the
// pre-tail launch unchanged.
constexpr int TAIL_PF_WG = 1024;
constexpr int TAIL_PF_THREADS = TAIL_PF_WG / 8 * 64;
static_assert(9 * TAIL_MAX_VERTICES <= 4 * TAIL_PF_THREADS && 2 * TAIL_MAX_VERTICES + 1 <= 2 * TAIL_PF_THREADS,
              "the prefetch covers the largest tail");
template <class T>
SGP_DEV void tail_prefetch(int j, int32_t Qt, int32_t nt, const T *F, int64_t fs, const T *Dinv,
                           const int32_t *tslot, const int32_t *upq, const int32_t *elim, const int32_t *iptr,
                           T *sink, int32_t never)
{
    const int64_t g = (int64_t)j * 64 + threadIdx.x, G = TAIL_PF_THREADS;
    const int64_t lt[3] = {6 * (int64_t)nt, 9 * (int64_t)nt, 9 * (int64_t)nt};
    const T *at[3] = {Dinv + 6 * (int64_t)Qt, F + 9 * (int64_t)Qt, F + fs + 9 * (int64_t)Qt};
    const int64_t li[4] = {2 * (int64_t)nt, 2 * (int64_t)nt, (int64_t)nt, (int64_t)nt + 1};
    const int32_t *ai[4] = {tslot, upq + 2 * (int64_t)Qt, elim + Qt, iptr};
    T v[3][4];
    int32_t w[4][2];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int u = 0; u < 4; u++) v[a][u] = g + u * G < lt[a] ? at[a][g + u * G] : (T)0;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int u = 0; u < 2; u++) w[a][u] = g + u * G < li[a] ? ai[a][g + u * G] : 0;
    T acc = 0;
    int32_t iacc = 0;
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int u = 0; u < 4; u++) acc += v[a][u];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int u = 0; u < 2; u++) iacc += w[a][u];
    if (never) sink[0] = acc + (T)iacc;
}

// The tail's right-hand sides before its first step: r minus the pushes from
// vertices eliminated before the tail (all finished by the launch boundary).
// Many small workgroups, one tail vertex per thread, so the dependent loads
// of different vertices overlap across CUs instead of queueing in the tail's
// single workgroup.  Workgroups from npre on prefetch the tail's constants
// (tail_prefetch) when there are any.
template <class T>
__global__ __launch_bounds__(64) void k_tail_pre(int32_t Qt, int32_t nt, const int32_t *elim, const int32_t *in_ptr,
                                                 const int32_t *iptr, const T *r, const T *cs, T *tb,
                                                 const PcgScalars *s, int32_t npre, const T *F, int64_t fs,
                                                 const T *Dinv, const int32_t *tslot, const int32_t *upq,
                                                 int32_t never)
{
    if ((int32_t)blockIdx.x >= npre) {
        if (blockIdx.x % 8 != 0) return;
        const int j = ((int32_t)blockIdx.x - (npre + 7) / 8 * 8) / 8;
        tail_prefetch<T>(j, Qt, nt, F, fs, Dinv, tslot, upq, elim, iptr, tb, never);
        return;
    }
    const int32_t i = blockIdx.x * 64 + threadIdx.x;
    if (i >= nt) return;
    const int32_t q = Qt + i;
    const int32_t dn = done_flag(s);
    const int64_t v = elim[q];
    T b0 = r[3 * v], b1 = r[3 * v + 1], b2 = r[3 * v + 2];
    const int32_t te = in_ptr[q + 1] - (iptr[i + 1] - iptr[i]);
    sum_slots_early<T>(in_ptr[q], te, cs, b0, b1, b2);
    keep_loads_above();
    if (dn) return;
    tb[3 * (int64_t)i] = b0;
    tb[3 * (int64_t)i + 1] = b1;
    tb[3 * (int64_t)i + 2] = b2;
}

// the per-vertex constants of one tail vertex, loaded a step ahead
template <class T>
struct TailPre {
    T d[6], f0[9], f1[9];
    int32_t a0, a1;   // forward: push slots; backward: up-links (elimination index)
    int32_t b0, b1;   // forward: first and end internal in-slot; backward: vertex id
};

// the constants of a thread's vertex in the last TAIL_THREADS tail vertices,
// for both sweeps, loaded once per launch
template <class T>
struct TailReg {
    T d[6], f0[9], f1[9];
    int32_t slot0, slot1, in0, in1;   // forward: push slots, internal in-slot range
    int32_t up0, up1, id;             // backward: up-links, vertex id
};

// The loaders never branch on a value they load: a branch would wait for
// every load issued before it and turn the prefetch into a stall.  Both F
// planes are read (the second is zero where there is no second link).
template <class T>
SGP_DEV void tail_load_common(T *d, T *f0, T *f1, int32_t q, const T *F, int64_t fs, const T *Dinv)
{
    for (int t = 0; t < 6; t++) d[t] = Dinv[6 * (int64_t)q + t];
    for (int t = 0; t < 9; t++) f0[t] = F[9 * (int64_t)q + t];
    for (int t = 0; t < 9; t++) f1[t] = F[fs + 9 * (int64_t)q + t];
}

// forward: push slots and the internal in-slot range
template <class T>
SGP_DEV void tail_load_fwd(TailPre<T> &p, int32_t q, int32_t i, const int32_t *tslot, const int32_t *iptr,
                           const T *F, int64_t fs, const T *Dinv)
{
    p.a0 = tslot[2 * i];
    p.a1 = tslot[2 * i + 1];
    p.b0 = iptr[i];
    p.b1 = iptr[i + 1];
    tail_load_common(p.d, p.f0, p.f1, q, F, fs, Dinv);
}

// backward: up-links and the vertex id
template <class T>
SGP_DEV void tail_load_bwd(TailPre<T> &p, int32_t q, const int32_t *upq, const int32_t *elim, const T *F,
                           int64_t fs, const T *Dinv)
{
    p.a0 = upq[2 * q];
    p.a1 = upq[2 * q + 1];
    p.b0 = elim[q];
    tail_load_common(p.d, p.f0, p.f1, q, F, fs, Dinv);
}

template <class T>
SGP_DEV void tail_load_reg(TailReg<T> &p, int32_t q, int32_t i, const int32_t *tslot, const int32_t *iptr,
                           const int32_t *upq, const int32_t *elim, const T *F, int64_t fs, const T *Dinv)
{
    p.slot0 = tslot[2 * i];
    p.slot1 = tslot[2 * i + 1];
    p.in0 = iptr[i];
    p.in1 = iptr[i + 1];
    p.up0 = upq[2 * q];
    p.up1 = upq[2 * q + 1];
    p.id = elim[q];
    tail_load_common(p.d, p.f0, p.f1, q, F, fs, Dinv);
}

// x += alpha p of the CG (SideX) by workgroup wg of nwg extra workgroups of
// the tail launch: SIDE_BLOCKS vector blocks per round, every load of a round
// issued before its first store (blocks are disjoint row ranges, so no store
// of a round aliases one of its loads).  Same expression as the CG's own
// update pass, so x is bitwise the same.
constexpr int SIDE_BLOCKS = 4;
static_assert(2 * TAIL_THREADS >= SIDE_BLOCK_VALUES, "two values per thread cover a vector block");
template <class T>
SGP_DEV void side_x_update(const SideX &sd, int wg, int nwg)
{
    T *x = (T *)sd.x;
    const T *p = (const T *)sd.p;
    const int tid = threadIdx.x;
    for (int b0 = wg * SIDE_BLOCKS; b0 < sd.nb; b0 += nwg * SIDE_BLOCKS) {
        int64_t e0[SIDE_BLOCKS];
        int nel[SIDE_BLOCKS], inst[SIDE_BLOCKS];
#pragma unroll
        for (int u = 0; u < SIDE_BLOCKS; u++) {
            const int b = min(b0 + u, sd.nb - 1);
            e0[u] = 3 * (int64_t)sd.row0[b];
            nel[u] = b0 + u < sd.nb ? 3 * (sd.row1[b] - sd.row0[b]) : 0;
            inst[u] = sd.inst[b];
        }
        T xv[SIDE_BLOCKS][2], pv[SIDE_BLOCKS][2], al[SIDE_BLOCKS];
        int32_t dn[SIDE_BLOCKS];
#pragma unroll
        for (int u = 0; u < SIDE_BLOCKS; u++) {
            dn[u] = sd.S[inst[u]].done;
            al[u] = (T)sd.S[inst[u]].alpha;
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int64_t e = e0[u] + min(tid + TAIL_THREADS * h, max(nel[u] - 1, 0));
                xv[u][h] = nel[u] > 0 ? x[e] : (T)0;
                pv[u][h] = nel[u] > 0 ? p[e] : (T)0;
            }
        }
#pragma unroll
        for (int u = 0; u < SIDE_BLOCKS; u++)
#pragma unroll
            for (int h = 0; h < 2; h++)
                if (dn[u] == 0 && tid + TAIL_THREADS * h < nel[u])
                    x[e0[u] + tid + TAIL_THREADS * h] = xv[u][h] + al[u] * pv[u][h];
    }
}

// The backward mid steps' constants (ids, up-links, their local indices,
// pivots, both coupling planes) loaded ahead, from the XCD whose k_bwd_mid
// workgroups will sweep them (the counters show k_bwd_mid fetching as many
// bytes from beyond L2 as without it: the gain, 14.7 -> 12.7 us at 1M cells,
// is the last-level cache's), by this XCD's extra workgroups of
// the tail launch (block b of a launch runs on XCD b mod 8; k_bwd_mid's
// group of block b is xcd_block(b), so XCD x sweeps one contiguous range of
// groups, and in every mid step their positions are contiguous).  The
// step ranges go through LDS; each workgroup takes its share of the
// positions, two per thread per round, every load of a round issued before
// any is used; the sums are stored only if sd.never says so.
template <class T>
SGP_DEV void mid_prefetch(const SideX &sd, int32_t nside, const int32_t *elim, const int32_t *upq, const T *F,
                          int64_t fs, const T *Dinv, int32_t *rg, T *sink)
{
    const int32_t b = (int32_t)blockIdx.x, x = b % NUM_XCD, L = sd.mid_L;
    const int32_t firstb = x == 0 ? NUM_XCD : x;   // this XCD's extra workgroups: firstb, firstb + 8, ...
    const int32_t nx = (nside - firstb) / NUM_XCD + 1, ix = (b - firstb) / NUM_XCD;
    const int32_t nw = sd.mid_nwg, q8 = nw / NUM_XCD, r8 = nw % NUM_XCD;
    const int32_t w0 = x < r8 ? x * (q8 + 1) : r8 * (q8 + 1) + (x - r8) * q8;
    const int32_t w1 = w0 + q8 + (x < r8 ? 1 : 0);
    const int tid = threadIdx.x;
    if (tid < 2 * L) rg[tid] = sd.mid_wptr[(int64_t)(tid >> 1) * nw + ((tid & 1) ? w1 : w0)];
    __syncthreads();
    int32_t P = 0;
    for (int32_t k = 0; k < L; k++) P += rg[2 * k + 1] - rg[2 * k];
    const int32_t f0 = (int32_t)((int64_t)P * ix / nx), f1 = (int32_t)((int64_t)P * (ix + 1) / nx);
    T acc = 0;
    int32_t iacc = 0;
    for (int32_t f = f0 + tid; f < f1; f += 2 * TAIL_THREADS) {
        int32_t q[2];
        bool on[2];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            int32_t l = f + TAIL_THREADS * u, k = 0;
            on[u] = l < f1;
            while (k < L - 1 && l >= rg[2 * k + 1] - rg[2 * k]) {
                l -= rg[2 * k + 1] - rg[2 * k];
                k++;
            }
            q[u] = on[u] ? rg[2 * k] + l : rg[0];
        }
        T d[2][6], g0[2][9], g1[2][9];
        int32_t iv[2][5];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int64_t qq = q[u];
            iv[u][0] = elim[qq];
            iv[u][1] = upq[2 * qq];
            iv[u][2] = upq[2 * qq + 1];
            iv[u][3] = sd.mid_lup[2 * (qq - sd.mid_Q0)];
            iv[u][4] = sd.mid_lup[2 * (qq - sd.mid_Q0) + 1];
            for (int t = 0; t < 6; t++) d[u][t] = Dinv[6 * qq + t];
            for (int t = 0; t < 9; t++) g0[u][t] = F[9 * qq + t];
            for (int t = 0; t < 9; t++) g1[u][t] = F[fs + 9 * qq + t];
        }
#pragma unroll
        for (int u = 0; u < 2; u++) {
            for (int t = 0; t < 5; t++) iacc += iv[u][t];
            for (int t = 0; t < 6; t++) acc += d[u][t];
            for (int t = 0; t < 9; t++) acc += g0[u][t] + g1[u][t];
        }
    }
    if (sd.never) sink[0] = acc + (T)iacc;
}

// The tail's steps fall in two parts.  Steps whose vertices all lie in the
// last TAIL_WINDOW tail vertices (the window, from step kw on: usually most
// of the steps, few vertices each) give vertices base + t and base +
// TAIL_THREADS + t to thread t, whose constants are loaded once per launch
// for both sweeps, so these steps touch no global memory but the backward
// sweep's stores.  The steps before kw (one or two, large) give their
// vertices to threads in order; a thread's first vertex of the first such
// step of each sweep is loaded ahead (while the prologue or the window's
// steps run), the others when their step comes.
template <class T>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail(int32_t s0, int32_t S, int32_t kw, int32_t kx, int32_t wx,
                                                       int32_t Qt, int32_t q1a,
                                                       int32_t nt, int32_t ni, const int32_t *sp_g, const int32_t *elim,
                                                       const int32_t *in_ptr, const int32_t *iptr,
                                                       const int32_t *tslot, const int32_t *upq, const T *F,
                                                       int64_t fs, const T *Dinv, const T *tb, T *y, T *z,
                                                       const PcgScalars *s, SideX side)
{
    extern __shared__ unsigned char lds_raw[];
    // workgroups past the first: the CG's x update, meanwhile, then the
    // backward mid steps' constants into the caches
    if (blockIdx.x > 0) {
        // unless the tail's constants were prefetched (k_tail_pre),
        // wait about 7 us (2 x 127 x 64 clocks) first, so that the tail's
        // own first loads are served before these streams fill the memory
        // queues (1M cells, without the prefetches: the tail launch with the
        // x update 35.9 us without the wait, 33.6 us with it, 32.6 us without
        // the x update; with both prefetches, 26.3 us without the wait and
        // 30.3 us with it)
        if (side.wait) {
            __builtin_amdgcn_s_sleep(127);
            __builtin_amdgcn_s_sleep(127);
        }
        if (side.nb > 0) side_x_update<T>(side, blockIdx.x - 1, gridDim.x - 1);
        if (side.mid_L > 0) mid_prefetch<T>(side, gridDim.x - 1, elim, upq, F, fs, Dinv, (int32_t *)lds_raw, z);
        return;
    }
    T *sv = (T *)lds_raw;
    T *slot = sv + 3 * nt;
    // step bounds of the tail steps, sp[k] for k = s0..S, kept in LDS
    int32_t *ssp = (int32_t *)(slot + 3 * ni) - s0;
    const int32_t dn = done_flag(s);
    const int tid = threadIdx.x;
    // the window's vertices of this thread (clamped: a thread past the end
    // loads the last vertex and never uses it)
    const int32_t base = nt > TAIL_WINDOW ? nt - TAIL_WINDOW : 0;
    const int32_t ir0 = base + tid, ir1 = base + TAIL_THREADS + tid;
    TailReg<T> R0, R1;
    {
        const int32_t i0 = ir0 < nt ? ir0 : nt - 1, i1 = ir1 < nt ? ir1 : nt - 1;
        tail_load_reg(R0, Qt + i0, i0, tslot, iptr, upq, elim, F, fs, Dinv);
        tail_load_reg(R1, Qt + i1, i1, tslot, iptr, upq, elim, F, fs, Dinv);
    }
    // a thread's first vertex of step k, clamped into the step
    auto vtx = [&](const int32_t *b, int32_t k) {
        const int32_t qe = b[k + 1] - 1;
        const int32_t q = b[k] + tid;
        return q < qe ? q : qe;
    };
    // the first step's first vertices (q1a: the end of step s0 when it lies
    // before the window, else Qt + 1), addressed from the arguments alone
    TailPre<T> pa;
    {
        const int32_t q = Qt + tid < q1a - 1 ? Qt + tid : q1a - 1;
        tail_load_fwd(pa, q, q - Qt, tslot, iptr, F, fs, Dinv);
    }
    // the step bounds and the right-hand sides with the pre-tail
    // contributions (k_tail_pre), loaded with the constants above (clamped,
    // surplus unused) so that one wait covers them all
    int32_t spv = sp_g[min(s0 + tid, S)];
    T tbv[TAIL_RHS_PER_THREAD];
#pragma unroll
    for (int m = 0; m < TAIL_RHS_PER_THREAD; m++) tbv[m] = tb[min(tid + TAIL_THREADS * m, 3 * nt - 1)];
    keep_loads_above();
    if (dn) return;   // uniform: the whole workgroup leaves
    if (s0 + tid <= S) ssp[s0 + tid] = spv;
    for (int32_t k = s0 + tid + TAIL_THREADS; k <= S; k += TAIL_THREADS) ssp[k] = sp_g[k];
    const int32_t *sp = ssp;
#pragma unroll
    for (int m = 0; m < TAIL_RHS_PER_THREAD; m++)
        if (tid + TAIL_THREADS * m < 3 * nt) sv[tid + TAIL_THREADS * m] = tbv[m];
    lds_barrier();
    // forward: y_q = Dinv_q (b_q - its in-slots), pushes F_q y_q to its
    // up-links' slots
    auto fwd_one = [&](int32_t i, const T *d, const T *f0, const T *f1, int32_t a0, int32_t a1, int32_t b0,
                       int32_t b1) {
        T c0 = sv[3 * i], c1 = sv[3 * i + 1], c2 = sv[3 * i + 2];
        // in-slots in slot order, TAIL_SLOTS reads in flight at a time
        // (clamped addresses, surplus masked)
        for (int32_t j = b0; j < b1; j += TAIL_SLOTS) {
            const int32_t last = b1 - 1;
            T c[3 * TAIL_SLOTS];
#pragma unroll
            for (int u = 0; u < TAIL_SLOTS; u++) {
                const int32_t ju = j + u < last ? j + u : last;
                c[3 * u] = slot[3 * ju];
                c[3 * u + 1] = slot[3 * ju + 1];
                c[3 * u + 2] = slot[3 * ju + 2];
            }
#pragma unroll
            for (int u = 0; u < TAIL_SLOTS; u++) {
                const bool on = j + u < b1;
                c0 = on ? c0 - c[3 * u] : c0;
                c1 = on ? c1 - c[3 * u + 1] : c1;
                c2 = on ? c2 - c[3 * u + 2] : c2;
            }
        }
        T o0, o1, o2;
        sym_mv(d, c0, c1, c2, o0, o1, o2);
        sv[3 * i] = o0;
        sv[3 * i + 1] = o1;
        sv[3 * i + 2] = o2;
        if (a0 >= 0) {
            slot[3 * a0] = f0[0] * o0 + f0[1] * o1 + f0[2] * o2;
            slot[3 * a0 + 1] = f0[3] * o0 + f0[4] * o1 + f0[5] * o2;
            slot[3 * a0 + 2] = f0[6] * o0 + f0[7] * o1 + f0[8] * o2;
        }
        if (a1 >= 0) {
            slot[3 * a1] = f1[0] * o0 + f1[1] * o1 + f1[2] * o2;
            slot[3 * a1 + 1] = f1[3] * o0 + f1[4] * o1 + f1[5] * o2;
            slot[3 * a1 + 2] = f1[6] * o0 + f1[7] * o1 + f1[8] * o2;
        }
    };
    auto fwd_pre = [&](int32_t q, const TailPre<T> &c) {
        fwd_one(q - Qt, c.d, c.f0, c.f1, c.a0, c.a1, c.b0, c.b1);
    };
    // A step before the window: the thread's first vertex from pa (loaded
    // ahead for the first such step, here for later ones), further ones
    // loaded here.
    auto fstep = [&](int32_t k) {
        if (k > s0) {
            const int32_t q = vtx(sp, k);
            tail_load_fwd(pa, q, q - Qt, tslot, iptr, F, fs, Dinv);
        }
        const int32_t q1 = sp[k + 1];
        int32_t q = sp[k] + tid;
        if (q < q1) fwd_pre(q, pa);
        for (q += TAIL_THREADS; q < q1; q += TAIL_THREADS) {
            TailPre<T> extra;
            tail_load_fwd(extra, q, q - Qt, tslot, iptr, F, fs, Dinv);
            fwd_pre(q, extra);
        }
        lds_barrier();
    };
    for (int32_t k = s0; k < kw; k++) fstep(k);
    // the window's steps; from kx on (the last few, all of whose vertices
    // belong to wave wx) that wave alone, with wave-level syncs
    for (int32_t k = kw; k < kx; k++) {
        const int32_t lo = sp[k] - Qt, hi = sp[k + 1] - Qt;
        if (ir0 >= lo && ir0 < hi) fwd_one(ir0, R0.d, R0.f0, R0.f1, R0.slot0, R0.slot1, R0.in0, R0.in1);
        if (ir1 >= lo && ir1 < hi) fwd_one(ir1, R1.d, R1.f0, R1.f1, R1.slot0, R1.slot1, R1.in0, R1.in1);
        lds_barrier();
    }
    const bool top = (tid >> 6) == wx;
    if (top)
        for (int32_t k = kx; k < S; k++) {
            const int32_t lo = sp[k] - Qt, hi = sp[k + 1] - Qt;
            if (ir0 >= lo && ir0 < hi) fwd_one(ir0, R0.d, R0.f0, R0.f1, R0.slot0, R0.slot1, R0.in0, R0.in1);
            if (ir1 >= lo && ir1 < hi) fwd_one(ir1, R1.d, R1.f0, R1.f1, R1.slot0, R1.slot1, R1.in0, R1.in1);
            lds_wave_barrier();
        }
    // backward: x_q = y_q - Dinv_q (sum over up-links of F^T x), also written
    // to y (global) for the steps before the tail and to z
    auto bwd_one = [&](int32_t i, const T *d, const T *f0, const T *f1, int32_t a0, int32_t a1, int64_t v) {
        T c0 = 0, c1 = 0, c2 = 0;
        if (a0 >= 0) {
            const int32_t wi = a0 - Qt;
            const T x0 = sv[3 * wi], x1 = sv[3 * wi + 1], x2 = sv[3 * wi + 2];
            c0 = c0 + (f0[0] * x0 + f0[3] * x1 + f0[6] * x2);
            c1 = c1 + (f0[1] * x0 + f0[4] * x1 + f0[7] * x2);
            c2 = c2 + (f0[2] * x0 + f0[5] * x1 + f0[8] * x2);
        }
        if (a1 >= 0) {
            const int32_t wi = a1 - Qt;
            const T x0 = sv[3 * wi], x1 = sv[3 * wi + 1], x2 = sv[3 * wi + 2];
            c0 = c0 + (f1[0] * x0 + f1[3] * x1 + f1[6] * x2);
            c1 = c1 + (f1[1] * x0 + f1[4] * x1 + f1[7] * x2);
            c2 = c2 + (f1[2] * x0 + f1[5] * x1 + f1[8] * x2);
        }
        T d0, d1, d2;
        sym_mv(d, c0, c1, c2, d0, d1, d2);
        const T x0 = sv[3 * i] - d0, x1 = sv[3 * i + 1] - d1, x2 = sv[3 * i + 2] - d2;
        sv[3 * i] = x0;
        sv[3 * i + 1] = x1;
        sv[3 * i + 2] = x2;
        const int64_t q = Qt + i;
        y[3 * q] = x0;
        y[3 * q + 1] = x1;
        y[3 * q + 2] = x2;
        z[3 * v] = x0;
        z[3 * v + 1] = x1;
        z[3 * v + 2] = x2;
    };
    auto bwd_pre = [&](int32_t q, const TailPre<T> &c) {
        bwd_one(q - Qt, c.d, c.f0, c.f1, c.a0, c.a1, c.b0);
    };
    // the first backward step before the window is loaded now, while the
    // window's steps run
    {
        const int32_t q = vtx(sp, kw > s0 ? kw - 1 : s0);
        tail_load_bwd(pa, q, upq, elim, F, fs, Dinv);
    }
    if (top)
        for (int32_t k = S - 1; k >= kx; k--) {
            const int32_t lo = sp[k] - Qt, hi = sp[k + 1] - Qt;
            if (ir0 >= lo && ir0 < hi) bwd_one(ir0, R0.d, R0.f0, R0.f1, R0.up0, R0.up1, R0.id);
            if (ir1 >= lo && ir1 < hi) bwd_one(ir1, R1.d, R1.f0, R1.f1, R1.up0, R1.up1, R1.id);
            lds_wave_barrier();
        }
    lds_barrier();   // the top steps' x for every wave
    for (int32_t k = kx - 1; k >= kw; k--) {
        const int32_t lo = sp[k] - Qt, hi = sp[k + 1] - Qt;
        if (ir0 >= lo && ir0 < hi) bwd_one(ir0, R0.d, R0.f0, R0.f1, R0.up0, R0.up1, R0.id);
        if (ir1 >= lo && ir1 < hi) bwd_one(ir1, R1.d, R1.f0, R1.f1, R1.up0, R1.up1, R1.id);
        lds_barrier();
    }
    auto bstep = [&](int32_t k) {
        if (k < kw - 1) {
            const int32_t q = vtx(sp, k);
            tail_load_bwd(pa, q, upq, elim, F, fs, Dinv);
        }
        const int32_t q1 = sp[k + 1];
        int32_t q = sp[k] + tid;
        if (q < q1) bwd_pre(q, pa);
        for (q += TAIL_THREADS; q < q1; q += TAIL_THREADS) {
            TailPre<T> extra;
            tail_load_bwd(extra, q, upq, elim, F, fs, Dinv);
            bwd_pre(q, extra);
        }
        lds_barrier();
    };
    for (int32_t k = kw - 1; k >= s0; k--) bstep(k);
}

// ---------------------------------------------------------------- mid steps in LDS

// The mid steps (between the large first steps and the tail) split into
// groups of components, one workgroup each
// (mid_ptr); every push between mid vertices, and every read of x between
// them, stays inside a group.  The sweeps below keep a group's push slots and
// x values in LDS: a thread takes the group's local vertices tid and tid +
// MID_THREADS (local order: by step, then position), loads all their
// constants, their r and their slots filled by earlier launches at the start,
// and then only LDS and barriers separate the steps.  Pushes to vertices
// outside the group (later steps, the tail) and x of up-links outside it go
// through global memory as before.  Same operations in the same order as
// fwd_vertex / bwd_vertex, so results are bitwise unchanged.
constexpr int MID_THREADS = 512;
// vertices of one group at most (components are packed by their first
// vertex's offset / light_cap, so a group can exceed light_cap by up to one
// component less a vertex)
constexpr int MID_LDS_MAX = 1024;
constexpr int MID_VPT = MID_LDS_MAX / MID_THREADS;   // a thread's vertices
static_assert(MID_VPT * MID_THREADS == MID_LDS_MAX, "whole vertices per thread");

// per mid vertex (index q - Q0): local index, first LDS slot and number of
// in-entries from mid vertices; per push (2 (q - Q0) + k): its LDS slot or -1;
// per up-link: the local index of a mid up-link or -1
struct MidTab {
    const int32_t *lid, *lin0, *nint, *lsl, *lup;
};

constexpr int MID_MAX_STEPS = 64;   // mid steps at most for the LDS sweeps
constexpr int TAIL_EXTRA_WG = 255;   // extra workgroups of the tail launch that prefetch: one per other CU
static_assert(2 * MID_MAX_STEPS <= TAIL_THREADS, "the step ranges load in one round");

// the group's position range of each of its L steps, rg[2k] .. rg[2k + 1],
// loaded into LDS in one round (a walk over global memory would take a
// dependent round trip per step); ends with a barrier
SGP_DEV void mid_ranges(int32_t L, int32_t nwg, const int32_t *wptr, int32_t w, int32_t *rg)
{
    const int32_t t = threadIdx.x;
    if (t < 2 * L) rg[t] = wptr[(int64_t)(t >> 1) * nwg + w + (t & 1)];
    __syncthreads();
}

// position of local vertex l (ranges in LDS), and its step (-1: none)
SGP_DEV int32_t mid_local(int32_t L, const int32_t *rg, int32_t l, int32_t &step)
{
    int32_t cum = 0;
    step = -1;
    int32_t q = 0;
    for (int32_t k = 0; k < L; k++) {
        const int32_t a = rg[2 * k], b = rg[2 * k + 1];
        if (step < 0 && l < cum + (b - a)) {
            step = k;
            q = a + (l - cum);
        }
        cum += b - a;
    }
    return q;
}

__global__ void k_mid_nint(int32_t Q0, int32_t Q1, const int32_t *in_ptr, const int32_t *in_src, int32_t *nint)
{
    const int64_t q = Q0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q1) return;
    int32_t c = 0;
    for (int32_t t = in_ptr[q]; t < in_ptr[q + 1]; t++) c += (in_src[t] >> 1) >= Q0 ? 1 : 0;
    nint[q - Q0] = c;
}

// one workgroup per group: local indices and the first LDS slot of every
// vertex's mid in-entries (exclusive sum in local order); flag: a group with
// more than MID_LDS_MAX vertices or 2 MID_LDS_MAX slots
__global__ __launch_bounds__(MID_THREADS) void k_mid_local(int32_t L, int32_t nwg, const int32_t *wptr, int32_t Q0,
                                                           const int32_t *nint, int32_t *lid, int32_t *lin0,
                                                           int32_t *flag)
{
    __shared__ int32_t cnt[MID_LDS_MAX], tot_sh[1], rg[2 * MID_MAX_STEPS];
    const int32_t w = blockIdx.x, tid = threadIdx.x;
    if (L > MID_MAX_STEPS) {
        if (tid == 0) flag[0] = 1;
        return;
    }
    mid_ranges(L, nwg, wptr, w, rg);
    int32_t tot = 0;
    for (int32_t k = 0; k < L; k++) tot += rg[2 * k + 1] - rg[2 * k];
    if (tot > MID_LDS_MAX) {
        if (tid == 0) flag[0] = 1;
        return;
    }
    int32_t q[MID_VPT], st[MID_VPT];
    for (int u = 0; u < MID_VPT; u++) {
        const int32_t l = tid + MID_THREADS * u;
        q[u] = mid_local(L, rg, l, st[u]);
        cnt[l] = l < tot ? nint[q[u] - Q0] : 0;
    }
    __syncthreads();
    if (tid == 0) {   // exclusive sum, in local order
        int32_t s = 0;
        for (int32_t l = 0; l < tot; l++) {
            const int32_t c = cnt[l];
            cnt[l] = s;
            s += c;
        }
        tot_sh[0] = s;
        if (s > 2 * MID_LDS_MAX) flag[0] = 1;
    }
    __syncthreads();
    for (int u = 0; u < MID_VPT; u++) {
        const int32_t l = tid + MID_THREADS * u;
        if (l >= tot) continue;
        lid[q[u] - Q0] = l;
        lin0[q[u] - Q0] = cnt[l];
    }
}

// LDS slot of every push between mid vertices (the target's mid in-entries
// are the last of its in-list: sources ascend in elimination order)
__global__ void k_mid_lsl(int32_t Q0, int32_t Q1, const int32_t *in_ptr, const int32_t *in_src, const int32_t *nint,
                          const int32_t *lin0, int32_t *lsl)
{
    const int64_t q = Q0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q1) return;
    const int32_t ni = nint[q - Q0], f = in_ptr[q + 1] - ni, l0 = lin0[q - Q0];
    for (int32_t j = 0; j < ni; j++) {
        const int32_t src = in_src[f + j];
        lsl[2 * (int64_t)((src >> 1) - Q0) + (src & 1)] = l0 + j;
    }
}

__global__ void k_mid_lup(int32_t Q0, int32_t Q1, const int32_t *upq, const int32_t *lid, int32_t *lup)
{
    const int64_t q = Q0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q1) return;
    for (int k = 0; k < 2; k++) {
        const int32_t a = upq[2 * q + k];
        lup[2 * (q - Q0) + k] = a >= Q0 && a < Q1 ? lid[a - Q0] : -1;
    }
}

// the forward sweep of the mid steps: y_q = Dinv_q (r_v - its slots), the
// pushes to LDS (inside the group) or to cs (outside)
template <class T>
__global__ __launch_bounds__(MID_THREADS) void k_fwd_mid(int32_t L, int32_t nwg, const int32_t *wptr, int32_t Q0,
                                                         const int32_t *elim, const int32_t *in_ptr,
                                                         const int32_t *tout, const T *F, int64_t fs, const T *Dinv,
                                                         const T *r, T *y, T *cs, MidTab tab, const PcgScalars *s)
{
    __shared__ T sl[3 * 2 * MID_LDS_MAX];
    __shared__ int32_t rg[2 * MID_MAX_STEPS];
    if (s && s->done) return;
    const int32_t w = (int32_t)xcd_block(blockIdx.x, gridDim.x), tid = threadIdx.x;
    mid_ranges(L, nwg, wptr, w, rg);
    int32_t q[MID_VPT], st[MID_VPT], ni[MID_VPT], l0[MID_VPT], ls[MID_VPT][2], to[MID_VPT][2], t0[MID_VPT], t1[MID_VPT];
    int64_t v[MID_VPT];
    T d[MID_VPT][6], f0[MID_VPT][9], f1[MID_VPT][9], b[MID_VPT][3], h[MID_VPT][12];
    // two rounds of loads for both vertices: what the position gives, then
    // what those values address (r, the second coupling, the first four slots
    // filled by earlier launches, clamped); one wait between them
#pragma unroll
    for (int u = 0; u < MID_VPT; u++) {
        q[u] = mid_local(L, rg, tid + MID_THREADS * u, st[u]);
        const int32_t qc = st[u] >= 0 ? q[u] : Q0;   // a thread without a vertex loads a valid one
        v[u] = elim[qc];
        t0[u] = in_ptr[qc];
        t1[u] = in_ptr[qc + 1];
        ni[u] = tab.nint[qc - Q0];
        l0[u] = tab.lin0[qc - Q0];
        for (int k = 0; k < 2; k++) {
            to[u][k] = tout[2 * qc + k];
            ls[u][k] = tab.lsl[2 * (int64_t)(qc - Q0) + k];
        }
        for (int t = 0; t < 6; t++) d[u][t] = Dinv[6 * (int64_t)qc + t];
        for (int t = 0; t < 9; t++) f0[u][t] = F[9 * (int64_t)qc + t];
    }
    keep_loads_above();
#pragma unroll
    for (int u = 0; u < MID_VPT; u++) {
        const int32_t qc = st[u] >= 0 ? q[u] : Q0;
        b[u][0] = r[3 * v[u]];
        b[u][1] = r[3 * v[u] + 1];
        b[u][2] = r[3 * v[u] + 2];
        // (the second plane is zero without a second link)
        for (int t = 0; t < 9; t++) f1[u][t] = F[fs + 9 * (int64_t)qc + t];
        const int32_t te = t1[u] - ni[u], last = te > t0[u] ? te - 1 : t0[u];
        for (int m = 0; m < 4; m++) {
            const T *c = cs + 3 * (int64_t)min(t0[u] + m, last);
            h[u][3 * m] = c[0];
            h[u][3 * m + 1] = c[1];
            h[u][3 * m + 2] = c[2];
        }
    }
    keep_loads_above();
    // r minus the slots filled by earlier launches (the first in-entries), in
    // slot order: the first four from h, any further ones loaded here
#pragma unroll
    for (int u = 0; u < MID_VPT; u++) {
        const int32_t te = t1[u] - ni[u];
        for (int m = 0; m < 4; m++)
            if (t0[u] + m < te) {
                b[u][0] = b[u][0] - h[u][3 * m];
                b[u][1] = b[u][1] - h[u][3 * m + 1];
                b[u][2] = b[u][2] - h[u][3 * m + 2];
            }
        if (t0[u] + 4 < te) sum_slots<T>(t0[u] + 4, te, cs, b[u][0], b[u][1], b[u][2]);
    }
    for (int32_t k = 0; k < L; k++) {
#pragma unroll
        for (int u = 0; u < MID_VPT; u++) {
            if (st[u] != k) continue;
            T c0 = b[u][0], c1 = b[u][1], c2 = b[u][2];
            for (int32_t j = 0; j < ni[u]; j++) {
                const T *c = sl + 3 * (l0[u] + j);
                c0 = c0 - c[0];
                c1 = c1 - c[1];
                c2 = c2 - c[2];
            }
            T o0, o1, o2;
            sym_mv(d[u], c0, c1, c2, o0, o1, o2);
            const int64_t qq = q[u];
            y[3 * qq] = o0;
            y[3 * qq + 1] = o1;
            y[3 * qq + 2] = o2;
            for (int m = 0; m < 2; m++) {
                if (to[u][m] < 0) continue;
                const T *g = m == 0 ? f0[u] : f1[u];
                T *c = ls[u][m] >= 0 ? sl + 3 * ls[u][m] : cs + 3 * (int64_t)to[u][m];
                c[0] = g[0] * o0 + g[1] * o1 + g[2] * o2;
                c[1] = g[3] * o0 + g[4] * o1 + g[5] * o2;
                c[2] = g[6] * o0 + g[7] * o1 + g[8] * o2;
            }
        }
        // LDS only: the global stores (y, z, pushes out of the group) are
        // read by no thread of this launch
        lds_barrier();
    }
}

// the backward sweep of the mid steps: x_q = y_q - Dinv_q (sum over up-links
// of F^T x), x of a mid up-link from LDS, of others from y; x written to y
// (for the steps below) and to z
template <class T>
__global__ __launch_bounds__(MID_THREADS) void k_bwd_mid(int32_t L, int32_t nwg, const int32_t *wptr, int32_t Q0,
                                                         const int32_t *elim, const int32_t *upq, const T *F,
                                                         int64_t fs, const T *Dinv, T *y, T *z, MidTab tab,
                                                         const PcgScalars *s)
{
    __shared__ T xl[3 * MID_LDS_MAX];
    __shared__ int32_t rg[2 * MID_MAX_STEPS];
    if (s && s->done) return;
    const int32_t w = (int32_t)xcd_block(blockIdx.x, gridDim.x), tid = threadIdx.x;
    mid_ranges(L, nwg, wptr, w, rg);
    int32_t q[MID_VPT], st[MID_VPT], lu[MID_VPT][2], ua[MID_VPT][2];
    int64_t v[MID_VPT];
    T d[MID_VPT][6], f0[MID_VPT][9], f1[MID_VPT][9], yo[MID_VPT][3], xo[MID_VPT][2][3];
    // two rounds of loads for both vertices, one wait between them
#pragma unroll
    for (int u = 0; u < MID_VPT; u++) {
        q[u] = mid_local(L, rg, tid + MID_THREADS * u, st[u]);
        const int32_t qc = st[u] >= 0 ? q[u] : Q0;
        v[u] = elim[qc];
        for (int k = 0; k < 2; k++) {
            ua[u][k] = upq[2 * qc + k];
            lu[u][k] = tab.lup[2 * (int64_t)(qc - Q0) + k];
        }
        for (int t = 0; t < 6; t++) d[u][t] = Dinv[6 * (int64_t)qc + t];
        for (int t = 0; t < 9; t++) f0[u][t] = F[9 * (int64_t)qc + t];
        for (int t = 0; t < 9; t++) f1[u][t] = F[fs + 9 * (int64_t)qc + t];
        for (int t = 0; t < 3; t++) yo[u][t] = y[3 * (int64_t)qc + t];
    }
    keep_loads_above();
    // x of up-links outside the group (final: swept by earlier launches)
#pragma unroll
    for (int u = 0; u < MID_VPT; u++) {
        const int32_t qc = st[u] >= 0 ? q[u] : Q0;
        for (int k = 0; k < 2; k++) {
            const int64_t a = ua[u][k] >= 0 && lu[u][k] < 0 ? ua[u][k] : qc;
            for (int t = 0; t < 3; t++) xo[u][k][t] = y[3 * a + t];
        }
    }
    for (int32_t k = L - 1; k >= 0; k--) {
#pragma unroll
        for (int u = 0; u < MID_VPT; u++) {
            if (st[u] != k) continue;
            T a0 = 0, a1 = 0, a2 = 0;
            for (int m = 0; m < 2; m++) {
                if (ua[u][m] < 0) continue;
                const T *g = m == 0 ? f0[u] : f1[u];
                T x0 = xo[u][m][0], x1 = xo[u][m][1], x2 = xo[u][m][2];
                if (lu[u][m] >= 0) {
                    const T *xs = xl + 3 * lu[u][m];
                    x0 = xs[0];
                    x1 = xs[1];
                    x2 = xs[2];
                }
                a0 = a0 + (g[0] * x0 + g[3] * x1 + g[6] * x2);
                a1 = a1 + (g[1] * x0 + g[4] * x1 + g[7] * x2);
                a2 = a2 + (g[2] * x0 + g[5] * x1 + g[8] * x2);
            }
            T e0, e1, e2;
            sym_mv(d[u], a0, a1, a2, e0, e1, e2);
            const T n0 = yo[u][0] - e0, n1 = yo[u][1] - e1, n2 = yo[u][2] - e2;
            const int32_t l = tid + MID_THREADS * u;
            xl[3 * l] = n0;
            xl[3 * l + 1] = n1;
            xl[3 * l + 2] = n2;
            const int64_t qq = q[u];
            y[3 * qq] = n0;
            y[3 * qq + 1] = n1;
            y[3 * qq + 2] = n2;
            z[3 * v[u]] = n0;
            z[3 * v[u] + 1] = n1;
            z[3 * v[u] + 2] = n2;
        }
        // LDS only: the global stores (y, z, pushes out of the group) are
        // read by no thread of this launch
        lds_barrier();
    }
}

int tail_setup_attr(sgp_ctx ctx)
{
    static bool done = false;
    if (done) return SGP_OK;
    HIP_TRY(ctx, hipFuncSetAttribute((const void *)k_tail<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     TAIL_LDS_BYTES));
    HIP_TRY(ctx, hipFuncSetAttribute((const void *)k_tail<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     TAIL_LDS_BYTES));
    done = true;
    return SGP_OK;
}

// tail tables: internal flags of the tail targets' in-entries, their ranks,
// each target's first internal rank, each tail source's slot
__global__ void k_tail_flags(int32_t t0, int32_t t1, const int32_t *in_src, int32_t Qt, int32_t *flag)
{
    int32_t t = t0 + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t < t1) flag[t - t0] = (in_src[t] >> 1) >= Qt ? 1 : 0;
}

__global__ void k_tail_tables(int32_t Qt, int32_t nt, int32_t t0, const int32_t *in_ptr, const int32_t *tout,
                              const int32_t *rank, int32_t *iptr, int32_t *tslot)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nt) return;
    iptr[i] = rank[in_ptr[Qt + i] - t0];
    if (i == nt) return;
    for (int k = 0; k < 2; k++) {
        int32_t to = tout[2 * (Qt + i) + k];
        tslot[2 * i + k] = to >= 0 ? rank[to - t0] : -1;
    }
}

template <class T>
__global__ void k_jacobi_apply(int64_t n, const T *dinv, const T *r, T *z, const PcgScalars *s)
{
    if (s && s->done) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T o0, o1, o2;
    sym_mv(dinv + 6 * i, r[3 * i], r[3 * i + 1], r[3 * i + 2], o0, o1, o2);
    z[3 * i] = o0;
    z[3 * i + 1] = o1;
    z[3 * i + 2] = o2;
}

template <class T>
__global__ void k_copy_vec(int64_t len, const T *a, T *b, const PcgScalars *s)
{
    if (s && s->done) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) b[i] = a[i];
}

// The first elimination step runs as launches of its own (k_fwd_step0,
// k_bwd_step0): its vertices (elimination positions 0..q1-1) are then in the
// internal order, since the schedule's sort is stable and gives them all the
// same key.  Returns q1, or 0 where that step is swept otherwise (light
// subtrees, grouped components, the tail) or the factor has no (w, u) table.
int32_t prec_step0_launch(sgp_prec M)
{
    if (!M || M->kind != PREC_TREE || M->n_wu0 <= 0 || !M->step0_sorted || M->light_steps > 0 || M->tail_step <= 0)
        return 0;
    if ((int64_t)M->h_step_ptr.size() < 2 || M->n_wu0 != M->h_step_ptr[1]) return 0;
    const int32_t m1 = std::min(M->mid_step0 + M->mid_steps, M->tail_step);
    if (M->mid_steps > 0 && M->mid_step0 == 0 && m1 >= 2) return 0;
    return M->h_step_ptr[1];
}

// skip0: leave out the first elimination step (both sweeps); the caller runs
// it (the fused vector passes of the CG), only where prec_step0_launch > 0
template <class T>
static int tree_sweeps(sgp_ctx ctx, sgp_prec M, const T *F, const T *Dinv, T *y, T *cs, const T *r, T *z,
                       PcgScalars *s, const T *wu0, bool skip0, SideX *side)
{
    hipStream_t st = ctx->stream;
    // r and z are in the internal order
    const int32_t *elim = (const int32_t *)M->elim_int.p, *in_ptr = (const int32_t *)M->in_ptr.p;
    const int32_t *tout = (const int32_t *)M->tout.p, *upq = (const int32_t *)M->up.p;
    const int32_t *dsp = (const int32_t *)M->step_ptr.p;
    const std::vector<int32_t> &sp = M->h_step_ptr;
    const int32_t S = M->steps, ts = M->tail_step, L = M->light_steps;
    const int64_t fs = 9 * M->n;   // second plane of F
    const int32_t *wptr = (const int32_t *)M->light_ptr.p;
    if (L > 0)
        k_fwd_light<T><<<M->light_nwg, 256, 0, st>>>(L, M->light_nwg, wptr, elim, in_ptr, tout, F, fs, Dinv, r, y,
                                                    cs, s);
    // the first step from the contacts' (w, u) when it is one of these launches
    const bool step0_wu = wu0 && L == 0 && ts > 0 && M->n_wu0 == sp[1];
    const T gp = (T)M->gpar, gq = (T)M->gperp, gm = (T)M->gmed;
    // the mid steps m0..m1-1 below the tail: one launch per sweep, a
    // workgroup per packed group of components
    const int32_t m0 = M->mid_step0, m1 = std::min(M->mid_step0 + M->mid_steps, ts);
    const bool mid = M->mid_steps > 0 && m0 >= L && m1 - m0 >= 2;
    const int32_t *mptr = (const int32_t *)M->mid_ptr.p;
    // the mid steps in LDS when their tables were built (knob mid_lds)
    const bool mid_lds = mid && M->mid_lds && ctx->mid_lds && m0 >= 1;
    MidTab mtab = {};
    if (mid_lds) {
        const int32_t Nm = sp[m1] - sp[m0];
        const int32_t *tb = (const int32_t *)M->mid_tab.p;
        mtab = {tb, tb + Nm, tb + 2 * (size_t)Nm, tb + 3 * (size_t)Nm, tb + 5 * (size_t)Nm};
    }
    for (int k = L; k < ts; k++) {
        int32_t q0 = sp[k], q1 = sp[k + 1];
        if (mid && k == m0 && mid_lds) {
            k_fwd_mid<T><<<M->mid_nwg, MID_THREADS, 0, st>>>(m1 - m0, M->mid_nwg, mptr, sp[m0], elim, in_ptr, tout, F,
                                                            fs, Dinv, r, y, cs, mtab, s);
            k = m1 - 1;
            continue;
        }
        if (mid && k == m0) {
            k_fwd_light<T><<<M->mid_nwg, 256, 0, st>>>(m1 - m0, M->mid_nwg, mptr, elim, in_ptr, tout, F, fs, Dinv, r,
                                                       y, cs, s);
            k = m1 - 1;
            continue;
        }
        if (k == 0 && step0_wu && skip0) continue;
        if (k == 0 && step0_wu)
            k_fwd_step0<T><<<grid_for(q1, 256), 256, 0, st>>>(q1, elim, tout, wu0, 4 * (int64_t)q1, gp, gq, gm, Dinv,
                                                              r, y, cs, s);
        else if (q1 > q0)
            k_fwd_step<T><<<grid_for(q1 - q0, 256), 256, 0, st>>>(q0, q1, elim, in_ptr, tout, F, fs, Dinv, r, y, cs,
                                                                  s);
    }
    if (ts < S) {
        size_t lds = tail_lds_bytes(sizeof(T), M->tail_nt, M->tail_ni, S - ts);
        const int32_t nt = M->tail_nt;
        if (nt > TAIL_MAX_VERTICES) return set_err(ctx, SGP_EINVAL, "tree sweeps: tail of %d vertices", nt);
        T *tb = (T *)M->tail_b.p;
        // and TAIL_PF_WG more workgroups that prefetch the tail's constants
        // (knob prefetch)
        const int32_t npre = (nt + 63) / 64;
        const int32_t *tslot = (const int32_t *)M->tail_tslot.p;
        k_tail_pre<T><<<npre + (ctx->prefetch ? TAIL_PF_WG : 0), 64, 0, st>>>(
            sp[ts], nt, elim, in_ptr, (const int32_t *)M->tail_iptr.p, r, cs, tb, s, npre, F, fs, Dinv, tslot, upq, 0);
        // the first step whose vertices all lie in the last TAIL_WINDOW tail vertices
        const int32_t base = nt > TAIL_WINDOW ? nt - TAIL_WINDOW : 0;
        int32_t kw = ts;
        while (kw < S && sp[kw] - sp[ts] < base) kw++;
        const int32_t q1a = kw > ts ? sp[ts + 1] : sp[ts] + 1;
        // extra workgroups take the CG's x update (a block holds at most
        // 2 TAIL_THREADS values)
        SideX sd = {};
        if (side && side->nb > 0 && side->nwg > 0) {
            sd = *side;
            side->ran = true;
        }
        // and, one per other CU, they load the backward mid steps' constants
        // ahead of k_bwd_mid (knob prefetch)
        sd.wait = !ctx->prefetch;
        if (ctx->prefetch && mid_lds) {
            sd.mid_wptr = mptr;
            sd.mid_lup = mtab.lup;
            sd.mid_L = m1 - m0;
            sd.mid_nwg = M->mid_nwg;
            sd.mid_Q0 = sp[m0];
            sd.nwg = TAIL_EXTRA_WG;
            lds = std::max(lds, (size_t)(2 * MID_MAX_STEPS * sizeof(int32_t)));
        }
        // the last window steps whose vertices all belong to one wave (the
        // owner of tail-local index i: i - base in the first half of the
        // window, i - base - TAIL_THREADS in the second), which sweeps them
        // alone
        int32_t kx = S, wx = 0;
        if (kw < S) {
            auto owner = [&](int32_t i) { return i < base + TAIL_THREADS ? i - base : i - base - TAIL_THREADS; };
            const bool hi_half = nt - 1 >= base + TAIL_THREADS;
            wx = owner(nt - 1) / 64;
            for (int32_t k = S - 1; k >= kw; k--) {
                const int32_t lo = sp[k] - sp[ts];
                if (lo < base || (lo >= base + TAIL_THREADS) != hi_half || owner(lo) / 64 != wx) break;
                kx = k;
            }
        }
        k_tail<T><<<1 + (unsigned)sd.nwg, TAIL_THREADS, lds, st>>>(
            ts, S, kw, kx, wx, sp[ts], q1a, nt, M->tail_ni, dsp, elim, in_ptr, (const int32_t *)M->tail_iptr.p,
            tslot, upq, F, fs, Dinv, tb, y, z, s, sd);
    }
    for (int k = ts - 1; k >= L; k--) {
        int32_t q0 = sp[k], q1 = sp[k + 1];
        if (mid && k == m1 - 1 && mid_lds) {
            k_bwd_mid<T><<<M->mid_nwg, MID_THREADS, 0, st>>>(m1 - m0, M->mid_nwg, mptr, sp[m0], elim, upq, F, fs, Dinv,
                                                            y, z, mtab, s);
            k = m0;
            continue;
        }
        if (mid && k == m1 - 1) {
            k_bwd_light<T><<<M->mid_nwg, 256, 0, st>>>(m1 - m0, M->mid_nwg, mptr, elim, upq, F, fs, Dinv, y, z, s);
            k = m0;
            continue;
        }
        if (k == 0 && step0_wu && skip0) continue;
        if (k == 0 && step0_wu)
            k_bwd_step0<T><<<grid_for(q1, 256), 256, 0, st>>>(q1, elim, upq, wu0, 4 * (int64_t)q1, gp, gq, gm, Dinv,
                                                              y, z, s);
        else if (q1 > q0)
            k_bwd_step<T><<<grid_for(q1 - q0, 256), 256, 0, st>>>(q0, q1, elim, upq, F, fs, Dinv, y, z, s, k > 0);
    }
    if (L > 0)
        k_bwd_light<T><<<M->light_nwg, 256, 0, st>>>(L, M->light_nwg, wptr, elim, upq, F, fs, Dinv, y, z, s);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

int prec_apply_f64(sgp_ctx ctx, sgp_prec M, const double *r, double *z, PcgScalars *s, bool skip0, SideX *side)
{
    hipStream_t st = ctx->stream;
    if (!M || M->kind == PREC_NONE) {
        int64_t len = 3 * (M ? M->n : 0);
        (void)len;
        return set_err(ctx, SGP_EINVAL, "prec_apply: identity handled by caller");
    }
    if (M->kind == PREC_JACOBI) {
        k_jacobi_apply<double><<<grid_for(M->n, 256), 256, 0, st>>>(M->n, (const double *)M->jdinv.p, r, z, s);
        LAUNCH_CHECK(ctx);
        return SGP_OK;
    }
    return tree_sweeps<double>(ctx, M, (const double *)M->F.p, (const double *)M->Dinv.p, (double *)M->y.p,
                               (double *)M->cs.p, r, z, s, M->n_wu0 > 0 ? (const double *)M->wu0.p : nullptr,
                               skip0 && prec_step0_launch(M) > 0, side);
}

int prec_apply_f32(sgp_ctx ctx, sgp_prec M, const float *r, float *z, PcgScalars *s, bool skip0, SideX *side)
{
    hipStream_t st = ctx->stream;
    if (M->kind == PREC_JACOBI) {
        k_jacobi_apply<float><<<grid_for(M->n, 256), 256, 0, st>>>(M->n, (const float *)M->Dinv32.p, r, z, s);
        LAUNCH_CHECK(ctx);
        return SGP_OK;
    }
    return tree_sweeps<float>(ctx, M, (const float *)M->F32.p, (const float *)M->Dinv32.p, (float *)M->y32.p,
                              (float *)M->cs32.p, r, z, s, M->n_wu0 > 0 ? (const float *)M->wu032.p : nullptr,
                              skip0 && prec_step0_launch(M) > 0, side);
}

__global__ void k_to_f32(int64_t len, const double *a, float *b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) b[i] = (float)a[i];
}

// FP32 copies of the factors: computed in FP64, rounded once
int prec_make32(sgp_ctx ctx, sgp_prec M)
{
    if (M->have32) return SGP_OK;
    hipStream_t st = ctx->stream;
    int64_t n = M->n;
    float *F32, *D32, *y32;
    if (M->kind == PREC_TREE) {
        float *cs32;
        SGP_TRY(ensure_t(ctx, M->F32, 18 * n + 1, &F32));
        SGP_TRY(ensure_t(ctx, M->Dinv32, 6 * n + 1, &D32));
        SGP_TRY(ensure_t(ctx, M->y32, 3 * n + 1, &y32));
        SGP_TRY(ensure_t(ctx, M->cs32, 6 * n + 6, &cs32));
        k_to_f32<<<grid_for(18 * n, 256), 256, 0, st>>>(18 * n, (const double *)M->F.p, F32);
        k_to_f32<<<grid_for(6 * n, 256), 256, 0, st>>>(6 * n, (const double *)M->Dinv.p, D32);
        if (M->n_wu0 > 0) {
            float *w32;
            SGP_TRY(ensure_t(ctx, M->wu032, 8 * M->n_wu0 + 8, &w32));
            k_to_f32<<<grid_for(8 * M->n_wu0, 256), 256, 0, st>>>(8 * M->n_wu0, (const double *)M->wu0.p, w32);
        }
    } else if (M->kind == PREC_JACOBI) {
        SGP_TRY(ensure_t(ctx, M->Dinv32, 6 * n + 1, &D32));
        k_to_f32<<<grid_for(6 * n, 256), 256, 0, st>>>(6 * n, (const double *)M->jdinv.p, D32);
    }
    LAUNCH_CHECK(ctx);
    M->have32 = true;
    return SGP_OK;
}

__global__ void k_pair(const int32_t *a, const int32_t *b, int32_t *out)
{
    out[0] = *a;
    out[1] = *b;
}

static int tail_tables(sgp_ctx ctx, sgp_prec M, int64_t n, const int32_t *in_ptr, const int32_t *in_src,
                       const int32_t *tout)
{
    hipStream_t st = ctx->stream;
    M->tail_nt = 0;
    M->tail_ni = 0;
    if (M->tail_step >= M->steps) return SGP_OK;
    SGP_TRY(tail_setup_attr(ctx));
    const int32_t Qt = M->h_step_ptr[M->tail_step];
    const int32_t nt = (int32_t)(n - Qt);
    int32_t hin[2], *pair;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PAIR], 2, &pair));
    k_pair<<<1, 1, 0, st>>>(in_ptr + Qt, in_ptr + n, pair);
    LAUNCH_CHECK(ctx);
    SGP_TRY(readback(ctx, hin, pair, sizeof hin));
    const int32_t t0 = hin[0], t1 = hin[1];
    int32_t *flag, *rank, *iptr, *tslot;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP8], (size_t)(t1 - t0) + 2, &flag));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP7], (size_t)(t1 - t0) + 2, &rank));
    SGP_TRY(ensure_t(ctx, M->tail_iptr, (size_t)nt + 2, &iptr));
    SGP_TRY(ensure_t(ctx, M->tail_tslot, 2 * (size_t)nt + 2, &tslot));
    double *tb;
    SGP_TRY(ensure_t(ctx, M->tail_b, 3 * (size_t)nt + 3, &tb));   // FP64 or FP32 sweeps
    if (t1 > t0) k_tail_flags<<<grid_for(t1 - t0, 256), 256, 0, st>>>(t0, t1, in_src, Qt, flag);
    SGP_TRY(scan_exclusive(ctx, flag, rank, t1 - t0));
    k_tail_tables<<<grid_for(nt + 1, 256), 256, 0, st>>>(Qt, nt, t0, in_ptr, tout, rank, iptr, tslot);
    LAUNCH_CHECK(ctx);
    int32_t ni;
    SGP_TRY(readback(ctx, &ni, rank + (t1 - t0), 4));
    M->tail_nt = nt;
    M->tail_ni = ni;
    if (tail_lds_bytes(8, nt, ni, M->steps - M->tail_step) > (size_t)TAIL_LDS_BYTES)
        return set_err(ctx, SGP_EINVAL, "factor_tree: tail does not fit in LDS (%d + %d)", nt, ni);
    return SGP_OK;
}

// the tables of the LDS mid sweeps (MidTab); flag[0] set when a group is too
// large for them (the caller then keeps the generic workgroup sweeps)
static int mid_tables(sgp_ctx ctx, sgp_prec M, const int32_t *in_ptr, const int32_t *in_src, const int32_t *upq,
                      int32_t *flag)
{
    hipStream_t st = ctx->stream;
    M->mid_lds_built = false;
    if (M->mid_steps <= 0 || M->light_steps > 0) return SGP_OK;
    const int32_t m0 = M->mid_step0, m1 = std::min(M->mid_step0 + M->mid_steps, M->tail_step);
    // (grouped from step 0: the local forest keeps its sweeps)
    if (m1 - m0 < 2 || m1 - m0 > MID_MAX_STEPS || m0 < 1) return SGP_OK;
    const int32_t Q0 = M->h_step_ptr[m0], Q1 = M->h_step_ptr[m1], Nm = Q1 - Q0;
    if (Nm <= 0) return SGP_OK;
    int32_t *tb;
    SGP_TRY(ensure_t(ctx, M->mid_tab, 7 * (size_t)Nm + 8, &tb));
    int32_t *lid = tb, *lin0 = tb + Nm, *nint = tb + 2 * (size_t)Nm, *lsl = tb + 3 * (size_t)Nm,
            *lup = tb + 5 * (size_t)Nm;
    SGP_TRY(fill_i32(ctx, lsl, -1, 2 * (int64_t)Nm));
    k_mid_nint<<<grid_for(Nm, 256), 256, 0, st>>>(Q0, Q1, in_ptr, in_src, nint);
    k_mid_local<<<M->mid_nwg, MID_THREADS, 0, st>>>(m1 - m0, M->mid_nwg, (const int32_t *)M->mid_ptr.p, Q0, nint, lid,
                                                    lin0, flag);
    k_mid_lsl<<<grid_for(Nm, 256), 256, 0, st>>>(Q0, Q1, in_ptr, in_src, nint, lin0, lsl);
    k_mid_lup<<<grid_for(Nm, 256), 256, 0, st>>>(Q0, Q1, upq, lid, lup);
    LAUNCH_CHECK(ctx);
    M->mid_lds_built = true;
    return SGP_OK;
}

// ---------------------------------------------------------------- entry points

extern "C" int sgp_factor_tree(sgp_ctx ctx, sgp_graph g, sgp_tree T, double g_par, double g_perp, double g_med,
                               int32_t schedule, sgp_prec M)
{
    if (!ctx || !g || !T || !M) return set_err(ctx, SGP_EINVAL, "factor_tree: null handle");
    if (!(g_par > 0) || !(g_perp > 0) || !(g_med >= 0))
        return set_err(ctx, SGP_EINVAL, "factor_tree: friction coefficients must be positive");
    if (schedule != SGP_SCHED_LEVEL && schedule != SGP_SCHED_CONTRACT)
        return set_err(ctx, SGP_EINVAL, "factor_tree: unknown schedule %d", schedule);
    if (T->n != g->n) return set_err(ctx, SGP_EINVAL, "factor_tree: tree and graph differ in size");
    hipStream_t st = ctx->stream;
    phase_begin(ctx, 3);
    const int64_t n = g->n;
    M->kind = PREC_TREE;
    M->gen = next_gen();
    M->n = n;
    M->schedule = schedule;
    M->have32 = false;
    M->aug = 0;
    M->light_steps = 0;
    M->light_nwg = 0;
    if (n == 0) {
        M->steps = 0;
        M->h_step_ptr.assign(1, 0);
        return SGP_OK;
    }
    int32_t *stepv, *up0, *up1, *hbuf = (int32_t *)ctx->pinned;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP0], n + 1, &stepv));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP1], n + 1, &up0));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP2], n + 1, &up1));
    const int32_t *parent = (const int32_t *)T->parent.p;
    int32_t S = 0;
    int32_t light = 0, nwg = 1;   // light steps and their workgroups (CONTRACT only)
    int32_t *wgv = nullptr;       // workgroup of every light vertex
    if (schedule == SGP_SCHED_LEVEL) {
        k_sched_level<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)T->depth.p, parent, T->max_depth, stepv,
                                                      up0, up1);
        LAUNCH_CHECK(ctx);
        S = T->max_depth + 1;
    } else {
        int32_t *par, *nch, *xch, *stat;
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], n + 1, &par));
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], n + 1, &nch));
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP5], n + 1, &xch));
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP6], 2 * SCHED_STAT_BLOCKS + 4, &stat));   // per-block stats, then out[2]
        SGP_TRY(fill_i32(ctx, nch, 0, n));
        SGP_TRY(fill_i32(ctx, xch, 0, n));
        k_contract_init<<<grid_for(n, 256), 256, 0, st>>>(n, parent, par, nch, xch, stepv);
        LAUNCH_CHECK(ctx);
        const int stat_nb = (int)std::min<int64_t>(SCHED_STAT_BLOCKS, grid_for(n, 256));
        int32_t *stat_out = stat + 2 * SCHED_STAT_BLOCKS;
        // host copy of (unscheduled, largest step) after the rounds so far
        auto progress = [&](int64_t &alive, int32_t &maxstep) -> int {
            k_sched_stats<<<stat_nb, 256, 0, st>>>(n, stepv, stat);
            k_sched_final<<<1, 256, 0, st>>>(stat_nb, stat, stat_out);
            LAUNCH_CHECK(ctx);
            SGP_TRY(readback(ctx, hbuf, stat_out, 8));
            alive = hbuf[0];
            maxstep = hbuf[1];
            return SGP_OK;
        };
        int64_t done = 0;
        // rake-only rounds: the light subtrees
        while (done < n && S < ctx->light_height) {
            k_rake_select<<<grid_for(n, 256), 256, 0, st>>>(n, S, par, nch, stepv, up0, up1);
            k_contract_apply<<<grid_for(n, 256), 256, 0, st>>>(n, S, stepv, up0, up1, par, nch, xch);
            LAUNCH_CHECK(ctx);
            S++;
            int64_t alive;
            int32_t maxstep;
            SGP_TRY(progress(alive, maxstep));
            if (n - alive <= done) return set_err(ctx, SGP_EINVAL, "factor_tree: raking made no progress");
            done = n - alive;
        }
        // a tree raked away completely runs as ordinary steps
        if (S > 0 && done < n) {
            light = S;
            int32_t *ja, *jb, *lcnt, *lstart, *wgr;
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_A], n + 1, &ja));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_B], n + 1, &jb));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP7], n + 1, &lcnt));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP8], n + 2, &lstart));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_B], n + 1, &wgr));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP9], n + 1, &wgv));
            k_light_init<<<grid_for(n, 256), 256, 0, st>>>(n, parent, stepv, ja);
            // a light vertex is at most `light` - 1 links below its root
            for (int span = 1; span < light; span *= 2) {
                k_light_jump<<<grid_for(n, 256), 256, 0, st>>>(n, ja, jb);
                std::swap(ja, jb);
            }
            SGP_TRY(fill_i32(ctx, lcnt, 0, n));
            k_light_count<<<grid_for(n, 256), 256, 0, st>>>(n, ja, lcnt);
            k_light_vals<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)g->perm.p, ja, lcnt, jb);
            LAUNCH_CHECK(ctx);
            SGP_TRY(scan_exclusive(ctx, jb, lstart, n));
            int32_t total;
            SGP_TRY(readback(ctx, &total, lstart + n, 4));
            const int32_t cap = std::max(ctx->light_cap, 1);
            nwg = (total + cap - 1) / cap;
            k_light_rootwg<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)g->perm.p, ja, lstart, cap, wgr);
            k_light_wg<<<grid_for(n, 256), 256, 0, st>>>(n, ja, wgr, wgv);
            LAUNCH_CHECK(ctx);
        }
        // rounds in batches of ROUNDS_PER_READ with one readback of the
        // progress: rounds past the last vertex select nothing, and every
        // round before it schedules at least one vertex (a forest always has
        // a leaf), so the step count is the largest step given plus one
        constexpr int ROUNDS_PER_READ = 8;
        while (done < n) {
            if (S > 100000) return set_err(ctx, SGP_EINVAL, "factor_tree: contraction did not finish");
            for (int b = 0; b < ROUNDS_PER_READ; b++) {
                const int32_t s = S + b;
                k_contract_select<<<grid_for(n, 256), 256, 0, st>>>(n, s, par, nch, xch, stepv, up0, up1);
                if (s == 0)
                    k_contract_pull0<<<grid_for(n, 256), 256, 0, st>>>(n, parent, (const int32_t *)T->tptr.p,
                                                                      (const int32_t *)T->tadj.p, stepv, up0, up1,
                                                                      par, nch, xch);
                else
                    k_contract_apply<<<grid_for(n, 256), 256, 0, st>>>(n, s, stepv, up0, up1, par, nch, xch);
            }
            LAUNCH_CHECK(ctx);
            int64_t alive;
            int32_t maxstep;
            SGP_TRY(progress(alive, maxstep));
            if (n - alive <= done) return set_err(ctx, SGP_EINVAL, "factor_tree: contraction made no progress");
            done = n - alive;
            S = maxstep + 1;
        }
    }
    M->steps = S;
    M->mid_step0 = M->mid_steps = M->mid_nwg = 0;
    // elimination order: by (step, id)
    uint32_t *ka, *kb;
    int32_t *elim, *vb, *pos, *scnt, *sptr;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_A], 2 * n + 2, &ka));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_B], 2 * n + 2, &kb));
    SGP_TRY(ensure_t(ctx, M->elim, n + 1, &elim));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_B], 2 * n + 2, &vb));
    SGP_TRY(ensure_t(ctx, M->pos, n + 1, &pos));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP7], (size_t)S + 2, &scnt));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP8], (size_t)S + 2, &sptr));
    (void)scnt;
    SGP_TRY(copy_order(ctx, M->perm, M->inv, g->perm, g->inv, n));
    int32_t *elim_int;
    SGP_TRY(ensure_t(ctx, M->elim_int, n + 1, &elim_int));
    // keys (step, workgroup of a light or mid vertex, else 0); the sort is
    // stable, so the vertices of one key stay in the internal order
    auto order = [&](const int32_t *wg, int32_t nw) -> int {
        if ((int64_t)S * nw >= ((int64_t)1 << 31)) return set_err(ctx, SGP_EINVAL, "factor_tree: schedule too large");
        int sbits = 1;
        while (((int64_t)1 << sbits) < (int64_t)S * nw) sbits++;
        k_stepkeys<<<grid_for(n, 256), 256, 0, st>>>(n, stepv, wg, (uint32_t)nw, (const int32_t *)g->perm.p, ka,
                                                   elim);
        LAUNCH_CHECK(ctx);
        SGP_TRY(radix_sort_pairs(ctx, ka, elim, kb, vb, n, sbits));
        k_map_ids<<<grid_for(n, 256), 256, 0, st>>>(n, elim, (const int32_t *)g->inv.p, elim_int);
        k_invperm<<<grid_for(n, 256), 256, 0, st>>>(n, elim, pos);
        k_step_bounds<<<grid_for(n + 1, 256), 256, 0, st>>>(n, ka, (uint32_t)nw, S, sptr);
        LAUNCH_CHECK(ctx);
        M->h_step_ptr.resize(S + 1);
        return readback(ctx, M->h_step_ptr.data(), sptr, (S + 1) * sizeof(int32_t));
    };
    M->light_steps = light;
    M->light_nwg = light ? nwg : 0;
    // the mid steps (CONTRACT without light steps): from the first step
    // (after the first two) with at most MID_MAX_VERTICES vertices left, up to
    // the first step with at most the default tail size left.  Fixed by the
    // schedule alone (not by tail_max), so the elimination order does not
    // depend on the tail.  The step sizes come from a histogram of the steps,
    // the components' workgroups from the labelling, and one sort orders the
    // vertices by (step, workgroup).
    int32_t *mw = nullptr, mnwg = 1, m0 = 2, m1 = S;
    // A local forest (sgp_build_forest): every push stays inside a cluster's
    // tree, so all steps are grouped by component (one launch per sweep, no
    // single-workgroup tail)
    const bool forest = T->cluster_size > 0 && !light && schedule == SGP_SCHED_CONTRACT && S >= 2;
    if (forest) m0 = 0;
    if (!light && schedule == SGP_SCHED_CONTRACT && ((S <= HIST_MAX_STEPS && S >= 4) || forest)) {
        if (!forest) {
            const int hnb = (int)std::min<int64_t>(SCHED_STAT_BLOCKS, grid_for(n, 256));
            int32_t *hpart;
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP6], (size_t)hnb * S + S + 8, &hpart));
            int32_t *hout = hpart + (size_t)hnb * S;
            k_step_hist<<<hnb, 256, 0, st>>>(n, stepv, S, hpart);
            k_step_hist_sum<<<S, 256, 0, st>>>(hnb, S, hpart, hout);
            LAUNCH_CHECK(ctx);
            std::vector<int32_t> cnt(S);
            SGP_TRY(readback(ctx, cnt.data(), hout, S * sizeof(int32_t)));
            std::vector<int64_t> left(S + 1, 0);   // left[k]: vertices of steps >= k
            for (int32_t k = S - 1; k >= 0; k--) left[k] = left[k + 1] + cnt[k];
            while (m0 < S && left[m0] > MID_MAX_VERTICES) m0++;
            const int tdef = std::min(TAIL_DEFAULT_VERTICES, TAIL_MAX_VERTICES);
            while (m1 > m0 && left[m1 - 1] <= tdef) m1--;
        }
        if (m1 - m0 >= 2) {
            int32_t *ja, *jb, *lcnt, *lstart, *wgr, *flag;
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], n + 1, &ja));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], n + 1, &jb));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP5], n + 1, &lcnt));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_B], 2 * n + 2, &lstart));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_A], n + 1, &wgr));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP9], n + 1, &mw));
            SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP6], 2 * SCHED_STAT_BLOCKS + 4, &flag));
            k_mid_init<<<grid_for(n, 256), 256, 0, st>>>(n, stepv, m0, m1, ja);
            LAUNCH_CHECK(ctx);
            // hooking and jumping, four rounds per check (components are small)
            bool converged = false;
            for (int it = 0; it < 64 && !converged; it++) {
                SGP_TRY(fill_i32(ctx, flag, 0, 1));
                for (int r = 0; r < 4; r++) {
                    k_mid_link<<<grid_for(n, 256), 256, 0, st>>>(n, up0, up1, ja, flag);
                    k_mid_jump<<<grid_for(n, 256), 256, 0, st>>>(n, ja);
                }
                LAUNCH_CHECK(ctx);
                int32_t hf;
                SGP_TRY(readback(ctx, &hf, flag, 4));
                // a check whose rounds found no link between two labels: every component is uniform
                if (!hf) converged = true;
            }
            if (converged) {
                SGP_TRY(fill_i32(ctx, lcnt, 0, n));
                k_light_count<<<grid_for(n, 256), 256, 0, st>>>(n, ja, lcnt);
                k_light_vals<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)g->perm.p, ja, lcnt, jb);
                LAUNCH_CHECK(ctx);
                SGP_TRY(scan_exclusive(ctx, jb, lstart, n));
                int32_t total;
                SGP_TRY(readback(ctx, &total, lstart + n, 4));
                const int32_t cap = std::max(forest ? std::max(ctx->light_cap, T->cluster_size) : ctx->light_cap, 1);
                mnwg = std::max((total + cap - 1) / cap, 1);
                k_light_rootwg<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)g->perm.p, ja, lstart, cap, wgr);
                k_light_wg<<<grid_for(n, 256), 256, 0, st>>>(n, ja, wgr, mw);
                LAUNCH_CHECK(ctx);
            } else {
                mw = nullptr;
            }
        }
    }
    if (light) {
        SGP_TRY(order(wgv, nwg));
        int32_t *wptr;
        const int64_t lim = (int64_t)light * nwg;
        SGP_TRY(ensure_t(ctx, M->light_ptr, (size_t)lim + 2, &wptr));
        k_light_ptr<<<grid_for(n + 1, 256), 256, 0, st>>>(n, ka, lim, wptr);
        LAUNCH_CHECK(ctx);
    } else if (mw) {
        SGP_TRY(order(mw, mnwg));
        int32_t *wptr;
        const int64_t lo = (int64_t)m0 * mnwg, hi = (int64_t)m1 * mnwg;
        SGP_TRY(ensure_t(ctx, M->mid_ptr, (size_t)(hi - lo) + 2, &wptr));
        k_mid_ptr<<<grid_for(n + 1, 256), 256, 0, st>>>(n, ka, lo, hi, wptr);
        LAUNCH_CHECK(ctx);
        M->mid_step0 = m0;
        M->mid_steps = m1 - m0;
        M->mid_nwg = mnwg;
    } else {
        SGP_TRY(order(nullptr, 1));
    }
    int32_t *dsp;
    SGP_TRY(ensure_t(ctx, M->step_ptr, (size_t)S + 2, &dsp));
    HIP_TRY(ctx, hipMemcpyAsync(dsp, sptr, (S + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    // steps from tail_step on hold at most ctx->tail_max vertices in all (and
    // never more than fit in LDS, TAIL_MAX_VERTICES)
    M->tail_step = S;
    int tmax = std::min(ctx->tail_max, TAIL_MAX_VERTICES);
    while (!(forest && mw) && M->tail_step > light && n - M->h_step_ptr[M->tail_step - 1] <= tmax) M->tail_step--;
    // up links and in-lists
    int32_t *upq, *icnt, *in_ptr, *in_src;
    SGP_TRY(ensure_t(ctx, M->up, 2 * n + 2, &upq));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_DEG], n + 2, &icnt));
    SGP_TRY(ensure_t(ctx, M->in_ptr, n + 2, &in_ptr));
    SGP_TRY(ensure_t(ctx, M->in_src, 2 * n + 2, &in_src));
    SGP_TRY(fill_i32(ctx, icnt, 0, n));
    k_uplinks<<<grid_for(n, 256), 256, 0, st>>>(n, elim, pos, up0, up1, upq, ka, in_src, icnt);
    LAUNCH_CHECK(ctx);
    int kbits = 1;
    while (((int64_t)1 << kbits) <= n) kbits++;
    SGP_TRY(radix_sort_pairs(ctx, ka, in_src, kb, vb, 2 * n, kbits));
    SGP_TRY(scan_exclusive(ctx, icnt, in_ptr, n));
    // numeric factorisation
    double *Pd, *E0, *E, *C, *F, *Dinv;
    int32_t *status;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], 9 * n + 9, &Pd));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], 9 * n + 9, &E0));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP5], 9 * n + 9, &E));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_SLOTS], 12 * n + 12, &C));
    SGP_TRY(ensure_t(ctx, M->F, 18 * n + 18, &F));
    SGP_TRY(ensure_t(ctx, M->Dinv, 6 * n + 6, &Dinv));
    double *y;
    SGP_TRY(ensure_t(ctx, M->y, 3 * n + 3, &y));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP9], 4, &status));
    SGP_TRY(fill_i32(ctx, status, 0, 3));
    SGP_TRY(fill_f64(ctx, F, 0.0, 18 * n));
    k_tree_blocks<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)T->tptr.p, (const int32_t *)T->tadje.p,
                                                  (const int32_t *)T->pedge.p, (const double4 *)g->wu.p, g_par,
                                                  g_perp, g_med, Pd, E0);
    k_permute9<<<grid_for(9 * n, 256), 256, 0, st>>>(n, elim, E0, E);
    LAUNCH_CHECK(ctx);
    for (int k = 0; k < S; k++) {
        int32_t q0 = M->h_step_ptr[k], q1 = M->h_step_ptr[k + 1];
        if (q1 > q0)
            k_factor_step<<<grid_for(q1 - q0, 128), 128, 0, st>>>(q0, q1, elim, upq, in_ptr, in_src, Pd, E, C, F,
                                                                  9 * n, Dinv, status);
    }
    LAUNCH_CHECK(ctx);
    // the first step's couplings in their (w, u) form (no light steps: with
    // them the first step runs inside the light-subtree sweeps)
    M->n_wu0 = 0;
    M->step0_sorted = false;
    M->mid_lds = M->mid_lds_built = false;
    M->gpar = g_par;
    M->gperp = g_perp;
    M->gmed = g_med;
    if (S > 0 && M->light_steps == 0 && M->h_step_ptr[1] > 0) {
        const int32_t q1 = M->h_step_ptr[1];
        double *w0;
        SGP_TRY(ensure_t(ctx, M->wu0, 8 * (size_t)q1 + 8, &w0));
        k_step0_wu<<<grid_for(q1, 256), 256, 0, st>>>(q1, elim, upq, (const int32_t *)T->pedge.p,
                                                      (const double4 *)g->wu.p, (double4 *)w0);
        // the first step's positions ascend in the internal order (status[1]
        // otherwise), which lets the CG's vector passes sweep that step
        k_step0_sorted<<<grid_for(q1, 256), 256, 0, st>>>(q1, elim_int, status + 1);
        LAUNCH_CHECK(ctx);
        M->n_wu0 = q1;
    }
    // push slots of the forward sweep: in-list position of every (q, k)
    int32_t *tout;
    double *cs;
    SGP_TRY(ensure_t(ctx, M->tout, 2 * n + 2, &tout));
    SGP_TRY(ensure_t(ctx, M->cs, 6 * n + 6, &cs));
    SGP_TRY(fill_i32(ctx, tout, -1, 2 * n));
    k_slot_of<<<grid_for(2 * n, 256), 256, 0, st>>>(in_ptr + n, in_src, tout);
    LAUNCH_CHECK(ctx);
    SGP_TRY(tail_tables(ctx, M, n, in_ptr, in_src, tout));
    SGP_TRY(mid_tables(ctx, M, in_ptr, in_src, upq, status + 2));
    SGP_TRY(readback(ctx, hbuf, status, 12));
    phase_end(ctx, 3);
    if (hbuf[0]) return set_err(ctx, SGP_ENOTSPD, "factor_tree: a pivot block is not positive definite");
    M->step0_sorted = M->n_wu0 > 0 && hbuf[1] == 0;
    M->mid_lds = M->mid_lds_built && hbuf[2] == 0;
    return SGP_OK;
}

// from the diagonal blocks of the edge form (64-row groups of 6 planes)
__global__ void k_jacobi_make(int64_t n, const double *dg, double *dinv, int32_t *status)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *g = dg + (i >> 6) * 384 + (i & 63);
    double D[9] = {g[0], g[64], g[128], g[64], g[192], g[256], g[128], g[256], g[320]};
    double inv[6];
    if (!spd_inverse3(D, inv)) {
        atomicOr(status, 1);
        for (int t = 0; t < 6; t++) inv[t] = 0.0;
    }
    for (int t = 0; t < 6; t++) dinv[6 * i + t] = inv[t];
}

extern "C" int sgp_make_jacobi(sgp_ctx ctx, sgp_bsr A, sgp_prec M)
{
    if (M) M->aug = 0;
    if (!ctx || !A || !M) return set_err(ctx, SGP_EINVAL, "make_jacobi: null handle");
    hipStream_t st = ctx->stream;
    M->kind = PREC_JACOBI;
    M->gen = next_gen();
    M->n = A->n;
    M->steps = 0;
    M->have32 = false;
    SGP_TRY(copy_order(ctx, M->perm, M->inv, A->perm, A->inv, A->n));
    double *dinv;
    int32_t *status;
    SGP_TRY(ensure_t(ctx, M->jdinv, 6 * A->n + 6, &dinv));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP9], 4, &status));
    SGP_TRY(fill_i32(ctx, status, 0, 1));
    if (A->n > 0)
        k_jacobi_make<<<grid_for(A->n, 256), 256, 0, st>>>(A->n, (const double *)A->dg.p, dinv, status);
    LAUNCH_CHECK(ctx);
    int32_t *h = (int32_t *)ctx->pinned;
    SGP_TRY(readback(ctx, h, status, 4));
    if (h[0]) return set_err(ctx, SGP_ENOTSPD, "make_jacobi: a diagonal block is not positive definite");
    return SGP_OK;
}

extern "C" int sgp_prec_info(sgp_prec M, int32_t *steps, int32_t *tail_step, int32_t *light_steps,
                             int32_t *step_sizes)
{
    if (!M) return SGP_EINVAL;
    if (steps) *steps = M->steps;
    if (tail_step) *tail_step = M->tail_step;
    if (light_steps) *light_steps = M->light_steps;
    if (step_sizes && M->kind == PREC_TREE)
        for (int32_t k = 0; k < M->steps; k++) step_sizes[k] = M->h_step_ptr[k + 1] - M->h_step_ptr[k];
    return SGP_OK;
}

extern "C" int sgp_prec_steps(sgp_prec M, int32_t *steps)
{
    if (!M || !steps) return SGP_EINVAL;
    *steps = M->steps;
    return SGP_OK;
}

// ---- the apply without allocation
//
// sgp_prec_apply_noalloc keeps r and z in the internal order in this
// file-scope device array instead of the context's grow-only workspaces.  In
// host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress (at
// context creation) and only that address is ever passed to kernels.
static __device__ __align__(256) double scratch[2 * 3 * NOALLOC_MAX_CELLS];

constexpr int NOALLOC_MAX_DEVICES = 64;
static double *g_scratch_addr[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

int noalloc_scratch_init(sgp_ctx ctx)
{
    const int dev = ctx->device;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return set_err(ctx, SGP_EINVAL, "device %d beyond the %d devices the static scratch serves", dev,
                       NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[dev]) return SGP_OK;
    void *p = nullptr;
    HIP_TRY(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_err(ctx, SGP_EHIP, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_addr[dev] = (double *)p;
    return SGP_OK;
}

extern "C" int sgp_prec_apply_noalloc(sgp_ctx ctx, sgp_prec M, const double *r, double *z)
{
    if (!ctx || !M) return set_err(ctx, SGP_EINVAL, "prec_apply_noalloc: null handle");
    const int64_t n = M->n;
    if (n == 0) return SGP_OK;
    if (!r || !z) return set_err(ctx, SGP_EINVAL, "prec_apply_noalloc: null vector");
    if (n > NOALLOC_MAX_CELLS)
        return set_err(ctx, SGP_EINVAL, "prec_apply_noalloc: %lld cells exceed the static scratch (at most %lld)",
                       (long long)n, (long long)NOALLOC_MAX_CELLS);
    double *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (ctx->device >= 0 && ctx->device < NOALLOC_MAX_DEVICES) base = g_scratch_addr[ctx->device];
    }
    if (!base) return set_err(ctx, SGP_EHIP, "prec_apply_noalloc: static scratch not set up on device %d", ctx->device);
    double *ri = base, *zi = base + 3 * NOALLOC_MAX_CELLS;
    const int32_t *perm = (const int32_t *)M->perm.p;
    SGP_TRY(permute_rows(ctx, perm, r, ri, n, 0));
    SGP_TRY(prec_apply_f64(ctx, M, ri, zi, nullptr));
    return permute_rows(ctx, perm, zi, z, n, 1);
}

extern "C" int sgp_prec_apply(sgp_ctx ctx, sgp_prec M, const double *r, double *z)
{
    if (!ctx || !M) return set_err(ctx, SGP_EINVAL, "prec_apply: null handle");
    const int64_t n = M->n;
    if (n == 0) return SGP_OK;
    double *ri, *zi;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP0], 3 * n + 3, &ri));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP1], 3 * n + 3, &zi));
    const int32_t *perm = (const int32_t *)M->perm.p;
    SGP_TRY(permute_rows(ctx, perm, r, ri, n, 0));
    SGP_TRY(prec_apply_f64(ctx, M, ri, zi, nullptr));
    return permute_rows(ctx, perm, zi, z, n, 1);
}
