// Section 3.1: the maximum spanning forest of the collision graph, rooted.
//
// The paper builds the tree with Prim's algorithm, which is sequential.  On
// the GPU we use Boruvka's algorithm under the same strict total order on
// edges -- heavier first, then smaller edge id -- so the forest is unique and
// equal to Prim's (and Kruskal's) edge for edge:
//   each round, every component finds its best outgoing edge with two integer
//   atomic passes (max of the IEEE bits of w, which order like the values for
//   w > 0; then min edge id among the edges of that weight); components hook
//   along their best edges; the only cycles of the hook graph are mutual pairs,
//   broken toward the smaller component id; pointer jumping finds each hook
//   tree's root, and the merged component takes the smallest representative
//   of its hook tree as its label.  Representatives start as the vertices
//   themselves, so every component is always labelled by its smallest vertex
//   -- the root the forest is oriented from.  Edges inside one component are
//   dropped from the active list after every round.
//
// Rooting: every tree is rooted at its smallest cell id.  An Euler tour of the
// forest (neighbour lists sorted, successor of dart a->b is b->next(a)) is cut
// at the root, list ranking by pointer jumping orders the darts, a dart a->b
// points away from the root iff it comes before its twin b->a, and the depth
// of b is the running sum of +1 (down) / -1 (up) darts along the tour.
#include "sgp_internal.h"

#include <climits>

__global__ void k_bv_reset(int32_t *comp, int64_t n)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) comp[v] = (int32_t)v;
}

__global__ void k_bv_clear_best(unsigned long long *bestw, int32_t *beste, int64_t n)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) {
        bestw[v] = 0ull;
        beste[v] = INT_MAX;
    }
}

// atomicMax of val into slot[key] for the lanes with ok set.  Lanes of a wave
// that share a key are combined first (up to four keys, each led by the lowest
// pending lane); the rest use their own atomic.  Late rounds send most edges
// of a wave to one or two large components, whose slots would otherwise take
// one atomic per edge.  Must be called by every lane of the wave.
SGP_DEV void wave_max_by_key(unsigned long long *slot, int32_t key, unsigned long long val, bool ok)
{
    const int lane = threadIdx.x & 63;
    bool pending = ok;
    for (int it = 0; it < 4; it++) {
        const unsigned long long mask = __ballot(pending);
        if (mask == 0ull) return;
        const int leader = __ffsll((long long)mask) - 1;
        const int32_t k = __shfl(key, leader, 64);
        const bool mine = pending && key == k;
        unsigned long long v = mine ? val : 0ull;
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long w = __shfl_xor(v, o, 64);
            v = v > w ? v : w;
        }
        if (lane == leader && v > slot[k]) atomicMax(&slot[k], v);
        pending = pending && !mine;
    }
    if (pending && val > slot[key]) atomicMax(&slot[key], val);
}

__global__ void k_bv_maxw(const int32_t *act, int64_t na, const int32_t *ei, const int32_t *ej, const double *w,
                          const int32_t *comp, unsigned long long *bestw)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t a = 0, b = 0;
    unsigned long long wb = 0ull;
    bool ok = false;
    if (k < na) {
        const int32_t e = act[k];
        a = comp[ei[e]];
        b = comp[ej[e]];
        ok = a != b;
        wb = (unsigned long long)__double_as_longlong(w[e]);
    }
    wave_max_by_key(bestw, a, wb, ok);
    wave_max_by_key(bestw, b, wb, ok);
}

__global__ void k_bv_mine(const int32_t *act, int64_t na, const int32_t *ei, const int32_t *ej, const double *w,
                          const int32_t *comp, const unsigned long long *bestw, int32_t *beste)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= na) return;
    int32_t e = act[k];
    int32_t a = comp[ei[e]], b = comp[ej[e]];
    if (a == b) return;
    unsigned long long wb = (unsigned long long)__double_as_longlong(w[e]);
    if (wb == bestw[a] && e < beste[a]) atomicMin(&beste[a], e);
    if (wb == bestw[b] && e < beste[b]) atomicMin(&beste[b], e);
}

// The first round's best edges, pulled by every vertex from its own edge list
// (every vertex is its own component then): the same maximum of (w, then
// smaller id) as the two atomic passes, without their atomics.
// With a partition (cl != null), entries to another cluster are not edges.
__global__ void k_bv_first(int64_t n, const int32_t *rowptr, const int32_t *ent_edge, const int32_t *col,
                           const int32_t *cl, const double *w, unsigned long long *bestw, int32_t *beste)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    unsigned long long bw = 0ull;
    int32_t be = INT_MAX;
    const int32_t cv = cl ? cl[v] : 0;
    for (int32_t p = rowptr[v]; p < rowptr[v + 1]; p++) {
        if (cl && cl[col[p]] != cv) continue;
        const int32_t e = ent_edge[p];
        const unsigned long long wb = (unsigned long long)__double_as_longlong(w[e]);
        if (wb > bw || (wb == bw && e < be)) {
            bw = wb;
            be = e;
        }
    }
    bestw[v] = bw;
    beste[v] = be;
}

__global__ void k_bv_hook(const int32_t *ei, const int32_t *ej, int64_t n, const int32_t *comp,
                          const int32_t *beste, int32_t *nxt, int32_t *is_tree, int32_t *flag)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    if (comp[c] != c) return;   // representatives only
    int32_t e = beste[c];
    if (e == INT_MAX) {
        nxt[c] = (int32_t)c;
        return;
    }
    int32_t a = comp[ei[e]], b = comp[ej[e]];
    int32_t o = (a == c) ? b : a;
    if (beste[o] == e && c < o) {
        nxt[c] = (int32_t)c;   // root of a mutual pair
        return;
    }
    nxt[c] = o;
    is_tree[e] = 1;
    *flag = 1;
}

__global__ void k_bv_jump(int64_t n, const int32_t *comp, const int32_t *nxt_in, int32_t *nxt_out, int32_t *flag)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || comp[c] != c) return;
    int32_t p = nxt_in[c];
    int32_t pp = nxt_in[p];
    nxt_out[c] = pp;
    if (pp != p) *flag = 1;
}

// smallest representative of every hook tree, at the tree's root
__global__ void k_bv_minrep(int64_t n, const int32_t *comp, const int32_t *nxt, int32_t *mr)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || comp[c] != c) return;
    int32_t root = nxt[c];
    if ((int32_t)c < mr[root]) atomicMin(&mr[root], (int32_t)c);
}

__global__ void k_bv_relabel(int64_t n, int32_t *comp, const int32_t *nxt, const int32_t *mr)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    comp[v] = mr[nxt[comp[v]]];
}

// active-edge compaction: keep the edges that still join two components
__global__ void k_bv_live(const int32_t *act, int64_t na, const int32_t *ei, const int32_t *ej, const int32_t *comp,
                          int32_t *flag)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= na) return;
    int32_t e = act[k];
    flag[k] = comp[ei[e]] != comp[ej[e]] ? 1 : 0;
}

__global__ void k_bv_pack(const int32_t *act, int64_t na, const int32_t *flag, const int32_t *off, int32_t *out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < na && flag[k]) out[off[k]] = act[k];
}

// edges inside one cluster
__global__ void k_intra(const int32_t *ei, const int32_t *ej, int64_t m, const int32_t *cl, int32_t *flag)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) flag[e] = cl[ei[e]] == cl[ej[e]] ? 1 : 0;
}

__global__ void k_compact_flags(const int32_t *flag, const int32_t *off, int64_t m, int32_t *out)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m && flag[e]) out[off[e]] = (int32_t)e;
}

// ---------------------------------------------------------------- rooting

__global__ void k_tdeg(const int32_t *tree_edge, int64_t nt, const int32_t *ei, const int32_t *ej, int32_t *deg)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    int32_t e = tree_edge[k];
    atomicAdd(&deg[ei[e]], 1);
    atomicAdd(&deg[ej[e]], 1);
}

__global__ void k_tfill(const int32_t *tree_edge, int64_t nt, const int32_t *ei, const int32_t *ej,
                        const int32_t *tptr, int32_t *cur, int32_t *adj, int32_t *adje)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    int32_t e = tree_edge[k];
    int32_t a = ei[e], b = ej[e];
    int32_t pa = tptr[a] + atomicAdd(&cur[a], 1);
    adj[pa] = b;
    adje[pa] = e;
    int32_t pb = tptr[b] + atomicAdd(&cur[b], 1);
    adj[pb] = a;
    adje[pb] = e;
}

// sort each incidence row by edge id (rows are short); record dart owners.
// The cyclic order of a row is all an Euler tour needs; edge-id order also
// makes the sum of a vertex's tree blocks follow ascending edge id.
__global__ void k_tsort(int64_t n, const int32_t *tptr, int32_t *adj, int32_t *adje, int32_t *from)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t b = tptr[v], e = tptr[v + 1];
    for (int32_t p = b + 1; p < e; p++) {
        int32_t x = adj[p], xe = adje[p];
        int32_t q = p;
        while (q > b && adje[q - 1] > xe) {
            adj[q] = adj[q - 1];
            adje[q] = adje[q - 1];
            q--;
        }
        adj[q] = x;
        adje[q] = xe;
    }
    for (int32_t p = b; p < e; p++) from[p] = (int32_t)v;
}

// twin, Euler successor, cut at the root of each tree
// sr[k] = (successor, rank so far) of dart k, one 8-byte word: a jump reads
// both with one gather
__global__ void k_tour(int64_t nd, const int32_t *tptr, const int32_t *adj, const int32_t *adje,
                       const int32_t *comp, int32_t *twin, int2 *sr)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nd) return;
    int32_t b = adj[k], ek = adje[k];
    int32_t lo = tptr[b], hi = tptr[b + 1];
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (adje[mid] < ek) lo = mid + 1; else hi = mid;
    }
    twin[k] = lo;
    int32_t nx = (lo + 1 < tptr[b + 1]) ? lo + 1 : tptr[b];
    bool is_root = comp[b] == b;   // components are labelled by their smallest vertex
    if (is_root && nx == tptr[b]) nx = -1;   // tour of b's tree ends when it returns to b the last time
    sr[k] = make_int2(nx, nx < 0 ? 0 : 1);
}

__global__ void k_rank_jump(int64_t nd, const int2 *sr_in, int2 *sr_out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nd) return;
    const int2 a = sr_in[k];
    if (a.x < 0) {
        sr_out[k] = a;
        return;
    }
    const int2 b = sr_in[a.x];
    sr_out[k] = make_int2(b.x, a.y + b.y);
}

__global__ void k_rank_unpack(int64_t nd, const int2 *sr, int32_t *rank)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nd) rank[k] = sr[k].y;
}

// component tour lengths at the root's index: 2 (size - 1) = rank(first dart) + 1
__global__ void k_tour_len(int64_t n, const int32_t *tptr, const int32_t *comp, const int32_t *rank, int32_t *len)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    bool is_root = comp[v] == v;
    len[v] = (is_root && tptr[v + 1] > tptr[v]) ? rank[tptr[v]] + 1 : 0;
}

__global__ void k_orient(int64_t nd, const int32_t *adj, const int32_t *adje, const int32_t *from,
                         const int32_t *twin, const int32_t *rank, const int32_t *tptr, const int32_t *comp,
                         const int32_t *base, int32_t *parent, int32_t *pedge,
                         int32_t *wval, int32_t *dpos, int32_t *bad)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nd) return;
    int32_t a = from[k], b = adj[k];
    bool down = rank[k] > rank[twin[k]];
    int32_t r = comp[a];
    int64_t g = (int64_t)base[r] + (rank[tptr[r]] - rank[k]);
    if (g < 0 || g >= nd) {   // only a broken tour could get here
        atomicOr(bad, 1);
        return;
    }
    wval[g] = down ? 1 : -1;
    if (down) {
        parent[b] = a;
        pedge[b] = adje[k];
        dpos[b] = (int32_t)g;
    }
}

__global__ __launch_bounds__(256) void k_depth(int64_t n, const int32_t *parent, const int32_t *dpos,
                                               const int32_t *excl, const int32_t *wval, int32_t *depth,
                                               int32_t *maxd)
{
    __shared__ int32_t sd[4];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t dv = 0;   // lanes past n take part in the block maximum with 0
    if (v < n && parent[v] >= 0) {
        const int32_t g = dpos[v];
        dv = excl[g] + wval[g];   // inclusive running sum of the tour up to v's entry
    }
    int32_t d = dv;
    // the block's largest depth, then one atomic per block that can raise it
    // (an atomic per vertex on one address would serialise); the current
    // maximum is read before any store, and the depth is stored last
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t d2 = __shfl_xor(d, o, 64);
        d = d2 > d ? d2 : d;
    }
    if ((threadIdx.x & 63) == 0) sd[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t bm = sd[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) bm = sd[w] > bm ? sd[w] : bm;
        if (bm > *(volatile int32_t *)maxd) atomicMax(maxd, bm);
    }
    if (v < n) depth[v] = dv;
}

__global__ void k_count_roots(int64_t n, const int32_t *parent, int32_t *cnt)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && parent[v] < 0) atomicAdd(cnt, 1);
}

// The maximum spanning forest of the graph, or with a partition (cl: the
// cluster of every cell) of the graph without its edges between clusters.
static int build_forest_impl(sgp_ctx ctx, sgp_graph g, sgp_tree T, const int32_t *cl)
{
    hipStream_t st = ctx->stream;
    const int64_t n = g->n, m = g->m;
    T->n = n;
    int32_t *comp, *parent, *pedge, *depth, *te;
    SGP_TRY(ensure_t(ctx, T->comp, n + 1, &comp));
    SGP_TRY(ensure_t(ctx, T->parent, n + 1, &parent));
    SGP_TRY(ensure_t(ctx, T->pedge, n + 1, &pedge));
    SGP_TRY(ensure_t(ctx, T->depth, n + 1, &depth));
    SGP_TRY(ensure_t(ctx, T->tree_edge, n + 1, &te));
    if (n == 0) {
        T->nt = 0;
        T->n_roots = 0;
        T->max_depth = 0;
        return SGP_OK;
    }
    const int32_t *ei = (const int32_t *)g->ei.p, *ej = (const int32_t *)g->ej.p;
    const double *wonly = (const double *)g->w.p;
    // ---- Boruvka
    unsigned long long *bestw;
    int32_t *beste, *nxt, *nxt2, *is_tree, *flag;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP0], n + 1, &bestw));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP1], n + 1, &beste));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP2], n + 1, &nxt));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], n + 1, &nxt2));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], m + 2, &is_tree));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP5], 8, &flag));
    int32_t *hflag = (int32_t *)ctx->pinned;
    int32_t *act, *act2, *lflag, *loff, *mr;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_A], m + 2, &act));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_B], m + 2, &act2));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_A], m + 2, &lflag));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_B], m + 2, &loff));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_DEG], n + 2, &mr));
    k_bv_reset<<<grid_for(n, 256), 256, 0, st>>>(comp, n);
    SGP_TRY(fill_i32(ctx, is_tree, 0, m + 1));
    int64_t na = m;
    if (cl) {
        // the active edges: those inside a cluster
        if (m > 0) {
            k_intra<<<grid_for(m, 256), 256, 0, st>>>(ei, ej, m, cl, lflag);
            LAUNCH_CHECK(ctx);
        }
        SGP_TRY(scan_exclusive(ctx, lflag, loff, m));
        if (m > 0) k_compact_flags<<<grid_for(m, 256), 256, 0, st>>>(lflag, loff, m, act);
        LAUNCH_CHECK(ctx);
        int32_t hn;
        SGP_TRY(readback(ctx, &hn, loff + m, 4));
        na = hn;
    } else {
        SGP_TRY(iota_i32(ctx, act, m));
    }
    for (int round = 0; round < 64 && na > 0; round++) {
        if (round == 0) {
            k_bv_first<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)g->rowptr.p,
                                                        (const int32_t *)g->ent_edge.p, (const int32_t *)g->col.p, cl,
                                                        wonly, bestw, beste);
        } else {
            k_bv_clear_best<<<grid_for(n, 256), 256, 0, st>>>(bestw, beste, n);
            k_bv_maxw<<<grid_for(na, 256), 256, 0, st>>>(act, na, ei, ej, wonly, comp, bestw);
            k_bv_mine<<<grid_for(na, 256), 256, 0, st>>>(act, na, ei, ej, wonly, comp, bestw, beste);
        }
        SGP_TRY(fill_i32(ctx, flag, 0, 1));
        k_bv_hook<<<grid_for(n, 256), 256, 0, st>>>(ei, ej, n, comp, beste, nxt, is_tree, flag);
        LAUNCH_CHECK(ctx);
        // pointer jumping: three pairs of jumps before the first check (hook
        // chains are short: one check usually ends it), then two per check;
        // jumps past convergence are no-ops
        for (int j = 0; j < 64; j++) {
            for (int r = 0; r < (j == 0 ? 3 : 1); r++) {
                if (r == (j == 0 ? 2 : 0)) SGP_TRY(fill_i32(ctx, flag, 0, 1));   // the last pair is checked
                k_bv_jump<<<grid_for(n, 256), 256, 0, st>>>(n, comp, nxt, nxt2, flag + 1);
                k_bv_jump<<<grid_for(n, 256), 256, 0, st>>>(n, comp, nxt2, nxt, flag);
            }
            LAUNCH_CHECK(ctx);
            SGP_TRY(readback(ctx, hflag, flag, 4));
            if (!hflag[0]) break;
        }
        SGP_TRY(fill_i32(ctx, mr, INT_MAX, n));
        k_bv_minrep<<<grid_for(n, 256), 256, 0, st>>>(n, comp, nxt, mr);
        k_bv_relabel<<<grid_for(n, 256), 256, 0, st>>>(n, comp, nxt, mr);
        k_bv_live<<<grid_for(na, 256), 256, 0, st>>>(act, na, ei, ej, comp, lflag);
        SGP_TRY(scan_exclusive(ctx, lflag, loff, na));
        k_bv_pack<<<grid_for(na, 256), 256, 0, st>>>(act, na, lflag, loff, act2);
        LAUNCH_CHECK(ctx);
        int32_t hn;
        SGP_TRY(readback(ctx, &hn, loff + na, 4));
        std::swap(act, act2);
        na = hn;
    }
    // tree edges ascending
    int32_t *toff;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP6], m + 2, &toff));
    SGP_TRY(scan_exclusive(ctx, is_tree, toff, m));
    if (m > 0) k_compact_flags<<<grid_for(m, 256), 256, 0, st>>>(is_tree, toff, m, te);
    int32_t hnt;
    SGP_TRY(readback(ctx, &hnt, toff + m, 4));
    const int64_t nt = hnt;
    T->nt = nt;
    // ---- rooting
    int32_t *tdeg = nxt, *tptr, *cur = beste;
    SGP_TRY(ensure_t(ctx, T->tptr, n + 2, &tptr));
    SGP_TRY(fill_i32(ctx, tdeg, 0, n));
    SGP_TRY(fill_i32(ctx, cur, 0, n));
    SGP_TRY(fill_i32(ctx, parent, -1, n));
    SGP_TRY(fill_i32(ctx, pedge, -1, n));
    if (nt > 0) k_tdeg<<<grid_for(nt, 256), 256, 0, st>>>(te, nt, ei, ej, tdeg);
    SGP_TRY(scan_exclusive(ctx, tdeg, tptr, n));
    const int64_t nd = 2 * nt;
    int32_t *adj, *adje, *from, *twin, *slots, *rank;
    SGP_TRY(ensure_t(ctx, T->tadj, nd + 1, &adj));
    SGP_TRY(ensure_t(ctx, T->tadje, nd + 1, &adje));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_A], nd + 1, &from));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_B], nd + 1, &twin));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_SLOTS], 6 * (nd + 1), &slots));
    int2 *sra = (int2 *)slots, *srb = sra + (nd + 1);
    rank = slots + 4 * (nd + 1);
    int32_t *hmax = (int32_t *)ctx->pinned;
    if (nt > 0) {
        k_tfill<<<grid_for(nt, 256), 256, 0, st>>>(te, nt, ei, ej, tptr, cur, adj, adje);
        k_tsort<<<grid_for(n, 256), 256, 0, st>>>(n, tptr, adj, adje, from);
        k_tour<<<grid_for(nd, 256), 256, 0, st>>>(nd, tptr, adj, adje, comp, twin, sra);
        LAUNCH_CHECK(ctx);
        for (int64_t span = 1; span < nd; span *= 2) {
            k_rank_jump<<<grid_for(nd, 256), 256, 0, st>>>(nd, sra, srb);
            std::swap(sra, srb);
        }
        k_rank_unpack<<<grid_for(nd, 256), 256, 0, st>>>(nd, sra, rank);
        LAUNCH_CHECK(ctx);
        // buffer reuse: cur (done) holds the tour lengths, then the entry
        // positions; tdeg (scanned into tptr already) holds the tour bases
        int32_t *len = cur, *base = tdeg;
        int32_t *wv, *wex, *dpos;
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP8], nd + 1, &wv));
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP9], nd + 2, &wex));
        dpos = cur;     // the lengths are consumed by the scan before k_orient writes
        k_tour_len<<<grid_for(n, 256), 256, 0, st>>>(n, tptr, comp, rank, len);
        SGP_TRY(scan_exclusive(ctx, len, base, n));
        SGP_TRY(fill_i32(ctx, flag, 0, 3));
        SGP_TRY(fill_i32(ctx, wv, 0, nd));
        k_orient<<<grid_for(nd, 256), 256, 0, st>>>(nd, adj, adje, from, twin, rank, tptr, comp, base,
                                                   parent, pedge, wv, dpos, flag + 2);
        SGP_TRY(scan_exclusive(ctx, wv, wex, nd));
        k_depth<<<grid_for(n, 256), 256, 0, st>>>(n, parent, dpos, wex, wv, depth, flag);
        k_count_roots<<<grid_for(n, 256), 256, 0, st>>>(n, parent, flag + 1);
        LAUNCH_CHECK(ctx);
        SGP_TRY(readback(ctx, hmax, flag, 12));
        if (hmax[2]) return set_err(ctx, SGP_EINVAL, "build_tree: inconsistent Euler tour");
        T->max_depth = hmax[0];
        T->n_roots = hmax[1];
    } else {
        SGP_TRY(fill_i32(ctx, depth, 0, n));
        T->max_depth = 0;
        T->n_roots = n;
    }
    return SGP_OK;
}

extern "C" int sgp_build_tree(sgp_ctx ctx, sgp_graph g, sgp_tree T)
{
    if (!ctx || !g || !T) return set_err(ctx, SGP_EINVAL, "build_tree: null handle");
    phase_begin(ctx, 2);
    T->cluster_size = 0;
    T->n_clusters = 0;
    SGP_TRY(build_forest_impl(ctx, g, T, nullptr));
    phase_end(ctx, 2);
    return SGP_OK;
}

extern "C" int sgp_build_forest(sgp_ctx ctx, sgp_graph g, const double *pos, const double *radius,
                                int32_t cluster_size, sgp_tree T)
{
    if (!ctx || !g || !T) return set_err(ctx, SGP_EINVAL, "build_forest: null handle");
    if (cluster_size < 1) return set_err(ctx, SGP_EINVAL, "build_forest: cluster_size must be positive");
    if (g->n > 0 && (!pos || !radius)) return set_err(ctx, SGP_EINVAL, "build_forest: null positions");
    phase_begin(ctx, 2);
    int32_t *cl;
    SGP_TRY(ensure_t(ctx, T->cluster, g->n + 1, &cl));
    int64_t nc = 0;
    SGP_TRY(forest_partition(ctx, g, pos, radius, cluster_size, cl, &nc));
    T->cluster_size = cluster_size;
    T->n_clusters = nc;
    SGP_TRY(build_forest_impl(ctx, g, T, cl));
    phase_end(ctx, 2);
    return SGP_OK;
}

extern "C" int sgp_tree_clusters(sgp_ctx ctx, sgp_tree T, int32_t *cluster, int64_t *n_clusters)
{
    if (!ctx || !T) return set_err(ctx, SGP_EINVAL, "tree_clusters: null handle");
    if (n_clusters) *n_clusters = T->n_clusters;
    if (cluster && T->cluster_size > 0 && T->n > 0)
        HIP_TRY(ctx, hipMemcpyAsync(cluster, T->cluster.p, T->n * 4, hipMemcpyDeviceToDevice, ctx->stream));
    return SGP_OK;
}

extern "C" int sgp_tree_size(sgp_tree T, int64_t *n_tree_edges, int64_t *n_roots, int32_t *max_depth)
{
    if (!T) return SGP_EINVAL;
    if (n_tree_edges) *n_tree_edges = T->nt;
    if (n_roots) *n_roots = T->n_roots;
    if (max_depth) *max_depth = T->max_depth;
    return SGP_OK;
}

extern "C" int sgp_tree_export(sgp_ctx ctx, sgp_tree T, int32_t *tree_edge, int32_t *parent, int32_t *depth)
{
    if (!ctx || !T) return set_err(ctx, SGP_EINVAL, "tree_export: null handle");
    hipStream_t st = ctx->stream;
    if (tree_edge && T->nt > 0)
        HIP_TRY(ctx, hipMemcpyAsync(tree_edge, T->tree_edge.p, T->nt * 4, hipMemcpyDeviceToDevice, st));
    if (parent && T->n > 0) HIP_TRY(ctx, hipMemcpyAsync(parent, T->parent.p, T->n * 4, hipMemcpyDeviceToDevice, st));
    if (depth && T->n > 0) HIP_TRY(ctx, hipMemcpyAsync(depth, T->depth.p, T->n * 4, hipMemcpyDeviceToDevice, st));
    return SGP_OK;
}
