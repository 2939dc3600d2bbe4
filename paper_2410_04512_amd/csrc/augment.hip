// Section 3.1, Vaidya's second preconditioner: the maximum spanning tree with
// contacts added back between its pieces, and the nested solve the paper
// uses for it (Sections 3 and 5): flexible CG on Gamma whose preconditioner is
// an inner CG on the augmented tree's block Laplacian P', itself
// preconditioned by the tree (the factor of sgp_factor_tree), run to a
// relative residual of inner_rtol (0.1 in the paper's experiments).
//
// Pieces: walking the forest children first, a vertex weighs 1 plus the
// weights of its children that were not cut off; a vertex of weight >= s
// (s = ceil(n / parts)) is cut off from its parent and heads a piece.  On
// the GPU the walk is one launch per depth level (children are one level
// deeper), and every vertex finds its piece's head by pointer jumping along
// the uncut parent links.  Added contacts: for every pair of pieces joined by
// a contact, the heaviest (ties: the smaller edge id), by one sort of the
// crossing contacts by their pair and a scan of each pair's run.
//
// The outer and inner iterations are driven from the host: each reads back
// its few dot products (fixed-shape two-stage reductions, so the results are
// bitwise reproducible).  The paper found no iteration gain for this variant
// and did not make it fast; it is built here to measure that on the GPU.
#include "sgp_internal.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

// ---------------------------------------------------------------- pieces

__global__ void k_depth_keys(int64_t n, const int32_t *depth, uint32_t *key, int32_t *val)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    key[v] = (uint32_t)depth[v];
    val[v] = (int32_t)v;
}

// first position of every depth in the sorted keys
__global__ void k_level_bounds(int64_t n, const uint32_t *key, int32_t L, int32_t *lptr)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q > n) return;
    const int32_t lo = q == 0 ? -1 : (int32_t)key[q - 1];
    const int32_t hi = q == n ? L : (int32_t)key[q];
    for (int32_t d = lo + 1; d <= hi; d++) lptr[d] = (int32_t)q;
}

// weights of one depth level: 1 + the weights (< s) of the children
__global__ void k_aug_weight(int32_t lo, int32_t hi, const int32_t *sorted, const int32_t *tptr, const int32_t *tadj,
                             const int32_t *parent, int32_t s, int32_t *w)
{
    const int32_t i = lo + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= hi) return;
    const int32_t v = sorted[i];
    int32_t wv = 1;
    for (int32_t k = tptr[v]; k < tptr[v + 1]; k++) {
        const int32_t j = tadj[k];
        if (parent[j] == v) {
            const int32_t wc = w[j];
            if (wc < s) wv += wc;
        }
    }
    w[v] = wv;
}

__global__ void k_aug_link(int64_t n, const int32_t *parent, const int32_t *w, int32_t s, int32_t *jr)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t p = parent[v];
    jr[v] = (p >= 0 && w[v] < s) ? p : (int32_t)v;
}

__global__ void k_aug_jump(int64_t n, const int32_t *a, int32_t *b)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) b[v] = a[a[v]];
}

__global__ void k_aug_heads(int64_t n, const int32_t *piece, int32_t *flag)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) flag[v] = piece[v] == (int32_t)v ? 1 : 0;
}

// ---------------------------------------------------------------- added contacts

__global__ void k_aug_cross(int64_t m, const int32_t *ei, const int32_t *ej, const int32_t *piece, int32_t *flag)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) flag[e] = piece[ei[e]] != piece[ej[e]] ? 1 : 0;
}

// the crossing contacts' pair keys: lo * np + hi over the pieces' dense ids
__global__ void k_aug_pairkeys(int64_t nc, const int32_t *cross, const int32_t *ei, const int32_t *ej,
                               const int32_t *piece, const int32_t *did, int64_t np, uint32_t *key, int32_t *val)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    const int32_t e = cross[k];
    const int64_t a = did[piece[ei[e]]], b = did[piece[ej[e]]];
    key[k] = (uint32_t)((a < b ? a : b) * np + (a < b ? b : a));
    val[k] = e;
}

// at the start of every pair's run: its heaviest contact (ties: smaller id)
__global__ void k_aug_best(int64_t nc, const uint32_t *key, const int32_t *val, const double *w,
                           const int32_t *is_tree, int32_t *added)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nc || (p > 0 && key[p - 1] == key[p])) return;
    int32_t be = val[p];
    double bw = w[be];
    for (int64_t q = p + 1; q < nc && key[q] == key[p]; q++) {
        const int32_t e = val[q];
        const double we = w[e];
        if (we > bw || (we == bw && e < be)) {
            bw = we;
            be = e;
        }
    }
    if (!is_tree[be]) added[be] = 1;
}

__global__ void k_aug_treeflags(int64_t nt, const int32_t *tree_edge, int32_t *is_tree)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nt) is_tree[tree_edge[k]] = 1;
}

__global__ void k_aug_compact(int64_t m, const int32_t *flag, const int32_t *off, int32_t *out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m && flag[e]) out[off[e]] = (int32_t)e;
}

// incidence rows of the added contacts (caller numbering), sorted by edge id
__global__ void k_aug_deg(int64_t na, const int32_t *list, const int32_t *ei, const int32_t *ej, int32_t *deg)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= na) return;
    const int32_t e = list[k];
    atomicAdd(&deg[ei[e]], 1);
    atomicAdd(&deg[ej[e]], 1);
}

__global__ void k_aug_fill(int64_t na, const int32_t *list, const int32_t *ei, const int32_t *ej, const int32_t *ptr,
                           int32_t *cur, int32_t *adj, int32_t *adje)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= na) return;
    const int32_t e = list[k], a = ei[e], b = ej[e];
    const int32_t pa = ptr[a] + atomicAdd(&cur[a], 1);
    adj[pa] = b;
    adje[pa] = e;
    const int32_t pb = ptr[b] + atomicAdd(&cur[b], 1);
    adj[pb] = a;
    adje[pb] = e;
}

__global__ void k_aug_rowsort(int64_t n, const int32_t *ptr, int32_t *adj, int32_t *adje)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t b = ptr[v], e = ptr[v + 1];
    for (int32_t p = b + 1; p < e; p++) {
        const int32_t x = adj[p], xe = adje[p];
        int32_t q = p;
        while (q > b && adje[q - 1] > xe) {
            adj[q] = adj[q - 1];
            adje[q] = adje[q - 1];
            q--;
        }
        adj[q] = x;
        adje[q] = xe;
    }
}

// (w, u) of every incidence entry, and the neighbour in the internal order
__global__ void k_aug_entries(int64_t ne, const int32_t *adj, const int32_t *adje, const double4 *wu,
                              const int32_t *inv, int32_t *adj_int, double4 *ewu)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ne) return;
    adj_int[k] = inv[adj[k]];
    ewu[k] = wu[adje[k]];
}

// ---------------------------------------------------------------- P' x

// y_i = g_med x_i + sum over i's tree contacts, then its added contacts (each
// ascending edge id) of W_e (x_i - x_j), W_e d = w (g_perp d + (g_par - g_perp)
// (u.d) u).  Rows in the caller numbering, vectors in the internal order.
__global__ void k_aug_mv(int64_t n, const int32_t *inv, const int32_t *tptr, const int32_t *tadj,
                         const double4 *twu, const int32_t *aptr, const int32_t *aadj, const double4 *awu,
                         double gpar, double gperp, double gmed, const double *x, double *y)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t i = inv[v];
    const double x0 = x[3 * i], x1 = x[3 * i + 1], x2 = x[3 * i + 2];
    double y0 = gmed * x0, y1 = gmed * x1, y2 = gmed * x2;
    for (int pass = 0; pass < 2; pass++) {
        const int32_t *ptr = pass ? aptr : tptr, *adj = pass ? aadj : tadj;
        const double4 *ewu = pass ? awu : twu;
        for (int32_t k = ptr[v]; k < ptr[v + 1]; k++) {
            const int64_t j = adj[k];
            const double4 e = ewu[k];
            const double d0 = x0 - x[3 * j], d1 = x1 - x[3 * j + 1], d2 = x2 - x[3 * j + 2];
            const double c = (gpar - gperp) * ((e.y * d0 + e.z * d1) + e.w * d2);
            y0 = y0 + e.x * (gperp * d0 + c * e.y);
            y1 = y1 + e.x * (gperp * d1 + c * e.z);
            y2 = y2 + e.x * (gperp * d2 + c * e.w);
        }
    }
    y[3 * i] = y0;
    y[3 * i + 1] = y1;
    y[3 * i + 2] = y2;
}

// ---------------------------------------------------------------- vector work

// partials of a.b and c.d (c may be null): fixed grid, fixed order
__global__ __launch_bounds__(256) void k_aug_dots(int64_t len, const double *a, const double *b, const double *c,
                                                  const double *d, double *part)
{
    __shared__ double sh[256];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256) {
        s0 = s0 + a[t] * b[t];
        if (c) s1 = s1 + c[t] * d[t];
    }
    const double r0 = block_sum_256(s0, sh);
    const double r1 = block_sum_256(s1, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = r0;
        part[gridDim.x + blockIdx.x] = r1;
    }
}

__global__ __launch_bounds__(256) void k_aug_dots_fin(int nb, const double *part, double *out)
{
    __shared__ double sh[256];
    const double r0 = sum_partials(part, nb, sh);
    const double r1 = sum_partials(part + nb, nb, sh);
    if (threadIdx.x == 0) {
        out[0] = r0;
        out[1] = r1;
    }
}

// x += alpha p; r -= alpha q
__global__ void k_aug_axpy2(int64_t len, double alpha, const double *p, const double *q, double *x, double *r)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= len) return;
    x[t] = x[t] + alpha * p[t];
    r[t] = r[t] - alpha * q[t];
}

// p = z + beta p
__global__ void k_aug_xpby(int64_t len, const double *z, double beta, double *p)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) p[t] = z[t] + beta * p[t];
}

__global__ void k_aug_sub(int64_t len, const double *a, const double *b, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) out[t] = a[t] - b[t];
}

// ---------------------------------------------------------------- construction

extern "C" int sgp_factor_augmented(sgp_ctx ctx, sgp_graph g, sgp_tree T, double g_par, double g_perp, double g_med,
                                    int32_t schedule, int32_t parts, double inner_rtol, sgp_prec M)
{
    if (!ctx || !g || !T || !M) return set_err(ctx, SGP_EINVAL, "factor_augmented: null handle");
    if (!(inner_rtol > 0.0) || !(inner_rtol < 1.0))
        return set_err(ctx, SGP_EINVAL, "factor_augmented: inner_rtol must lie in (0, 1)");
    if (T->cluster_size > 0) return set_err(ctx, SGP_EINVAL, "factor_augmented: needs a spanning tree, not a forest");
    SGP_TRY(sgp_factor_tree(ctx, g, T, g_par, g_perp, g_med, schedule, M));
    M->aug = 0;
    const int64_t n = g->n, m = g->m;
    if (parts <= 0) parts = std::max<int32_t>(1, (int32_t)ceil(pow((double)n, 0.25)));
    const int32_t s = (int32_t)std::max<int64_t>(1, (n + parts - 1) / parts);
    hipStream_t st = ctx->stream;
    M->inner_rtol = inner_rtol;
    M->aug_parts = parts;
    int32_t *piece, *aptr, *aadj_int;
    SGP_TRY(ensure_t(ctx, M->aug_piece, n + 1, &piece));
    SGP_TRY(ensure_t(ctx, M->aug_ptr, n + 2, &aptr));
    M->aug_pieces = 0;
    M->aug_added = 0;
    if (n == 0) {
        M->aug = 1;
        return SGP_OK;
    }
    // ---- pieces: weights level by level, children first
    const int32_t L = T->max_depth + 1;
    uint32_t *ka, *kb;
    int32_t *va, *vb, *lptr, *w, *jr;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_A], n, &ka));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_B], n, &kb));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_A], n, &va));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_B], n, &vb));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP0], (size_t)L + 2, &lptr));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP1], n + 1, &w));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP2], n + 1, &jr));
    const int32_t *parent = (const int32_t *)T->parent.p;
    const int32_t *tptr = (const int32_t *)T->tptr.p, *tadj = (const int32_t *)T->tadj.p;
    k_depth_keys<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)T->depth.p, ka, va);
    LAUNCH_CHECK(ctx);
    int dbits = 1;
    while (((int64_t)1 << dbits) < L) dbits++;
    SGP_TRY(radix_sort_pairs(ctx, ka, va, kb, vb, n, dbits));
    k_level_bounds<<<grid_for(n + 1, 256), 256, 0, st>>>(n, ka, L, lptr);
    LAUNCH_CHECK(ctx);
    std::vector<int32_t> hl(L + 1);
    SGP_TRY(readback(ctx, hl.data(), lptr, (L + 1) * sizeof(int32_t)));
    for (int32_t d = L - 1; d >= 0; d--) {
        const int32_t lo = hl[d], hi = hl[d + 1];
        if (hi > lo) k_aug_weight<<<grid_for(hi - lo, 256), 256, 0, st>>>(lo, hi, va, tptr, tadj, parent, s, w);
    }
    LAUNCH_CHECK(ctx);
    int32_t *ja = jr, *jb = piece;
    k_aug_link<<<grid_for(n, 256), 256, 0, st>>>(n, parent, w, s, ja);
    for (int32_t span = 1; span < L; span *= 2) {
        k_aug_jump<<<grid_for(n, 256), 256, 0, st>>>(n, ja, jb);
        std::swap(ja, jb);
    }
    if (ja != piece) HIP_TRY(ctx, hipMemcpyAsync(piece, ja, n * 4, hipMemcpyDeviceToDevice, st));
    LAUNCH_CHECK(ctx);
    // dense ids of the pieces' heads
    int32_t *hflag, *did;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], n + 1, &hflag));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], n + 2, &did));
    k_aug_heads<<<grid_for(n, 256), 256, 0, st>>>(n, piece, hflag);
    LAUNCH_CHECK(ctx);
    SGP_TRY(scan_exclusive(ctx, hflag, did, n));
    int32_t np32;
    SGP_TRY(readback(ctx, &np32, did + n, 4));
    const int64_t np = np32;
    M->aug_pieces = np;
    if (np * np >= ((int64_t)1 << 32))
        return set_err(ctx, SGP_EINVAL, "factor_augmented: %lld pieces are too many", (long long)np);
    // ---- added contacts
    int32_t *cflag, *coff, *cross, *is_tree, *added, *aoff, *alist;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP5], m + 2, &cflag));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP6], m + 2, &coff));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP7], m + 2, &cross));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP8], m + 2, &is_tree));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP9], m + 2, &added));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_SLOTS], m + 2, &aoff));
    SGP_TRY(fill_i32(ctx, is_tree, 0, m + 1));
    SGP_TRY(fill_i32(ctx, added, 0, m + 1));
    if (T->nt > 0)
        k_aug_treeflags<<<grid_for(T->nt, 256), 256, 0, st>>>(T->nt, (const int32_t *)T->tree_edge.p, is_tree);
    const int32_t *ei = (const int32_t *)g->ei.p, *ej = (const int32_t *)g->ej.p;
    if (m > 0) k_aug_cross<<<grid_for(m, 256), 256, 0, st>>>(m, ei, ej, piece, cflag);
    LAUNCH_CHECK(ctx);
    SGP_TRY(scan_exclusive(ctx, cflag, coff, m));
    if (m > 0) k_aug_compact<<<grid_for(m, 256), 256, 0, st>>>(m, cflag, coff, cross);
    LAUNCH_CHECK(ctx);
    int32_t nc32;
    SGP_TRY(readback(ctx, &nc32, coff + m, 4));
    const int64_t nc = nc32;
    if (nc > 0) {
        uint32_t *pk, *pk2;
        int32_t *pv, *pv2;
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_A], nc, &pk));
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_B], nc, &pk2));
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_A], nc, &pv));
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_B], nc, &pv2));
        k_aug_pairkeys<<<grid_for(nc, 256), 256, 0, st>>>(nc, cross, ei, ej, piece, did, np, pk, pv);
        LAUNCH_CHECK(ctx);
        int kbits = 1;
        while (((int64_t)1 << kbits) < np * np) kbits++;
        SGP_TRY(radix_sort_pairs(ctx, pk, pv, pk2, pv2, nc, kbits));
        k_aug_best<<<grid_for(nc, 256), 256, 0, st>>>(nc, pk, pv, (const double *)g->w.p, is_tree, added);
        LAUNCH_CHECK(ctx);
    }
    SGP_TRY(scan_exclusive(ctx, added, aoff, m));
    int32_t na32;
    SGP_TRY(readback(ctx, &na32, aoff + m, 4));
    const int64_t na = na32;
    M->aug_added = na;
    SGP_TRY(ensure_t(ctx, M->aug_list, na + 1, &alist));
    if (m > 0) k_aug_compact<<<grid_for(m, 256), 256, 0, st>>>(m, added, aoff, alist);
    LAUNCH_CHECK(ctx);
    // ---- incidence of P': the tree's rows and the added contacts' rows
    int32_t *deg, *cur, *aadj, *aadje, *ttp, *tadj_int;
    double4 *awu, *twu;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], n + 2, &deg));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], n + 2, &cur));
    SGP_TRY(fill_i32(ctx, deg, 0, n));
    SGP_TRY(fill_i32(ctx, cur, 0, n));
    if (na > 0) k_aug_deg<<<grid_for(na, 256), 256, 0, st>>>(na, alist, ei, ej, deg);
    LAUNCH_CHECK(ctx);
    SGP_TRY(scan_exclusive(ctx, deg, aptr, n));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP5], 2 * na + 2, &aadj));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP6], 2 * na + 2, &aadje));
    SGP_TRY(ensure_t(ctx, M->aug_adj, 2 * na + 2, &aadj_int));
    SGP_TRY(ensure_t(ctx, M->aug_wu, 2 * na + 2, &awu));
    if (na > 0) {
        k_aug_fill<<<grid_for(na, 256), 256, 0, st>>>(na, alist, ei, ej, aptr, cur, aadj, aadje);
        k_aug_rowsort<<<grid_for(n, 256), 256, 0, st>>>(n, aptr, aadj, aadje);
        k_aug_entries<<<grid_for(2 * na, 256), 256, 0, st>>>(2 * na, aadj, aadje, (const double4 *)g->wu.p,
                                                            (const int32_t *)g->inv.p, aadj_int, awu);
        LAUNCH_CHECK(ctx);
    }
    const int64_t nd = 2 * T->nt;
    SGP_TRY(ensure_t(ctx, M->aug_tptr, n + 2, &ttp));
    SGP_TRY(ensure_t(ctx, M->aug_tadj, nd + 1, &tadj_int));
    SGP_TRY(ensure_t(ctx, M->aug_twu, nd + 1, &twu));
    HIP_TRY(ctx, hipMemcpyAsync(ttp, tptr, (n + 1) * 4, hipMemcpyDeviceToDevice, st));
    if (nd > 0) {
        k_aug_entries<<<grid_for(nd, 256), 256, 0, st>>>(nd, tadj, (const int32_t *)T->tadje.p,
                                                        (const double4 *)g->wu.p, (const int32_t *)g->inv.p, tadj_int,
                                                        twu);
        LAUNCH_CHECK(ctx);
    }
    M->aug = 1;
    return SGP_OK;
}

extern "C" int sgp_prec_augmented(sgp_ctx ctx, sgp_prec M, int64_t *pieces, int64_t *added, int32_t *piece,
                                  int32_t *added_edges)
{
    if (!ctx || !M) return set_err(ctx, SGP_EINVAL, "prec_augmented: null handle");
    if (!M->aug) return set_err(ctx, SGP_EINVAL, "prec_augmented: not an augmented tree");
    if (pieces) *pieces = M->aug_pieces;
    if (added) *added = M->aug_added;
    if (piece && M->n > 0)
        HIP_TRY(ctx, hipMemcpyAsync(piece, M->aug_piece.p, M->n * 4, hipMemcpyDeviceToDevice, ctx->stream));
    if (added_edges && M->aug_added > 0)
        HIP_TRY(ctx, hipMemcpyAsync(added_edges, M->aug_list.p, M->aug_added * 4, hipMemcpyDeviceToDevice,
                                    ctx->stream));
    return SGP_OK;
}

// ---------------------------------------------------------------- the nested solve

struct AugWork {
    sgp_ctx ctx;
    sgp_prec M;
    int64_t n;
    double *part, *dd;
    int nb;
};

static int dots(AugWork &W, const double *a, const double *b, const double *c, const double *d, double *out)
{
    const int64_t len = 3 * W.n;
    k_aug_dots<<<W.nb, 256, 0, W.ctx->stream>>>(len, a, b, c, d, W.part);
    k_aug_dots_fin<<<1, 256, 0, W.ctx->stream>>>(W.nb, W.part, W.dd);
    LAUNCH_CHECK(W.ctx);
    return readback(W.ctx, out, W.dd, 2 * sizeof(double));
}

static int aug_mv(AugWork &W, const double *x, double *y)
{
    sgp_prec M = W.M;
    k_aug_mv<<<grid_for(W.n, 256), 256, 0, W.ctx->stream>>>(
        W.n, (const int32_t *)M->inv.p, (const int32_t *)M->aug_tptr.p, (const int32_t *)M->aug_tadj.p,
        (const double4 *)M->aug_twu.p, (const int32_t *)M->aug_ptr.p, (const int32_t *)M->aug_adj.p,
        (const double4 *)M->aug_wu.p, M->gpar, M->gperp, M->gmed, x, y);
    LAUNCH_CHECK(W.ctx);
    return SGP_OK;
}

// z ~ P'^{-1} r: tree-PCG on P' from zero until ||r_in|| <= inner_rtol ||r||
static int inner_solve(AugWork &W, const double *r, double *z, double *ri, double *zi, double *pi, double *qi,
                       int max_inner, int *iters)
{
    sgp_ctx ctx = W.ctx;
    hipStream_t st = ctx->stream;
    const int64_t len = 3 * W.n;
    const unsigned g = grid_for(len, 256);
    SGP_TRY(fill_f64(ctx, z, 0.0, len));
    HIP_TRY(ctx, hipMemcpyAsync(ri, r, len * 8, hipMemcpyDeviceToDevice, st));
    SGP_TRY(prec_apply_f64(ctx, W.M, ri, zi, nullptr));
    HIP_TRY(ctx, hipMemcpyAsync(pi, zi, len * 8, hipMemcpyDeviceToDevice, st));
    double h[2];
    SGP_TRY(dots(W, ri, ri, ri, zi, h));
    const double nb = sqrt(h[0]);
    double rho = h[1];
    int k = 0;
    while (nb > 0.0 && k < max_inner) {
        SGP_TRY(aug_mv(W, pi, qi));
        SGP_TRY(dots(W, pi, qi, nullptr, nullptr, h));
        if (!(h[0] > 0.0) || !std::isfinite(h[0])) return set_err(ctx, SGP_EBREAKDOWN, "augmented: inner breakdown");
        const double alpha = rho / h[0];
        k_aug_axpy2<<<g, 256, 0, st>>>(len, alpha, pi, qi, z, ri);
        LAUNCH_CHECK(ctx);
        k++;
        SGP_TRY(prec_apply_f64(ctx, W.M, ri, zi, nullptr));
        SGP_TRY(dots(W, ri, ri, ri, zi, h));
        if (sqrt(h[0]) <= W.M->inner_rtol * nb) break;
        const double beta = h[1] / rho;
        rho = h[1];
        k_aug_xpby<<<g, 256, 0, st>>>(len, zi, beta, pi);
        LAUNCH_CHECK(ctx);
    }
    *iters = k;
    return SGP_OK;
}

// Flexible CG (one direction kept): alpha = p.r / p.q, beta = -z.q / p.q.
// F and x in the internal order.
int solve_augmented(sgp_ctx ctx, sgp_bsr A, sgp_prec M, const double *F, double *x, const sgp_solve_opts *o,
                    sgp_solve_info *info)
{
    hipStream_t st = ctx->stream;
    const int64_t n = A->n, len = 3 * n;
    memset(info, 0, sizeof *info);
    if (M->n != n) return set_err(ctx, SGP_EINVAL, "pcg_solve: preconditioner and matrix differ in size");
    double *r, *z, *p, *q, *ri, *zi, *pi, *qi, *part, *dd;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP0], len + 3, &r));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP1], len + 3, &z));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP2], len + 3, &p));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], len + 3, &q));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], len + 3, &ri));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP5], len + 3, &zi));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP6], len + 3, &pi));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP7], len + 3, &qi));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PART], 2 * RED_BLOCKS + 8, &part));
    dd = part + 2 * RED_BLOCKS;
    AugWork W = {ctx, M, n, part, dd, RED_BLOCKS};
    const unsigned g = grid_for(len, 256);
    const int max_iter = o->max_iter > 0 ? o->max_iter : 10000;
    const int max_inner = 10000;
    if (!o->use_x0) SGP_TRY(fill_f64(ctx, x, 0.0, len));
    SGP_TRY(spmv_f64(ctx, A, x, q, nullptr, nullptr, 0));
    k_aug_sub<<<g, 256, 0, st>>>(len, F, q, r);
    LAUNCH_CHECK(ctx);
    double h[2];
    SGP_TRY(dots(W, F, F, r, r, h));
    const double nF = sqrt(h[0]);
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) {
        info->status = SGP_ENONFINITE;
        return set_err(ctx, SGP_ENONFINITE, "pcg_solve: non-finite input");
    }
    if (nF == 0.0) {
        SGP_TRY(fill_f64(ctx, x, 0.0, len));
        return SGP_OK;
    }
    double relres = sqrt(h[1]) / nF;
    int k = 0, inner_total = 0, status = SGP_OK;
    if (relres > o->rtol) {
        int it = 0;
        SGP_TRY(inner_solve(W, r, z, ri, zi, pi, qi, max_inner, &it));
        inner_total += it;
        HIP_TRY(ctx, hipMemcpyAsync(p, z, len * 8, hipMemcpyDeviceToDevice, st));
        for (;;) {
            if (k >= max_iter) {
                status = SGP_ENOCONV;
                break;
            }
            SGP_TRY(spmv_f64(ctx, A, p, q, nullptr, nullptr, 0));
            SGP_TRY(dots(W, p, q, p, r, h));
            const double pq = h[0];
            if (!(pq > 0.0) || !std::isfinite(pq)) {
                status = SGP_EBREAKDOWN;
                break;
            }
            k_aug_axpy2<<<g, 256, 0, st>>>(len, h[1] / pq, p, q, x, r);
            LAUNCH_CHECK(ctx);
            k++;
            SGP_TRY(dots(W, r, r, nullptr, nullptr, h));
            relres = sqrt(h[0]) / nF;
            if (!std::isfinite(relres)) {
                status = SGP_ENONFINITE;
                break;
            }
            if (relres <= o->rtol) break;
            SGP_TRY(inner_solve(W, r, z, ri, zi, pi, qi, max_inner, &it));
            inner_total += it;
            SGP_TRY(dots(W, z, q, nullptr, nullptr, h));
            k_aug_xpby<<<g, 256, 0, st>>>(len, z, -h[0] / pq, p);
            LAUNCH_CHECK(ctx);
        }
    }
    // true residual
    SGP_TRY(spmv_f64(ctx, A, x, q, nullptr, nullptr, 0));
    k_aug_sub<<<g, 256, 0, st>>>(len, F, q, r);
    LAUNCH_CHECK(ctx);
    SGP_TRY(dots(W, r, r, nullptr, nullptr, h));
    info->status = status;
    info->iters = k;
    info->inner_iters = inner_total;
    info->relres_rec = relres;
    info->relres_true = sqrt(h[0]) / nF;
    return status == SGP_OK ? SGP_OK : set_err(ctx, status, "pcg_solve (augmented): status %d", status);
}
