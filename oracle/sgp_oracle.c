/*
 * sgp_oracle.c -- plain, slow, single-threaded FP64 CPU reference of the
 * support-graph-preconditioned CG solve of Gamma v = F (Steinman &
 * Buttenschoen, "Support Graph Preconditioners for Off-Lattice Cell-Based
 * Models", arXiv 2410.04512).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU library is
 * compared against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library, and it includes nothing from it.
 *
 * Every function follows one passage of the paper and is written for reading,
 * not for speed: no blocking, no fusion, no reordering beyond what the cited
 * passage states.  Build with  gcc -O2 -ffp-contract=off  so that no multiply
 * is fused into an add behind our back (the contact geometry must round the
 * same way as the definition written here).
 *
 * Readings of the paper taken here (where it is silent or ambiguous):
 *  - contact: d_ij = sqrt((dx*dx + dy*dy) + dz*dz), dx = x_j - x_i, contact
 *    iff d_ij < R_i + R_j (strict), overlap w_ij = (R_i + R_j) - d_ij stands
 *    in for the contact area A_ij, u_ij = (r_j - r_i)/d_ij for i < j.
 *  - edges are numbered in lexicographic (i, j), i < j order.
 *  - maximum spanning tree weight: w_ij itself; ties broken by smaller edge
 *    id; disconnected graphs give a spanning forest.
 *  - each tree component is rooted at its smallest vertex id.
 *  - P_ii = g_med I + sum over TREE edges at i of W_e (self-loops included).
 *  - the transposes missing from Alg. 2 are restored: the child term is
 *    L_ij D_jj L_ij^T and L_{p(i),i} = A_{p(i),i} D_ii^{-1}.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOTSPD (-5)
#define ORC_ENOCONV (-6)
#define ORC_EBREAKDOWN (-7)
#define ORC_ENONFINITE (-8)

/* ------------------------------------------------------------------------ */
/* Step 1-2 of the off-lattice step (Section 2): which cells touch.          */
/* ------------------------------------------------------------------------ */

/* The contact test and geometry of one ordered pair i < j.
 * Returns 1 for a contact, 0 for none, -1 for coincident centres (u undefined). */
static int contact_pair(const double *pos, const double *R, int64_t i, int64_t j,
                        double *w, double u[3])
{
    double dx = pos[3 * j + 0] - pos[3 * i + 0];
    double dy = pos[3 * j + 1] - pos[3 * i + 1];
    double dz = pos[3 * j + 2] - pos[3 * i + 2];
    double d = sqrt((dx * dx + dy * dy) + dz * dz);
    double s = R[i] + R[j];
    if (!(d < s)) return 0;
    if (d == 0.0) return -1;
    *w = s - d;
    u[0] = dx / d;
    u[1] = dy / d;
    u[2] = dz / d;
    return 1;
}

/* Result of collision detection: the collision graph as an edge list in
 * lexicographic order plus its symmetric CSR neighbour list (rows sorted). */
typedef struct {
    int64_t n, m;
    int32_t *rowptr; /* [n+1] */
    int32_t *col;    /* [2m]  */
    int32_t *ei, *ej;/* [m]   */
    double *w;       /* [m]   */
    double *u;       /* [m][3] */
} orc_graph;

void orc_graph_free(orc_graph *g)
{
    if (!g) return;
    free(g->rowptr); free(g->col); free(g->ei); free(g->ej); free(g->w); free(g->u);
    free(g);
}

/* Growable edge list used while scanning pairs. */
typedef struct { int64_t m, cap; int32_t *ei, *ej; double *w, *u; } edge_buf;

static int edge_push(edge_buf *b, int32_t i, int32_t j, double w, const double u[3])
{
    if (b->m == b->cap) {
        int64_t nc = b->cap ? 2 * b->cap : 1024;
        int32_t *a = realloc(b->ei, nc * sizeof(int32_t));
        if (!a) return ORC_ENOMEM;
        b->ei = a;
        a = realloc(b->ej, nc * sizeof(int32_t));
        if (!a) return ORC_ENOMEM;
        b->ej = a;
        double *d = realloc(b->w, nc * sizeof(double));
        if (!d) return ORC_ENOMEM;
        b->w = d;
        d = realloc(b->u, 3 * nc * sizeof(double));
        if (!d) return ORC_ENOMEM;
        b->u = d;
        b->cap = nc;
    }
    b->ei[b->m] = i; b->ej[b->m] = j; b->w[b->m] = w;
    b->u[3 * b->m + 0] = u[0]; b->u[3 * b->m + 1] = u[1]; b->u[3 * b->m + 2] = u[2];
    b->m++;
    return ORC_OK;
}

/* Symmetric neighbour CSR from a lexicographically ordered edge list.  Rows
 * come out sorted: row i first receives the edges (k, i), k < i, in k order,
 * then the edges (i, j), j > i, in j order. */
static orc_graph *graph_from_edges(int64_t n, edge_buf *b, int *status)
{
    orc_graph *g = calloc(1, sizeof(orc_graph));
    if (!g) { *status = ORC_ENOMEM; return NULL; }
    g->n = n; g->m = b->m;
    g->ei = b->ei; g->ej = b->ej; g->w = b->w; g->u = b->u;
    g->rowptr = calloc((size_t)n + 1, sizeof(int32_t));
    g->col = malloc((size_t)(2 * b->m + 1) * sizeof(int32_t));
    int32_t *fill = calloc((size_t)n + 1, sizeof(int32_t));
    if (!g->rowptr || !g->col || !fill) { free(fill); orc_graph_free(g); *status = ORC_ENOMEM; return NULL; }
    for (int64_t e = 0; e < b->m; e++) { g->rowptr[b->ei[e] + 1]++; g->rowptr[b->ej[e] + 1]++; }
    for (int64_t i = 0; i < n; i++) g->rowptr[i + 1] += g->rowptr[i];
    for (int64_t e = 0; e < b->m; e++) {
        int32_t i = b->ei[e], j = b->ej[e];
        g->col[g->rowptr[i] + fill[i]++] = j;
        g->col[g->rowptr[j] + fill[j]++] = i;
    }
    free(fill);
    *status = ORC_OK;
    return g;
}

/* All-pairs collision detection: every pair i < j is tested.  O(n^2). */
orc_graph *orc_collide_brute(int64_t n, const double *pos, const double *R, int *status)
{
    edge_buf b = {0};
    for (int64_t i = 0; i < n; i++) {
        for (int64_t j = i + 1; j < n; j++) {
            double w, u[3];
            int c = contact_pair(pos, R, i, j, &w, u);
            if (c < 0) { *status = ORC_EINVAL; goto fail; }
            if (c > 0 && (*status = edge_push(&b, (int32_t)i, (int32_t)j, w, u)) != ORC_OK) goto fail;
        }
    }
    return graph_from_edges(n, &b, status);
fail:
    free(b.ei); free(b.ej); free(b.w); free(b.u);
    return NULL;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Uniform-grid collision detection: cells of side h = 2 max R, so every
 * contact pair lies in the same or an adjacent cell.  Same pair test and the
 * same lexicographic output as the all-pairs version. */
orc_graph *orc_collide_cells(int64_t n, const double *pos, const double *R, int *status)
{
    edge_buf b = {0};
    if (n == 0) return graph_from_edges(0, &b, status);
    double lo[3], hi[3], rmax = 0.0;
    for (int a = 0; a < 3; a++) { lo[a] = pos[a]; hi[a] = pos[a]; }
    for (int64_t i = 0; i < n; i++) {
        for (int a = 0; a < 3; a++) {
            if (!isfinite(pos[3 * i + a])) { *status = ORC_ENONFINITE; return NULL; }
            if (pos[3 * i + a] < lo[a]) lo[a] = pos[3 * i + a];
            if (pos[3 * i + a] > hi[a]) hi[a] = pos[3 * i + a];
        }
        if (!(R[i] >= 0.0) || !isfinite(R[i])) { *status = ORC_EINVAL; return NULL; }
        if (R[i] > rmax) rmax = R[i];
    }
    /* A touching pair is closer than 2 max R; the small margin keeps a pair
     * that is closer than h by less than a rounding error of (x - lo)/h from
     * landing two cells apart.  A larger cell never loses a pair. */
    double h = 2.0 * rmax * (1.0 + 0x1p-20);
    if (h <= 0.0) h = 1.0;
    int64_t dim[3];
    for (int a = 0; a < 3; a++) dim[a] = (int64_t)floor((hi[a] - lo[a]) / h) + 1;
    int64_t ncell = dim[0] * dim[1] * dim[2];
    int64_t *cell = malloc((size_t)n * sizeof(int64_t));
    int64_t *start = calloc((size_t)ncell + 1, sizeof(int64_t));
    int32_t *members = malloc((size_t)n * sizeof(int32_t));
    int32_t *cand = malloc((size_t)n * sizeof(int32_t));
    if (!cell || !start || !members || !cand) { *status = ORC_ENOMEM; goto fail; }
    for (int64_t i = 0; i < n; i++) {
        int64_t c[3];
        for (int a = 0; a < 3; a++) {
            c[a] = (int64_t)floor((pos[3 * i + a] - lo[a]) / h);
            if (c[a] >= dim[a]) c[a] = dim[a] - 1;
        }
        cell[i] = (c[2] * dim[1] + c[1]) * dim[0] + c[0];
        start[cell[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; c++) start[c + 1] += start[c];
    {
        int64_t *put = malloc((size_t)ncell * sizeof(int64_t));
        if (!put) { *status = ORC_ENOMEM; goto fail; }
        memcpy(put, start, (size_t)ncell * sizeof(int64_t));
        for (int64_t i = 0; i < n; i++) members[put[cell[i]]++] = (int32_t)i;
        free(put);
    }
    for (int64_t i = 0; i < n; i++) {
        int64_t ci = cell[i];
        int64_t c0 = ci % dim[0], c1 = (ci / dim[0]) % dim[1], c2 = ci / (dim[0] * dim[1]);
        int64_t nc = 0;
        for (int64_t z = c2 - 1; z <= c2 + 1; z++) {
            if (z < 0 || z >= dim[2]) continue;
            for (int64_t y = c1 - 1; y <= c1 + 1; y++) {
                if (y < 0 || y >= dim[1]) continue;
                for (int64_t x = c0 - 1; x <= c0 + 1; x++) {
                    if (x < 0 || x >= dim[0]) continue;
                    int64_t c = (z * dim[1] + y) * dim[0] + x;
                    for (int64_t k = start[c]; k < start[c + 1]; k++)
                        if (members[k] > i) cand[nc++] = members[k];
                }
            }
        }
        qsort(cand, (size_t)nc, sizeof(int32_t), cmp_i32);
        for (int64_t k = 0; k < nc; k++) {
            double w, u[3];
            int c = contact_pair(pos, R, i, cand[k], &w, u);
            if (c < 0) { *status = ORC_EINVAL; goto fail; }
            if (c > 0 && (*status = edge_push(&b, (int32_t)i, cand[k], w, u)) != ORC_OK) goto fail;
        }
    }
    free(cell); free(start); free(members); free(cand);
    return graph_from_edges(n, &b, status);
fail:
    free(cell); free(start); free(members); free(cand);
    free(b.ei); free(b.ej); free(b.w); free(b.u);
    return NULL;
}

/* The contact area of the Hertz model for the paper's benchmark cells
 * (Section 5.1 names the model without its formula): two spheres of radii
 * R_i, R_j pressed together by the overlap delta touch in a disc of radius
 * a = sqrt(R* delta), R* = R_i R_j / (R_i + R_j), so the area is
 * A = pi R* delta.  w holds delta on entry and A on return:
 * A = (pi * ((R_i * R_j) / (R_i + R_j))) * delta, in that order. */
void orc_hertz_area(int64_t m, const int32_t *ei, const int32_t *ej, const double *R, double *w)
{
    const double pi = 3.14159265358979323846;
    for (int64_t e = 0; e < m; e++) {
        double ri = R[ei[e]], rj = R[ej[e]];
        double rs = (ri * rj) / (ri + rj);
        w[e] = (pi * rs) * w[e];
    }
}

/* ------------------------------------------------------------------------ */
/* Section 6 (Discussion): clusters of a spatial subdivision, each with its  */
/* own spanning tree.                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t inst;
    uint64_t z;
    int32_t id;
} zcell;

static int cmp_zcell(const void *pa, const void *pb)
{
    const zcell *a = pa, *b = pb;
    if (a->inst != b->inst) return a->inst < b->inst ? -1 : 1;
    if (a->z != b->z) return a->z < b->z ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* The cells of every instance (instance k: cells off[k] .. off[k+1]-1) in the
 * Z-order of a uniform grid, cut into runs of K; cluster ids run instance by
 * instance.  Grid: cubes of side h = 2 max R (1 if every radius is 0) with a
 * corner at the bounding box's minimum over all cells; the coordinates of a
 * cell are floor((x - lo) / h) per axis, and its Z-order position is the
 * Morton code: bit b of the x, y and z coordinates becomes bit 3b, 3b + 1 and
 * 3b + 2.  Equal codes keep the cell ids in order. */
int orc_forest_clusters(int64_t n, const double *pos, const double *R, int64_t n_inst, const int64_t *off,
                        int32_t K, int32_t *cluster)
{
    if (n == 0) return ORC_OK;
    if (K < 1) return ORC_EINVAL;
    double lo[3] = {pos[0], pos[1], pos[2]}, rmax = 0.0;
    for (int64_t i = 0; i < n; i++) {
        for (int a = 0; a < 3; a++)
            if (pos[3 * i + a] < lo[a]) lo[a] = pos[3 * i + a];
        if (R[i] > rmax) rmax = R[i];
    }
    double h = rmax > 0.0 ? 2.0 * rmax : 1.0;
    zcell *c = malloc((size_t)n * sizeof(zcell));
    if (!c) return ORC_ENOMEM;
    int64_t k = 0;
    for (int64_t i = 0; i < n; i++) {
        while (i >= off[k + 1]) k++;
        uint64_t z = 0;
        for (int a = 0; a < 3; a++) {
            double f = floor((pos[3 * i + a] - lo[a]) / h);
            uint64_t ca = f > 0.0 ? (uint64_t)f : 0;
            for (int b = 0; b < 21; b++) z |= ((ca >> b) & 1u) << (3 * b + a);
        }
        c[i].inst = k;
        c[i].z = z;
        c[i].id = (int32_t)i;
    }
    qsort(c, (size_t)n, sizeof(zcell), cmp_zcell);
    int32_t first = 0;   /* first cluster id of the current instance */
    for (int64_t q = 0; q < n_inst; q++) {
        for (int64_t p = off[q]; p < off[q + 1]; p++) cluster[c[p].id] = first + (int32_t)((p - off[q]) / K);
        first += (int32_t)((off[q + 1] - off[q] + K - 1) / K);
    }
    free(c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Step 3 (eq. cell_cell_friction) and the block Laplacian (Definition).     */
/* ------------------------------------------------------------------------ */

/* W = w (g_par u (x) u + g_perp (I - u (x) u)), written out entry by entry. */
static void friction_block(double w, const double u[3], double g_par, double g_perp, double W[9])
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double uu = u[a] * u[b];
            double id = (a == b) ? 1.0 : 0.0;
            W[3 * a + b] = w * (g_par * uu + g_perp * (id - uu));
        }
}

void orc_friction_block(double w, const double *u, double g_par, double g_perp, double *W)
{
    friction_block(w, u, g_par, g_perp, W);
}

/* Edge id of the contact (i, j) in the lexicographic edge list (binary search
 * in row min(i,j) of the upper neighbour list). */
static int64_t edge_id(const orc_graph *g, const int32_t *first_edge, int32_t i, int32_t j)
{
    int32_t a = i < j ? i : j, b = i < j ? j : i;
    int64_t lo = first_edge[a], hi = first_edge[a + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (g->ej[mid] < b) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Gamma as a 3x3-block CSR matrix: row i holds the columns of its neighbours
 * and itself in ascending order.  Off-diagonal block -W_e; diagonal block
 * g_med I plus the W_e of row i's contacts added in ascending column order.
 * rowptr [n+1], bcol [n+2m], val [n+2m][9] are caller-allocated. */
int orc_assemble(int64_t n, int64_t m, const int32_t *g_rowptr, const int32_t *g_col,
                 const int32_t *ei, const int32_t *ej, const double *w, const double *u,
                 double g_par, double g_perp, double g_med,
                 int32_t *rowptr, int32_t *bcol, double *val)
{
    orc_graph g = {n, m, (int32_t *)g_rowptr, (int32_t *)g_col, (int32_t *)ei, (int32_t *)ej,
                   (double *)w, (double *)u};
    int32_t *first_edge = calloc((size_t)n + 1, sizeof(int32_t));
    if (!first_edge) return ORC_ENOMEM;
    for (int64_t e = 0; e < m; e++) first_edge[ei[e] + 1]++;
    for (int64_t i = 0; i < n; i++) first_edge[i + 1] += first_edge[i];
    rowptr[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t k = rowptr[i];
        double diag[9];
        for (int t = 0; t < 9; t++) diag[t] = (t % 4 == 0) ? g_med : 0.0;
        int placed_diag = 0;
        int32_t kdiag = -1;
        for (int32_t p = g_rowptr[i]; p < g_rowptr[i + 1]; p++) {
            int32_t j = g_col[p];
            if (!placed_diag && j > i) { kdiag = k; bcol[k++] = (int32_t)i; placed_diag = 1; }
            int64_t e = edge_id(&g, first_edge, (int32_t)i, j);
            double W[9];
            friction_block(w[e], &u[3 * e], g_par, g_perp, W);
            for (int t = 0; t < 9; t++) { val[9 * (int64_t)k + t] = -W[t]; diag[t] = diag[t] + W[t]; }
            bcol[k++] = j;
        }
        if (!placed_diag) { kdiag = k; bcol[k++] = (int32_t)i; }
        for (int t = 0; t < 9; t++) val[9 * (int64_t)kdiag + t] = diag[t];
        rowptr[i + 1] = k;
    }
    free(first_edge);
    return ORC_OK;
}

/* y = Gamma x for the block-CSR matrix (row by row, blocks in column order). */
void orc_spmv(int64_t n, const int32_t *rowptr, const int32_t *bcol, const double *val,
              const double *x, double *y)
{
    for (int64_t i = 0; i < n; i++) {
        double s[3] = {0.0, 0.0, 0.0};
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; k++) {
            const double *B = &val[9 * (int64_t)k];
            const double *xj = &x[3 * (int64_t)bcol[k]];
            for (int a = 0; a < 3; a++)
                s[a] = s[a] + (B[3 * a + 0] * xj[0] + B[3 * a + 1] * xj[1] + B[3 * a + 2] * xj[2]);
        }
        y[3 * i + 0] = s[0]; y[3 * i + 1] = s[1]; y[3 * i + 2] = s[2];
    }
}

/* ------------------------------------------------------------------------ */
/* Section 3.1: maximum spanning tree (forest) of the collision graph.        */
/* ------------------------------------------------------------------------ */

/* Strict total order on edges: heavier first, then smaller edge id. */
static int edge_before(const double *w, int64_t a, int64_t b)
{
    if (w[a] != w[b]) return w[a] > w[b];
    return a < b;
}

/* Binary max-heap of edge ids under edge_before. */
typedef struct { int64_t *e; int64_t size, cap; const double *w; } edge_heap;

static int heap_push(edge_heap *h, int64_t e)
{
    if (h->size == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        int64_t *a = realloc(h->e, (size_t)nc * sizeof(int64_t));
        if (!a) return ORC_ENOMEM;
        h->e = a; h->cap = nc;
    }
    int64_t k = h->size++;
    h->e[k] = e;
    while (k > 0) {
        int64_t p = (k - 1) / 2;
        if (!edge_before(h->w, h->e[k], h->e[p])) break;
        int64_t t = h->e[k]; h->e[k] = h->e[p]; h->e[p] = t;
        k = p;
    }
    return ORC_OK;
}

static int64_t heap_pop(edge_heap *h)
{
    int64_t top = h->e[0];
    h->e[0] = h->e[--h->size];
    int64_t k = 0;
    for (;;) {
        int64_t l = 2 * k + 1, r = l + 1, best = k;
        if (l < h->size && edge_before(h->w, h->e[l], h->e[best])) best = l;
        if (r < h->size && edge_before(h->w, h->e[r], h->e[best])) best = r;
        if (best == k) break;
        int64_t t = h->e[k]; h->e[k] = h->e[best]; h->e[best] = t;
        k = best;
    }
    return top;
}

/* Incidence lists: for each vertex the ids of its edges, ascending. */
static int incidence(int64_t n, int64_t m, const int32_t *ei, const int32_t *ej,
                     int32_t **ptr_out, int32_t **inc_out)
{
    int32_t *ptr = calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *inc = malloc((size_t)(2 * m + 1) * sizeof(int32_t));
    int32_t *fill = calloc((size_t)n + 1, sizeof(int32_t));
    if (!ptr || !inc || !fill) { free(ptr); free(inc); free(fill); return ORC_ENOMEM; }
    for (int64_t e = 0; e < m; e++) { ptr[ei[e] + 1]++; ptr[ej[e] + 1]++; }
    for (int64_t i = 0; i < n; i++) ptr[i + 1] += ptr[i];
    for (int64_t e = 0; e < m; e++) {
        inc[ptr[ei[e]] + fill[ei[e]]++] = (int32_t)e;
        inc[ptr[ej[e]] + fill[ej[e]]++] = (int32_t)e;
    }
    free(fill);
    *ptr_out = ptr; *inc_out = inc;
    return ORC_OK;
}

/* Prim's algorithm (Section 3.1, Fig. 1 C), lazy variant with a binary heap:
 * start at vertex 0; repeatedly take the heaviest edge (ties: smaller id)
 * leaving the visited set; when the heap runs dry and vertices remain, restart
 * at the smallest unvisited vertex (spanning forest).
 * tree_edge [n] receives the chosen edge ids in the order Prim adds them;
 * visit [n] receives the vertices in the order Prim visits them.
 * Returns the number of tree edges, or a negative status. */
int64_t orc_prim(int64_t n, int64_t m, const int32_t *ei, const int32_t *ej, const double *w,
                 int32_t *tree_edge, int32_t *visit)
{
    int32_t *ptr, *inc;
    if (incidence(n, m, ei, ej, &ptr, &inc) != ORC_OK) return ORC_ENOMEM;
    char *seen = calloc((size_t)n + 1, 1);
    edge_heap h = {NULL, 0, 0, w};
    if (!seen) { free(ptr); free(inc); return ORC_ENOMEM; }
    int64_t nt = 0, nv = 0;
    for (int64_t s = 0; s < n; s++) {
        if (seen[s]) continue;
        seen[s] = 1; visit[nv++] = (int32_t)s;
        for (int32_t k = ptr[s]; k < ptr[s + 1]; k++)
            if (heap_push(&h, inc[k]) != ORC_OK) goto nomem;
        while (h.size > 0) {
            int64_t e = heap_pop(&h);
            int32_t a = ei[e], b = ej[e];
            int32_t v = seen[a] ? b : a;
            if (seen[a] && seen[b]) continue;
            seen[v] = 1; visit[nv++] = v;
            tree_edge[nt++] = (int32_t)e;
            for (int32_t k = ptr[v]; k < ptr[v + 1]; k++) {
                int64_t f = inc[k];
                int32_t o = (ei[f] == v) ? ej[f] : ei[f];
                if (!seen[o] && heap_push(&h, f) != ORC_OK) goto nomem;
            }
        }
    }
    free(ptr); free(inc); free(seen); free(h.e);
    return nt;
nomem:
    free(ptr); free(inc); free(seen); free(h.e);
    return ORC_ENOMEM;
}

/* Kruskal's algorithm as an independent check of Prim: scan the edges in the
 * same strict order, keep an edge when it joins two different components
 * (union-find).  tree_edge receives the kept ids in scan order. */
static const double *g_sort_w;
static int cmp_edge_order(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (a == b) return 0;
    return edge_before(g_sort_w, a, b) ? -1 : 1;
}

static int32_t uf_find(int32_t *par, int32_t x)
{
    while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
    return x;
}

int64_t orc_kruskal(int64_t n, int64_t m, const int32_t *ei, const int32_t *ej, const double *w,
                    int32_t *tree_edge)
{
    int64_t *order = malloc((size_t)(m + 1) * sizeof(int64_t));
    int32_t *par = malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!order || !par) { free(order); free(par); return ORC_ENOMEM; }
    for (int64_t e = 0; e < m; e++) order[e] = e;
    g_sort_w = w;
    qsort(order, (size_t)m, sizeof(int64_t), cmp_edge_order);
    for (int64_t i = 0; i < n; i++) par[i] = (int32_t)i;
    int64_t nt = 0;
    for (int64_t k = 0; k < m; k++) {
        int64_t e = order[k];
        int32_t a = uf_find(par, ei[e]), b = uf_find(par, ej[e]);
        if (a == b) continue;
        par[a] = b;
        tree_edge[nt++] = (int32_t)e;
    }
    free(order); free(par);
    return nt;
}

/* Root every tree component at its smallest vertex and record parent, the
 * edge to the parent and the hop depth (breadth-first from the root).
 * parent[root] = -1, pedge[root] = -1. */
int orc_root_forest(int64_t n, int64_t nt, const int32_t *tree_edge,
                    const int32_t *ei, const int32_t *ej,
                    int32_t *parent, int32_t *pedge, int32_t *depth)
{
    int32_t *tei = malloc((size_t)(nt + 1) * sizeof(int32_t));
    int32_t *tej = malloc((size_t)(nt + 1) * sizeof(int32_t));
    int32_t *queue = malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!tei || !tej || !queue) { free(tei); free(tej); free(queue); return ORC_ENOMEM; }
    for (int64_t k = 0; k < nt; k++) { tei[k] = ei[tree_edge[k]]; tej[k] = ej[tree_edge[k]]; }
    int32_t *ptr, *inc;
    if (incidence(n, nt, tei, tej, &ptr, &inc) != ORC_OK) { free(tei); free(tej); free(queue); return ORC_ENOMEM; }
    for (int64_t v = 0; v < n; v++) { parent[v] = -2; pedge[v] = -1; depth[v] = -1; }
    for (int64_t s = 0; s < n; s++) {
        if (parent[s] != -2) continue;
        parent[s] = -1; depth[s] = 0;
        int64_t qh = 0, qt = 0;
        queue[qt++] = (int32_t)s;
        while (qh < qt) {
            int32_t v = queue[qh++];
            for (int32_t k = ptr[v]; k < ptr[v + 1]; k++) {
                int32_t t = inc[k];
                int32_t o = (tei[t] == v) ? tej[t] : tei[t];
                if (parent[o] != -2) continue;
                parent[o] = v; pedge[o] = tree_edge[t]; depth[o] = depth[v] + 1;
                queue[qt++] = o;
            }
        }
    }
    free(tei); free(tej); free(queue); free(ptr); free(inc);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Section 3.3, Alg. 2 (TreeLDLT) and Appendix B.1 (tree solves).             */
/* ------------------------------------------------------------------------ */

/* Cholesky of a symmetric 3x3 block, C lower triangular with D = C C^T.
 * Returns ORC_ENOTSPD on a non-positive (or non-finite) pivot. */
static int chol3(const double D[9], double C[9])
{
    for (int t = 0; t < 9; t++) C[t] = 0.0;
    for (int j = 0; j < 3; j++) {
        double s = D[3 * j + j];
        for (int k = 0; k < j; k++) s = s - C[3 * j + k] * C[3 * j + k];
        if (!(s > 0.0) || !isfinite(s)) return ORC_ENOTSPD;
        C[3 * j + j] = sqrt(s);
        for (int i = j + 1; i < 3; i++) {
            double t = D[3 * i + j];
            for (int k = 0; k < j; k++) t = t - C[3 * i + k] * C[3 * j + k];
            C[3 * i + j] = t / C[3 * j + j];
        }
    }
    return ORC_OK;
}

/* Solve (C C^T) x = b with the Cholesky factor from chol3. */
static void chol3_solve(const double C[9], const double b[3], double x[3])
{
    double y[3];
    for (int i = 0; i < 3; i++) {
        double s = b[i];
        for (int k = 0; k < i; k++) s = s - C[3 * i + k] * y[k];
        y[i] = s / C[3 * i + i];
    }
    for (int i = 2; i >= 0; i--) {
        double s = y[i];
        for (int k = i + 1; k < 3; k++) s = s - C[3 * k + i] * x[k];
        x[i] = s / C[3 * i + i];
    }
}

/* Vertices children-before-parent: decreasing depth, ties by id. */
static int64_t *g_depth_sort;
static int cmp_depth_desc(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    if (g_depth_sort[a] != g_depth_sort[b]) return g_depth_sort[a] > g_depth_sort[b] ? -1 : 1;
    return (a > b) - (a < b);
}

/* Elimination order (decreasing depth, as Alg. 2 line 3 states) and the
 * children lists (CSR, ascending ids). */
int orc_tree_order(int64_t n, const int32_t *parent, const int32_t *depth,
                   int32_t *order, int32_t *child_ptr, int32_t *child)
{
    g_depth_sort = malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!g_depth_sort) return ORC_ENOMEM;
    for (int64_t v = 0; v < n; v++) { g_depth_sort[v] = depth[v]; order[v] = (int32_t)v; }
    qsort(order, (size_t)n, sizeof(int32_t), cmp_depth_desc);
    free(g_depth_sort); g_depth_sort = NULL;
    for (int64_t v = 0; v <= n; v++) child_ptr[v] = 0;
    for (int64_t v = 0; v < n; v++) if (parent[v] >= 0) child_ptr[parent[v] + 1]++;
    for (int64_t v = 0; v < n; v++) child_ptr[v + 1] += child_ptr[v];
    int32_t *fill = calloc((size_t)n + 1, sizeof(int32_t));
    if (!fill) return ORC_ENOMEM;
    for (int64_t v = 0; v < n; v++)
        if (parent[v] >= 0) child[child_ptr[parent[v]] + fill[parent[v]]++] = (int32_t)v;
    free(fill);
    return ORC_OK;
}

/* Block Laplacian P of the spanning forest (Section 3.1, self-loops
 * included): P_ii = g_med I + sum of W_e over tree edges at i (ascending tree
 * edge id), P_{p(i),i} = -W_{pedge(i)}.  Then TreeLDLT (Alg. 2): for i in
 * decreasing depth, X = sum over children j (ascending) of L_ij D_jj L_ij^T,
 * D_ii = P_ii - X, and for the parent p: L_{p,i} = P_{p,i} D_ii^{-1}.
 * Outputs per vertex i: D [n][9] (the pivot block) and L [n][9] (the block
 * L_{p(i),i}, zero for roots).  tree_edge must be sorted ascending. */
int orc_tree_factor(int64_t n, int64_t nt, const int32_t *tree_edge,
                    const int32_t *ei, const int32_t *ej, const double *w, const double *u,
                    double g_par, double g_perp, double g_med,
                    const int32_t *parent, const int32_t *pedge,
                    const int32_t *order, const int32_t *child_ptr, const int32_t *child,
                    double *D, double *L)
{
    /* P_ii */
    double *Pd = malloc((size_t)(9 * n + 1) * sizeof(double));
    if (!Pd) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; i++)
        for (int t = 0; t < 9; t++) Pd[9 * i + t] = (t % 4 == 0) ? g_med : 0.0;
    for (int64_t k = 0; k < nt; k++) {
        int64_t e = tree_edge[k];
        double W[9];
        friction_block(w[e], &u[3 * e], g_par, g_perp, W);
        for (int t = 0; t < 9; t++) {
            Pd[9 * (int64_t)ei[e] + t] = Pd[9 * (int64_t)ei[e] + t] + W[t];
            Pd[9 * (int64_t)ej[e] + t] = Pd[9 * (int64_t)ej[e] + t] + W[t];
        }
    }
    int status = ORC_OK;
    for (int64_t q = 0; q < n; q++) {
        int32_t i = order[q];
        double X[9] = {0};
        for (int32_t c = child_ptr[i]; c < child_ptr[i + 1]; c++) {
            int32_t j = child[c];
            const double *Lij = &L[9 * (int64_t)j];  /* L_{i,j}, stored at the child */
            const double *Dj = &D[9 * (int64_t)j];
            double T[9];                               /* T = L_ij D_jj */
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    T[3 * a + b] = Lij[3 * a + 0] * Dj[0 + b] + Lij[3 * a + 1] * Dj[3 + b] + Lij[3 * a + 2] * Dj[6 + b];
            for (int a = 0; a < 3; a++)             /* X += T L_ij^T */
                for (int b = 0; b < 3; b++)
                    X[3 * a + b] = X[3 * a + b] + (T[3 * a + 0] * Lij[3 * b + 0] + T[3 * a + 1] * Lij[3 * b + 1] + T[3 * a + 2] * Lij[3 * b + 2]);
        }
        for (int t = 0; t < 9; t++) D[9 * (int64_t)i + t] = Pd[9 * (int64_t)i + t] - X[t];
        double C[9];
        if (chol3(&D[9 * (int64_t)i], C) != ORC_OK) { status = ORC_ENOTSPD; break; }
        if (parent[i] < 0) { for (int t = 0; t < 9; t++) L[9 * (int64_t)i + t] = 0.0; continue; }
        /* L_{p,i} = A_{p,i} D_ii^{-1}: solve D_ii L^T = A_{p,i}^T column by column. */
        int64_t e = pedge[i];
        double W[9], A[9];
        friction_block(w[e], &u[3 * e], g_par, g_perp, W);
        for (int t = 0; t < 9; t++) A[t] = -W[t];
        for (int r = 0; r < 3; r++) {           /* row r of L = solve(D, row r of A) */
            double b[3] = {A[3 * r + 0], A[3 * r + 1], A[3 * r + 2]}, x[3];
            chol3_solve(C, b, x);
            L[9 * (int64_t)i + 3 * r + 0] = x[0];
            L[9 * (int64_t)i + 3 * r + 1] = x[1];
            L[9 * (int64_t)i + 3 * r + 2] = x[2];
        }
    }
    free(Pd);
    return status;
}

/* P x = b through the factors (Appendix B.1):
 *   ForwardSolve  z_i = b_i - sum over children j of L_{i,j} z_j   (children first)
 *   DiagSolve     y_i = D_ii^{-1} z_i                               (3x3 Cholesky solve)
 *   BackwardSolve x_i = y_i - L_{p(i),i}^T x_{p(i)}                 (parents first) */
int orc_tree_solve(int64_t n, const int32_t *parent, const int32_t *order,
                   const int32_t *child_ptr, const int32_t *child,
                   const double *D, const double *L, const double *b, double *x)
{
    double *z = malloc((size_t)(3 * n + 1) * sizeof(double));
    if (!z) return ORC_ENOMEM;
    for (int64_t q = 0; q < n; q++) {
        int32_t i = order[q];
        double s[3] = {b[3 * (int64_t)i], b[3 * (int64_t)i + 1], b[3 * (int64_t)i + 2]};
        for (int32_t c = child_ptr[i]; c < child_ptr[i + 1]; c++) {
            int32_t j = child[c];
            const double *Lij = &L[9 * (int64_t)j];
            const double *zj = &z[3 * (int64_t)j];
            for (int a = 0; a < 3; a++)
                s[a] = s[a] - (Lij[3 * a + 0] * zj[0] + Lij[3 * a + 1] * zj[1] + Lij[3 * a + 2] * zj[2]);
        }
        z[3 * (int64_t)i] = s[0]; z[3 * (int64_t)i + 1] = s[1]; z[3 * (int64_t)i + 2] = s[2];
    }
    for (int64_t i = 0; i < n; i++) {
        double C[9];
        if (chol3(&D[9 * i], C) != ORC_OK) { free(z); return ORC_ENOTSPD; }
        chol3_solve(C, &z[3 * i], &x[3 * i]);
    }
    for (int64_t q = n - 1; q >= 0; q--) {
        int32_t i = order[q];
        int32_t p = parent[i];
        if (p < 0) continue;
        const double *Lpi = &L[9 * (int64_t)i];
        const double *xp = &x[3 * (int64_t)p];
        for (int a = 0; a < 3; a++)
            x[3 * (int64_t)i + a] = x[3 * (int64_t)i + a] - (Lpi[0 * 3 + a] * xp[0] + Lpi[1 * 3 + a] * xp[1] + Lpi[2 * 3 + a] * xp[2]);
    }
    free(z);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Section 1.1: preconditioned conjugate gradients.                          */
/* ------------------------------------------------------------------------ */

enum { ORC_PREC_NONE = 0, ORC_PREC_JACOBI = 1, ORC_PREC_TREE = 2 };

typedef struct {
    int kind;
    int64_t n;
    /* block Jacobi: the diagonal blocks of Gamma */
    const int32_t *rowptr, *bcol; const double *val;
    /* tree */
    const int32_t *parent, *order, *child_ptr, *child; const double *D, *L;
} orc_prec;

static int prec_apply(const orc_prec *M, const double *r, double *z)
{
    int64_t n = M->n;
    if (M->kind == ORC_PREC_NONE) { memcpy(z, r, (size_t)(3 * n) * sizeof(double)); return ORC_OK; }
    if (M->kind == ORC_PREC_JACOBI) {
        for (int64_t i = 0; i < n; i++) {
            const double *B = NULL;
            for (int32_t k = M->rowptr[i]; k < M->rowptr[i + 1]; k++)
                if (M->bcol[k] == i) B = &M->val[9 * (int64_t)k];
            double C[9];
            if (!B || chol3(B, C) != ORC_OK) return ORC_ENOTSPD;
            chol3_solve(C, &r[3 * i], &z[3 * i]);
        }
        return ORC_OK;
    }
    return orc_tree_solve(n, M->parent, M->order, M->child_ptr, M->child, M->D, M->L, r, z);
}

static double dot(int64_t len, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t k = 0; k < len; k++) s = s + a[k] * b[k];
    return s;
}

/* Left-preconditioned CG (Saad, Iterative Methods, Alg. 9.1), the equivalent
 * of the split form E^T Gamma E x^ = E^T F of Section 1.1 with H = E E^T = M^{-1}:
 *   r = F - Gamma x0, z = M^{-1} r, p = z, rho = r.z
 *   loop: q = Gamma p; alpha = rho/(p.q); x += alpha p; r -= alpha q; k++
 *         stop if ||r||/||F|| <= tol  (or after fixed_iters iterations)
 *         z = M^{-1} r; rho' = r.z; p = z + (rho'/rho) p
 * info_i[0] = iterations; info_d[0] = recurrence relres, info_d[1] = true relres. */
int orc_pcg(int64_t n, const int32_t *rowptr, const int32_t *bcol, const double *val,
            int prec_kind,
            const int32_t *parent, const int32_t *order, const int32_t *child_ptr, const int32_t *child,
            const double *Dt, const double *Lt,
            const double *F, double *x, int use_x0, double tol, int max_iter, int fixed_iters,
            int32_t *info_i, double *info_d)
{
    int64_t len = 3 * n;
    orc_prec M = {prec_kind, n, rowptr, bcol, val, parent, order, child_ptr, child, Dt, Lt};
    double *r = malloc((size_t)(len + 1) * sizeof(double));
    double *z = malloc((size_t)(len + 1) * sizeof(double));
    double *p = malloc((size_t)(len + 1) * sizeof(double));
    double *q = malloc((size_t)(len + 1) * sizeof(double));
    int status = ORC_OK, k = 0;
    double relres = 0.0;
    if (!r || !z || !p || !q) { status = ORC_ENOMEM; goto done; }
    for (int64_t t = 0; t < len; t++)
        if (!isfinite(F[t]) || (use_x0 && !isfinite(x[t]))) { status = ORC_ENONFINITE; goto done; }
    if (!use_x0) for (int64_t t = 0; t < len; t++) x[t] = 0.0;
    double nF = sqrt(dot(len, F, F));
    if (nF == 0.0) {
        for (int64_t t = 0; t < len; t++) x[t] = 0.0;
        goto done;
    }
    orc_spmv(n, rowptr, bcol, val, x, q);
    for (int64_t t = 0; t < len; t++) r[t] = F[t] - q[t];
    relres = sqrt(dot(len, r, r)) / nF;
    if (fixed_iters <= 0 && relres <= tol) goto done;
    if ((status = prec_apply(&M, r, z)) != ORC_OK) goto done;
    for (int64_t t = 0; t < len; t++) p[t] = z[t];
    double rho = dot(len, r, z);
    for (;;) {
        if (fixed_iters > 0 ? k >= fixed_iters : k >= max_iter) {
            if (fixed_iters <= 0) status = ORC_ENOCONV;
            break;
        }
        orc_spmv(n, rowptr, bcol, val, p, q);
        double pq = dot(len, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_EBREAKDOWN; break; }
        double alpha = rho / pq;
        for (int64_t t = 0; t < len; t++) x[t] = x[t] + alpha * p[t];
        for (int64_t t = 0; t < len; t++) r[t] = r[t] - alpha * q[t];
        k++;
        relres = sqrt(dot(len, r, r)) / nF;
        if (!isfinite(relres)) { status = ORC_ENONFINITE; break; }
        if (fixed_iters <= 0 && relres <= tol) break;
        if (fixed_iters > 0 && k >= fixed_iters) break;
        if ((status = prec_apply(&M, r, z)) != ORC_OK) break;
        double rho_new = dot(len, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t t = 0; t < len; t++) p[t] = z[t] + beta * p[t];
    }
done:
    if (info_i) info_i[0] = k;
    if (info_d) {
        info_d[0] = relres;
        info_d[1] = 0.0;
        if (r && q && status != ORC_ENOMEM) {
            double nF2 = sqrt(dot(len, F, F));
            orc_spmv(n, rowptr, bcol, val, x, q);
            for (int64_t t = 0; t < len; t++) r[t] = F[t] - q[t];
            info_d[1] = nF2 > 0.0 ? sqrt(dot(len, r, r)) / nF2 : 0.0;
        }
    }
    free(r); free(z); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Stopping on the energy-norm error (Section 5 monitors CG with Gauss-Radau */
/* error estimates; Section 4's lower eigenvalue bound supplies their mu).   */
/* ------------------------------------------------------------------------ */

/* PCG from x0 = 0 as orc_pcg, stopped when an upper bound of the relative
 * energy-norm error ||x - x_k||_G / ||x||_G falls to tol.
 *   rho_k = r_k' z_k, alpha_k = rho_k / p_k' G p_k, beta_{k+1} = rho_{k+1} / rho_k.
 *   eps_k = ||x - x_k||_G^2 drops by alpha_k rho_k in step k, so with x0 = 0
 *   ||x||_G^2 = S_k + eps_k, S_k = sum_{j<k} alpha_j rho_j.
 *   Gauss-Radau quadrature with a prescribed node mu, 0 < mu <= lambda_min of
 *   P^{-1} G, bounds eps_k <= phi_k rho_k, phi_0 = 1 / mu,
 *   phi_{k+1} = (phi_k - alpha_k) / (mu (phi_k - alpha_k) + beta_{k+1}).
 *   As e / (S + e) grows with e, the relative error squared is at most
 *   phi_k rho_k / (S_k + phi_k rho_k); the solve stops at the first k where
 *   that is <= tol^2 (k = 0 included: F = 0 gives x = 0).
 * hist (may be NULL): 2 (max_iter + 1) doubles, S_k and phi_k rho_k for
 * k = 0..iters.  info_i[0] = iterations; info_d[0] = the final bound of the
 * relative error, info_d[1] = the true relative residual. */
int orc_pcg_gr(int64_t n, const int32_t *rowptr, const int32_t *bcol, const double *val, int prec_kind,
               const int32_t *parent, const int32_t *order, const int32_t *child_ptr, const int32_t *child,
               const double *Dt, const double *Lt, const double *F, double *x, double tol, double mu,
               int max_iter, int32_t *info_i, double *info_d, double *hist)
{
    int64_t len = 3 * n;
    orc_prec M = {prec_kind, n, rowptr, bcol, val, parent, order, child_ptr, child, Dt, Lt};
    double *r = calloc((size_t)(len + 1), sizeof(double));
    double *z = malloc((size_t)(len + 1) * sizeof(double));
    double *p = malloc((size_t)(len + 1) * sizeof(double));
    double *q = malloc((size_t)(len + 1) * sizeof(double));
    int status = ORC_OK, k = 0;
    double rel = 0.0;
    if (!r || !z || !p || !q) { status = ORC_ENOMEM; goto done; }
    if (!(mu > 0.0)) { status = ORC_EINVAL; goto done; }
    if (len == 0) goto done;
    for (int64_t t = 0; t < len; t++) {
        if (!isfinite(F[t])) { status = ORC_ENONFINITE; goto done; }
        x[t] = 0.0;
        r[t] = F[t];
    }
    if ((status = prec_apply(&M, r, z)) != ORC_OK) goto done;
    for (int64_t t = 0; t < len; t++) p[t] = z[t];
    double rho = dot(len, r, z), S = 0.0, phi = 1.0 / mu;
    for (;;) {
        const double bound = phi * rho;
        rel = S + bound > 0.0 ? sqrt(bound / (S + bound)) : 0.0;
        if (hist) {
            hist[2 * k] = S;
            hist[2 * k + 1] = bound;
        }
        if (rel <= tol) break;
        if (k >= max_iter) { status = ORC_ENOCONV; break; }
        orc_spmv(n, rowptr, bcol, val, p, q);
        double pq = dot(len, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_EBREAKDOWN; break; }
        double alpha = rho / pq;
        for (int64_t t = 0; t < len; t++) x[t] = x[t] + alpha * p[t];
        for (int64_t t = 0; t < len; t++) r[t] = r[t] - alpha * q[t];
        k++;
        if ((status = prec_apply(&M, r, z)) != ORC_OK) break;
        double rho_new = dot(len, r, z);
        if (!isfinite(rho_new)) { status = ORC_ENONFINITE; break; }
        double beta = rho_new / rho;
        S = S + alpha * rho;
        phi = (phi - alpha) / (mu * (phi - alpha) + beta);
        rho = rho_new;
        for (int64_t t = 0; t < len; t++) p[t] = z[t] + beta * p[t];
    }
done:
    if (info_i) info_i[0] = k;
    if (info_d) {
        info_d[0] = rel;
        info_d[1] = 0.0;
        if (r && q && status != ORC_ENOMEM) {
            double nF = sqrt(dot(len, F, F));
            orc_spmv(n, rowptr, bcol, val, x, q);
            for (int64_t t = 0; t < len; t++) r[t] = F[t] - q[t];
            info_d[1] = nF > 0.0 ? sqrt(dot(len, r, r)) / nF : 0.0;
        }
    }
    free(r); free(z); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Section 3.1, Vaidya's second preconditioner: the MST plus edges back      */
/* between its pieces, solved by flexible CG around an inner tree-PCG        */
/* (the nested CG with the MST as preconditioner of Sections 3 and 5).       */
/* ------------------------------------------------------------------------ */

/* Cutting the MST into pieces (a tree partition in the manner of Vaidya's
 * construction): walking the forest children first, every vertex weighs 1
 * plus the weights of its children that were not cut off; a vertex of
 * weight >= s is cut off from its parent and heads a piece.  So a piece has
 * at least s vertices unless it holds a root, and there are at most n / s
 * pieces besides those of the roots.  order: the vertices children first
 * (decreasing depth, as orc_tree_order gives them); piece[v] = the head of
 * v's piece (a cut vertex or a root). */
int orc_aug_pieces(int64_t n, const int32_t *parent, const int32_t *order, const int32_t *child_ptr,
                   const int32_t *child, int32_t s, int32_t *piece)
{
    int32_t *w = malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!w) return ORC_ENOMEM;
    for (int64_t q = 0; q < n; q++) {
        int32_t v = order[q], wv = 1;
        for (int32_t c = child_ptr[v]; c < child_ptr[v + 1]; c++)
            if (w[child[c]] < s) wv += w[child[c]];
        w[v] = wv;
    }
    for (int64_t q = n - 1; q >= 0; q--) {   /* parents first */
        int32_t v = order[q], p = parent[v];
        piece[v] = (p >= 0 && w[v] < s) ? piece[p] : v;
    }
    free(w);
    return ORC_OK;
}

typedef struct {
    int32_t a, b, e;
    double w;
} pair_edge;

static int cmp_pair_edge(const void *pa, const void *pb)
{
    const pair_edge *x = pa, *y = pb;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    if (x->w != y->w) return x->w > y->w ? -1 : 1;   /* heavier first */
    return (x->e > y->e) - (x->e < y->e);             /* then the smaller id */
}

/* For every pair of pieces joined by a contact, the heaviest such contact
 * (ties: the smaller edge id): added[e] = 1 for the chosen edges. */
int orc_aug_edges(int64_t m, const int32_t *ei, const int32_t *ej, const double *w, const int32_t *piece,
                  int32_t *added)
{
    pair_edge *c = malloc((size_t)(m + 1) * sizeof(pair_edge));
    if (!c) return ORC_ENOMEM;
    int64_t k = 0;
    for (int64_t e = 0; e < m; e++) {
        added[e] = 0;
        int32_t a = piece[ei[e]], b = piece[ej[e]];
        if (a == b) continue;
        c[k].a = a < b ? a : b;
        c[k].b = a < b ? b : a;
        c[k].e = (int32_t)e;
        c[k].w = w[e];
        k++;
    }
    qsort(c, (size_t)k, sizeof(pair_edge), cmp_pair_edge);
    for (int64_t t = 0; t < k; t++)
        if (t == 0 || c[t].a != c[t - 1].a || c[t].b != c[t - 1].b) added[c[t].e] = 1;
    free(c);
    return ORC_OK;
}

/* Flexible CG (Notay 2000, one direction kept) on Gamma x = F with a
 * preconditioner that is itself an iteration: z = an approximate solution of
 * P' z = r by tree-PCG on P' (the block Laplacian of the augmented MST, given
 * as its BSR matrix) from zero to relative residual inner_tol.  Steps:
 *   r = F - Gamma x, z = inner(r), p = z;
 *   repeat: q = Gamma p, alpha = (p.r)/(p.q), x += alpha p, r -= alpha q,
 *           stop if ||r||/||F|| <= tol, z = inner(r), beta = -(z.q)/(p.q),
 *           p = z + beta p.
 * info_i[0] = outer iterations, info_i[1] = inner iterations in all;
 * info_d[0] = recurrence relres, info_d[1] = true relres. */
int orc_fcg(int64_t n, const int32_t *rowptr, const int32_t *bcol, const double *val, const int32_t *prow,
            const int32_t *pcol, const double *pval, const int32_t *parent, const int32_t *order,
            const int32_t *child_ptr, const int32_t *child, const double *Dt, const double *Lt, const double *F,
            double *x, int use_x0, double tol, double inner_tol, int max_iter, int max_inner, int32_t *info_i,
            double *info_d)
{
    int64_t len = 3 * n;
    double *r = malloc((size_t)(len + 1) * sizeof(double));
    double *z = malloc((size_t)(len + 1) * sizeof(double));
    double *p = malloc((size_t)(len + 1) * sizeof(double));
    double *q = malloc((size_t)(len + 1) * sizeof(double));
    int status = ORC_OK, k = 0, inner_total = 0;
    double relres = 0.0;
    if (!r || !z || !p || !q) { status = ORC_ENOMEM; goto done; }
    if (!use_x0) for (int64_t t = 0; t < len; t++) x[t] = 0.0;
    orc_spmv(n, rowptr, bcol, val, x, q);
    for (int64_t t = 0; t < len; t++) r[t] = F[t] - q[t];
    double nF = sqrt(dot(len, F, F));
    if (nF == 0.0) { for (int64_t t = 0; t < len; t++) x[t] = 0.0; goto done; }
    relres = sqrt(dot(len, r, r)) / nF;
    if (relres <= tol) goto done;
    int32_t ii[1];
    double dd[2];
#define INNER()                                                                                          \
    do {                                                                                                 \
        int s_ = orc_pcg(n, prow, pcol, pval, ORC_PREC_TREE, parent, order, child_ptr, child, Dt, Lt, r, z, \
                         0, inner_tol, max_inner, 0, ii, dd);                                            \
        inner_total += ii[0];                                                                            \
        if (s_ != ORC_OK && s_ != ORC_ENOCONV) { status = s_; goto done; }                               \
    } while (0)
    INNER();
    for (int64_t t = 0; t < len; t++) p[t] = z[t];
    while (k < max_iter) {
        orc_spmv(n, rowptr, bcol, val, p, q);
        double pq = dot(len, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_EBREAKDOWN; break; }
        double alpha = dot(len, p, r) / pq;
        for (int64_t t = 0; t < len; t++) x[t] = x[t] + alpha * p[t];
        for (int64_t t = 0; t < len; t++) r[t] = r[t] - alpha * q[t];
        k++;
        relres = sqrt(dot(len, r, r)) / nF;
        if (relres <= tol) break;
        INNER();
        double beta = -dot(len, z, q) / pq;
        for (int64_t t = 0; t < len; t++) p[t] = z[t] + beta * p[t];
    }
#undef INNER
    if (status == ORC_OK && k >= max_iter && relres > tol) status = ORC_ENOCONV;
done:
    if (info_i) { info_i[0] = k; info_i[1] = inner_total; }
    if (info_d) {
        info_d[0] = relres;
        info_d[1] = 0.0;
        if (r && q && status != ORC_ENOMEM) {
            double nF2 = sqrt(dot(len, F, F));
            orc_spmv(n, rowptr, bcol, val, x, q);
            for (int64_t t = 0; t < len; t++) r[t] = F[t] - q[t];
            info_d[1] = nF2 > 0.0 ? sqrt(dot(len, r, r)) / nF2 : 0.0;
        }
    }
    free(r); free(z); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Mixed precision: FP32 inner tree-PCG inside FP64 iterative refinement.     */
/* ------------------------------------------------------------------------ */

/* 3x3 inverse of a symmetric positive definite block through its Cholesky
 * factor (columns of the inverse = solves against unit vectors). */
static int inv3_spd(const double D[9], double Di[9])
{
    double C[9];
    if (chol3(D, C) != ORC_OK) return ORC_ENOTSPD;
    for (int c = 0; c < 3; c++) {
        double e[3] = {0.0, 0.0, 0.0}, x[3];
        e[c] = 1.0;
        chol3_solve(C, e, x);
        for (int r = 0; r < 3; r++) Di[3 * r + c] = x[r];
    }
    return ORC_OK;
}

/* The tree solve of Appendix B.1 in FP32: ForwardSolve, DiagSolve and
 * BackwardSolve as orc_tree_solve does them, with FP32 storage and FP32
 * arithmetic; the factor is given as FP32 copies (Dinvf = D^{-1} inverted in
 * FP64 and rounded, Lf = L_{p(i),i} rounded). */
static void tree_apply_f32(int64_t n, const int32_t *parent, const int32_t *order, const int32_t *child_ptr,
                           const int32_t *child, const float *Dinvf, const float *Lf, const float *src, float *dst)
{
    /* ForwardSolve: children before parents (decreasing depth) */
    for (int64_t qq = 0; qq < n; qq++) {
        int32_t i = order[qq];
        float s0 = src[3 * (int64_t)i], s1 = src[3 * (int64_t)i + 1], s2 = src[3 * (int64_t)i + 2];
        for (int32_t c = child_ptr[i]; c < child_ptr[i + 1]; c++) {
            int32_t j = child[c];
            const float *Lm = &Lf[9 * (int64_t)j];
            const float *zj = &dst[3 * (int64_t)j];
            s0 = s0 - (Lm[0] * zj[0] + Lm[1] * zj[1] + Lm[2] * zj[2]);
            s1 = s1 - (Lm[3] * zj[0] + Lm[4] * zj[1] + Lm[5] * zj[2]);
            s2 = s2 - (Lm[6] * zj[0] + Lm[7] * zj[1] + Lm[8] * zj[2]);
        }
        dst[3 * (int64_t)i] = s0; dst[3 * (int64_t)i + 1] = s1; dst[3 * (int64_t)i + 2] = s2;
    }
    /* DiagSolve: y_i = D_i^{-1} z_i */
    for (int64_t i = 0; i < n; i++) {
        const float *Di = &Dinvf[9 * i];
        float a0 = dst[3 * i], a1 = dst[3 * i + 1], a2 = dst[3 * i + 2];
        dst[3 * i] = Di[0] * a0 + Di[1] * a1 + Di[2] * a2;
        dst[3 * i + 1] = Di[3] * a0 + Di[4] * a1 + Di[5] * a2;
        dst[3 * i + 2] = Di[6] * a0 + Di[7] * a1 + Di[8] * a2;
    }
    /* BackwardSolve: parents before children, x_i = y_i - L_{p(i),i}^T x_{p(i)} */
    for (int64_t qq = n - 1; qq >= 0; qq--) {
        int32_t i = order[qq], pp = parent[i];
        if (pp < 0) continue;
        const float *Lm = &Lf[9 * (int64_t)i];
        const float *xp = &dst[3 * (int64_t)pp];
        for (int a = 0; a < 3; a++)
            dst[3 * (int64_t)i + a] = dst[3 * (int64_t)i + a] - (Lm[a] * xp[0] + Lm[3 + a] * xp[1] + Lm[6 + a] * xp[2]);
    }
}

/* y = Gamma x in FP32 storage and arithmetic (block rows as orc_spmv). */
static void spmv_f32(int64_t n, const int32_t *rowptr, const int32_t *bcol, const float *valf, const float *src,
                     float *dst)
{
    for (int64_t i = 0; i < n; i++) {
        float s[3] = {0.0f, 0.0f, 0.0f};
        for (int32_t kk = rowptr[i]; kk < rowptr[i + 1]; kk++) {
            const float *B = &valf[9 * (int64_t)kk];
            const float *xj = &src[3 * (int64_t)bcol[kk]];
            for (int a = 0; a < 3; a++)
                s[a] = s[a] + (B[3 * a] * xj[0] + B[3 * a + 1] * xj[1] + B[3 * a + 2] * xj[2]);
        }
        dst[3 * i] = s[0]; dst[3 * i + 1] = s[1]; dst[3 * i + 2] = s[2];
    }
}

/* Inner solve of one refinement step: CG on Gamma d = r with FP32 storage and
 * FP32 arithmetic for the matrix product and the tree sweeps; dot products
 * are accumulated in FP64 and the step lengths alpha, beta are FP64 numbers
 * rounded to FP32 when applied.  The tree factors are the FP64 factors
 * rounded to FP32 (pivots inverted in FP64 first). */
static int ir_inner(int64_t n, const int32_t *rowptr, const int32_t *bcol, const float *valf,
                    const int32_t *parent, const int32_t *order, const int32_t *child_ptr, const int32_t *child,
                    const float *Dinvf, const float *Lf,
                    const double *rhs, double *d, double inner_tol, int max_iter, int *iters)
{
    int64_t len = 3 * n;
    float *r = malloc((size_t)(len + 1) * sizeof(float));
    float *z = malloc((size_t)(len + 1) * sizeof(float));
    float *p = malloc((size_t)(len + 1) * sizeof(float));
    float *q = malloc((size_t)(len + 1) * sizeof(float));
    float *x = malloc((size_t)(len + 1) * sizeof(float));
    int status = ORC_OK, k = 0;
    if (!r || !z || !p || !q || !x) { status = ORC_ENOMEM; goto done; }
    double nb = 0.0;
    for (int64_t t = 0; t < len; t++) { r[t] = (float)rhs[t]; x[t] = 0.0f; nb = nb + (double)r[t] * (double)r[t]; }
    nb = sqrt(nb);
    if (nb == 0.0) goto done;
    tree_apply_f32(n, parent, order, child_ptr, child, Dinvf, Lf, r, z);
    for (int64_t t = 0; t < len; t++) p[t] = z[t];
    double rho = 0.0;
    for (int64_t t = 0; t < len; t++) rho = rho + (double)r[t] * (double)z[t];
    while (k < max_iter) {
        spmv_f32(n, rowptr, bcol, valf, p, q);
        double pq = 0.0;
        for (int64_t t = 0; t < len; t++) pq = pq + (double)p[t] * (double)q[t];
        if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_EBREAKDOWN; break; }
        float alpha = (float)(rho / pq);
        for (int64_t t = 0; t < len; t++) x[t] = x[t] + alpha * p[t];
        for (int64_t t = 0; t < len; t++) r[t] = r[t] - alpha * q[t];
        k++;
        double nr = 0.0;
        for (int64_t t = 0; t < len; t++) nr = nr + (double)r[t] * (double)r[t];
        if (sqrt(nr) / nb <= inner_tol) break;
        tree_apply_f32(n, parent, order, child_ptr, child, Dinvf, Lf, r, z);
        double rho_new = 0.0;
        for (int64_t t = 0; t < len; t++) rho_new = rho_new + (double)r[t] * (double)z[t];
        float beta = (float)(rho_new / rho);
        rho = rho_new;
        for (int64_t t = 0; t < len; t++) p[t] = z[t] + beta * p[t];
    }
done:
    if (x) for (int64_t t = 0; t < len; t++) d[t] = (double)x[t];
    *iters = k;
    free(r); free(z); free(p); free(q); free(x);
    return status;
}

/* The FP32 copies the inner solve uses: Gamma's blocks rounded, the pivots
 * inverted in FP64 and rounded, the couplings rounded. */
static int round_factor_f32(int64_t n, const double *Dt, const double *Lt, float *Dinvf, float *Lf)
{
    for (int64_t i = 0; i < n; i++) {
        double Di[9];
        if (inv3_spd(&Dt[9 * i], Di) != ORC_OK) return ORC_ENOTSPD;
        for (int t = 0; t < 9; t++) { Dinvf[9 * i + t] = (float)Di[t]; Lf[9 * i + t] = (float)Lt[9 * i + t]; }
    }
    return ORC_OK;
}

/* x = P^{-1} b by the FP32 tree solve above (b rounded to FP32 on entry, x
 * widened to FP64 on exit).  Exported so the FP32 sweeps can be pinned on
 * their own. */
int orc_tree_solve_f32(int64_t n, const int32_t *parent, const int32_t *order, const int32_t *child_ptr,
                       const int32_t *child, const double *Dt, const double *Lt, const double *b, double *x)
{
    float *Dinvf = malloc((size_t)(9 * n + 1) * sizeof(float));
    float *Lf = malloc((size_t)(9 * n + 1) * sizeof(float));
    float *bf = calloc((size_t)(3 * n + 1), sizeof(float));
    float *xf = malloc((size_t)(3 * n + 1) * sizeof(float));
    int status = ORC_OK;
    if (!Dinvf || !Lf || !bf || !xf) { status = ORC_ENOMEM; goto done; }
    if ((status = round_factor_f32(n, Dt, Lt, Dinvf, Lf)) != ORC_OK) goto done;
    for (int64_t t = 0; t < 3 * n; t++) bf[t] = (float)b[t];
    tree_apply_f32(n, parent, order, child_ptr, child, Dinvf, Lf, bf, xf);
    for (int64_t t = 0; t < 3 * n; t++) x[t] = (double)xf[t];
done:
    free(Dinvf); free(Lf); free(bf); free(xf);
    return status;
}

/* One inner FP32 solve of Gamma d = rhs to relative inner_tol (the inner
 * step of the refinement below), exported for its own pins. */
int orc_ir_inner(int64_t n, const int32_t *rowptr, const int32_t *bcol, const double *val,
                 const int32_t *parent, const int32_t *order, const int32_t *child_ptr, const int32_t *child,
                 const double *Dt, const double *Lt, const double *rhs, double *d, double inner_tol,
                 int max_iter, int32_t *iters)
{
    int64_t nnzb = rowptr[n];
    float *valf = malloc((size_t)(9 * nnzb + 1) * sizeof(float));
    float *Dinvf = malloc((size_t)(9 * n + 1) * sizeof(float));
    float *Lf = malloc((size_t)(9 * n + 1) * sizeof(float));
    int status = ORC_OK, it = 0;
    if (!valf || !Dinvf || !Lf) { status = ORC_ENOMEM; goto done; }
    for (int64_t t = 0; t < 9 * nnzb; t++) valf[t] = (float)val[t];
    if ((status = round_factor_f32(n, Dt, Lt, Dinvf, Lf)) != ORC_OK) goto done;
    status = ir_inner(n, rowptr, bcol, valf, parent, order, child_ptr, child, Dinvf, Lf, rhs, d, inner_tol,
                      max_iter, &it);
done:
    if (iters) *iters = it;
    free(valf); free(Dinvf); free(Lf);
    return status;
}

/* Iterative refinement: r = F - Gamma x (FP64); stop when ||r||/||F|| <= tol;
 * d = inner FP32 solve of Gamma d = r to relative inner_tol; x += d (FP64).
 * info_i[0] = total inner iterations, info_i[1] = outer steps;
 * info_d[0] = final FP64 relres. */
int orc_ir_solve(int64_t n, const int32_t *rowptr, const int32_t *bcol, const double *val,
                 const int32_t *parent, const int32_t *order, const int32_t *child_ptr, const int32_t *child,
                 const double *Dt, const double *Lt,
                 const double *F, double *x, double tol, double inner_tol, int max_outer, int max_inner,
                 int32_t *info_i, double *info_d)
{
    int64_t len = 3 * n;
    int64_t nnzb = rowptr[n];
    float *valf = malloc((size_t)(9 * nnzb + 1) * sizeof(float));
    float *Dinvf = malloc((size_t)(9 * n + 1) * sizeof(float));
    float *Lf = malloc((size_t)(9 * n + 1) * sizeof(float));
    double *r = malloc((size_t)(len + 1) * sizeof(double));
    double *q = malloc((size_t)(len + 1) * sizeof(double));
    double *d = malloc((size_t)(len + 1) * sizeof(double));
    int status = ORC_OK, outer = 0, inner_total = 0;
    double relres = 0.0;
    if (!valf || !Dinvf || !Lf || !r || !q || !d) { status = ORC_ENOMEM; goto done; }
    for (int64_t t = 0; t < 9 * nnzb; t++) valf[t] = (float)val[t];
    if (round_factor_f32(n, Dt, Lt, Dinvf, Lf) != ORC_OK) { status = ORC_ENOTSPD; goto done; }
    for (int64_t t = 0; t < len; t++) x[t] = 0.0;
    double nF = sqrt(dot(len, F, F));
    if (nF == 0.0) goto done;
    for (;;) {
        orc_spmv(n, rowptr, bcol, val, x, q);
        for (int64_t t = 0; t < len; t++) r[t] = F[t] - q[t];
        relres = sqrt(dot(len, r, r)) / nF;
        if (relres <= tol) break;
        if (outer >= max_outer) { status = ORC_ENOCONV; break; }
        int it = 0;
        status = ir_inner(n, rowptr, bcol, valf, parent, order, child_ptr, child, Dinvf, Lf,
                          r, d, inner_tol, max_inner, &it);
        inner_total += it;
        if (status != ORC_OK) break;
        for (int64_t t = 0; t < len; t++) x[t] = x[t] + d[t];
        outer++;
    }
done:
    if (info_i) { info_i[0] = inner_total; info_i[1] = outer; }
    if (info_d) info_d[0] = relres;
    free(valf); free(Dinvf); free(Lf); free(r); free(q); free(d);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Step 2 and Step 5 of Section 2 for the time-stepping workload.            */
/* ------------------------------------------------------------------------ */

/* Repulsive contact force plus an active (noise) force:
 *   F_i = noise_i + sum over neighbours j (ascending) of k w_ij (r_i - r_j)/d_ij,
 * with (r_i - r_j)/d_ij = -u_e when i < j and +u_e when i > j. */
void orc_forces(int64_t n, const int32_t *rowptr, const int32_t *col, const int32_t *ei,
                const int32_t *ej, const double *w, const double *u, double k_rep,
                const double *noise, double *F)
{
    int64_t m = rowptr[n] / 2;
    int32_t *first_edge = calloc((size_t)n + 1, sizeof(int32_t));
    for (int64_t e = 0; e < m; e++) first_edge[ei[e] + 1]++;
    for (int64_t i = 0; i < n; i++) first_edge[i + 1] += first_edge[i];
    orc_graph g = {n, m, (int32_t *)rowptr, (int32_t *)col, (int32_t *)ei, (int32_t *)ej,
                   (double *)w, (double *)u};
    for (int64_t i = 0; i < n; i++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            int32_t j = col[p];
            int64_t e = edge_id(&g, first_edge, (int32_t)i, j);
            double s = (i < j) ? -1.0 : 1.0;
            double mag = k_rep * w[e];
            for (int a = 0; a < 3; a++) acc[a] = acc[a] + mag * (s * u[3 * e + a]);
        }
        for (int a = 0; a < 3; a++) F[3 * i + a] = acc[a] + noise[3 * i + a];
    }
    free(first_edge);
}

/* Forward Euler (Step 5): r_i <- r_i + dt v_i. */
void orc_euler(int64_t n, double dt, const double *v, double *pos)
{
    for (int64_t t = 0; t < 3 * n; t++) pos[t] = pos[t] + dt * v[t];
}
