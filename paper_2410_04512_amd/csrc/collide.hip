// Steps 1-2 of the off-lattice step (Section 2): collision detection.
//
// Uniform cell list on the GPU: cells of side h >= 2 max R, so a touching
// pair sits in the same or an adjacent cell.  Cells are numbered per cluster
// (key = cluster * ncell + cell) so that independent clusters never meet.
//
//  1. bounding box, largest radius, finite check   (one fixed-grid reduction)
//  2. key per cell, stable radix sort by key        (cell ranges are contiguous)
//  3. one thread per sorted cell scans the 27 neighbouring cells of its own
//     cluster, keeps the contacts in a per-row slot list sorted by id
//  4. prefix sums give the CSR rows and the edge numbering (i, j), i < j
//  5. one thread per row writes its upper edges: w, u computed exactly as
//     the contact test defines them (same operation order, no FMA)
//  6. each CSR entry records the id of its edge (used by assembly and forces)
#include "sgp_internal.h"

#include <cmath>

constexpr int MAXD_LIMIT = 64;

// --------------------------------------------------------------- 1. box

__global__ void k_bbox(const double *pos, const double *R, int64_t n, double *part, double *out,
                       unsigned *ticket)
{
    __shared__ double sh[256];
    __shared__ int flag;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double rmax = 0.0, bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int a = 0; a < 3; a++) {
            double x = pos[3 * i + a];
            if (!isfinite(x)) bad = 1.0;
            lo[a] = fmin(lo[a], x);
            hi[a] = fmax(hi[a], x);
        }
        double r = R[i];
        if (!isfinite(r) || !(r >= 0.0)) bad = 2.0;
        rmax = fmax(rmax, r);
    }
    // min/max are order independent: a shared-memory tree is deterministic
    double vals[8] = {-lo[0], -lo[1], -lo[2], hi[0], hi[1], hi[2], rmax, bad};
    for (int q = 0; q < 8; q++) {
        sh[threadIdx.x] = vals[q];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) part[8 * blockIdx.x + q] = sh[0];
        __syncthreads();
    }
    if (!last_block(ticket, gridDim.x, &flag)) return;
    for (int q = 0; q < 8; q++) {
        double v = -INFINITY;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) v = fmax(v, part[8 * b + q]);
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = (q < 3) ? -sh[0] : sh[0];
        __syncthreads();
    }
}

// --------------------------------------------------------------- 2. keys

struct Grid {
    double lo[3];
    double inv_h;
    int32_t dim[3];
    int64_t ncell;   // cells per cluster
};

SGP_DEV int cell_coord(double x, double lo, double inv_h, int dim)
{
    int c = (int)floor((x - lo) * inv_h);
    return c < 0 ? 0 : (c >= dim ? dim - 1 : c);
}

__global__ void k_cell_keys(const double *pos, int64_t n, Grid g, const int32_t *inst_of,
                            uint32_t *key, int32_t *val)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cx = cell_coord(pos[3 * i + 0], g.lo[0], g.inv_h, g.dim[0]);
    int cy = cell_coord(pos[3 * i + 1], g.lo[1], g.inv_h, g.dim[1]);
    int cz = cell_coord(pos[3 * i + 2], g.lo[2], g.inv_h, g.dim[2]);
    int64_t c = ((int64_t)cz * g.dim[1] + cy) * g.dim[0] + cx;
    int64_t inst = inst_of ? inst_of[i] : 0;
    key[i] = (uint32_t)(inst * g.ncell + c);
    val[i] = (int32_t)i;
}

__global__ void k_cell_ranges(const uint32_t *key, int64_t n, int32_t *cstart, int32_t *cend)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t k = key[s];
    if (s == 0 || key[s - 1] != k) cstart[k] = (int32_t)s;
    if (s == n - 1 || key[s + 1] != k) cend[k] = (int32_t)(s + 1);
}

__global__ void k_gather_sorted(const double *pos, const double *R, const int32_t *sidx, int64_t n,
                                double4 *sp)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t i = sidx[s];
    sp[s] = make_double4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], R[i]);
}

__global__ void k_inverse(const int32_t *perm, int64_t n, int32_t *inv)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inv[perm[i]] = (int32_t)i;
}

// --------------------------------------------------------------- 3. contacts

// flags[0]: capacity overflow, flags[1]: coincident centres in contact
constexpr int NB_THREADS = 128;

__global__ __launch_bounds__(NB_THREADS) void k_neighbors(const double4 *sp, const int32_t *sidx,
                                                          const uint32_t *key, int64_t n, Grid g,
                                                          const int32_t *cstart, const int32_t *cend, int max_deg,
                                                          int32_t *slots, int32_t *deg, int32_t *upcnt,
                                                          int32_t *flags)
{
    // the thread's sorted neighbour list lives in LDS (max_deg rounded up to
    // an odd stride: the threads of a wave touch different banks): in
    // private memory its insertion stores would be vector-memory stores, and
    // every candidate load after them would wait for them
    extern __shared__ int32_t snb[];
    int32_t *nb = snb + threadIdx.x * (max_deg | 1);
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t i = sidx[s];
    const double4 me = sp[s];
    const uint32_t k = key[s];
    const int64_t inst = k / g.ncell;
    int64_t c = k - inst * g.ncell;
    const int cx = (int)(c % g.dim[0]);
    const int cy = (int)((c / g.dim[0]) % g.dim[1]);
    const int cz = (int)(c / ((int64_t)g.dim[0] * g.dim[1]));
    int cnt = 0, up = 0;
    bool overflow = false, coincident = false;
    for (int z = cz - 1; z <= cz + 1; z++) {
        if (z < 0 || z >= g.dim[2]) continue;
        for (int y = cy - 1; y <= cy + 1; y++) {
            if (y < 0 || y >= g.dim[1]) continue;
            for (int x = cx - 1; x <= cx + 1; x++) {
                if (x < 0 || x >= g.dim[0]) continue;
                int64_t cc = inst * g.ncell + ((int64_t)z * g.dim[1] + y) * g.dim[0] + x;
                int32_t b = cstart[cc], e = cend[cc];
                for (int32_t t = b; t < e; t++) {
                    if (t == s) continue;
                    double4 o = sp[t];
                    // the contact test: same expression as the definition, the
                    // pair's order does not change d (dx is only negated)
                    double dx = o.x - me.x, dy = o.y - me.y, dz = o.z - me.z;
                    double d = sqrt((dx * dx + dy * dy) + dz * dz);
                    double sr = me.w + o.w;
                    if (!(d < sr)) continue;
                    if (d == 0.0) coincident = true;
                    int32_t j = sidx[t];
                    if (cnt >= max_deg) { overflow = true; continue; }
                    // insertion into the sorted row
                    int p = cnt;
                    while (p > 0 && nb[p - 1] > j) { nb[p] = nb[p - 1]; p--; }
                    nb[p] = j;
                    cnt++;
                    if (j > i) up++;
                }
            }
        }
    }
    int32_t *row = slots + (int64_t)i * max_deg;
    for (int q = 0; q < cnt; q++) row[q] = nb[q];
    deg[i] = cnt;
    upcnt[i] = up;
    if (overflow) atomicOr(&flags[0], 1);
    if (coincident) atomicOr(&flags[1], 1);
}

// --------------------------------------------------------------- 4-6. CSR and edges

// The per-row passes below run ROW_LANES lanes per row, lane k taking the
// row's entries k, k + ROW_LANES, ...: a row's entries are independent, and
// one thread walking its row would wait for each entry's stores before the
// next entry's loads (a wave's memory counter is waited on in order).
constexpr int ROW_LANES = 16;

__global__ void k_compact_rows(const int32_t *slots, int max_deg, const int32_t *rowptr, int64_t n,
                               int32_t *col)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / ROW_LANES;
    if (i >= n) return;
    const int32_t b = rowptr[i], e = rowptr[i + 1];
    const int32_t *row = slots + i * max_deg;
    for (int32_t p = b + (int32_t)(t % ROW_LANES); p < e; p += ROW_LANES) col[p] = row[p - b];
}

// Upper edges of row i: ids eoff[i] .. eoff[i+1]-1, geometry as the contact
// test.  The row's columns ascend, so its upper entries are its last
// eoff[i+1] - eoff[i], and an upper entry's edge id is eoff[i] plus its rank
// among them.
// w of a contact: the overlap s - d, or with `hertz` the contact area of the
// Hertz model, pi R* (s - d) with R* = R_i R_j / (R_i + R_j), evaluated as
// (pi * ((R_i * R_j) / (R_i + R_j))) * (s - d)
__global__ void k_edges(const double *pos, const double *R, const int32_t *rowptr, const int32_t *col,
                        const int32_t *eoff, int64_t n, int hertz, int32_t *ei, int32_t *ej, double4 *wu, double *w)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / ROW_LANES;
    if (i >= n) return;
    const int32_t e0 = eoff[i], re = rowptr[i + 1];
    const int32_t up0 = re - (eoff[i + 1] - e0);   // first upper entry
    const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2], ri = R[i];
    for (int32_t p = up0 + (int32_t)(t % ROW_LANES); p < re; p += ROW_LANES) {
        const int64_t j = col[p];
        double dx = pos[3 * j + 0] - xi;
        double dy = pos[3 * j + 1] - yi;
        double dz = pos[3 * j + 2] - zi;
        double d = sqrt((dx * dx + dy * dy) + dz * dz);
        const double rj = R[j];
        double s = ri + rj;
        double a = s - d;
        if (hertz) a = (3.14159265358979323846 * ((ri * rj) / (ri + rj))) * a;
        const int32_t e = e0 + (p - up0);
        ei[e] = (int32_t)i;
        ej[e] = (int32_t)j;
        wu[e] = make_double4(a, dx / d, dy / d, dz / d);
        w[e] = a;
    }
}

// Edge id of every CSR entry.  Entry (i, j), j > i: its rank among row i's
// upper entries.  Entry (i, j), j < i: the edge (j, i), found by binary search
// of i in row j.
__global__ void k_entry_edges(const int32_t *rowptr, const int32_t *col, const int32_t *eoff, int64_t n,
                              int32_t *ent_edge)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / ROW_LANES;
    if (i >= n) return;
    int32_t b = rowptr[i], e = rowptr[i + 1];
    int32_t nlow_i = (e - b) - (eoff[i + 1] - eoff[i]);
    for (int32_t p = b + (int32_t)(t % ROW_LANES); p < e; p += ROW_LANES) {
        int32_t j = col[p];
        if (j > i) {
            ent_edge[p] = eoff[i] + (p - b - nlow_i);
        } else {
            int32_t lo = rowptr[j], hi = rowptr[j + 1];
            while (lo < hi) {
                int32_t mid = (lo + hi) >> 1;
                if (col[mid] < i) lo = mid + 1; else hi = mid;
            }
            int32_t nlow_j = (rowptr[j + 1] - rowptr[j]) - (eoff[j + 1] - eoff[j]);
            ent_edge[p] = eoff[j] + (lo - rowptr[j] - nlow_j);
        }
    }
}

__global__ void k_copy_count(const int32_t *src, int32_t *dst) { *dst = *src; }

__global__ void k_inst_of(const int64_t *off, int64_t n_inst, int32_t *inst_of)
{
    int64_t k = blockIdx.x;
    if (k >= n_inst) return;
    for (int64_t i = off[k] + threadIdx.x; i < off[k + 1]; i += blockDim.x) inst_of[i] = (int32_t)k;
}

static int collide_impl(sgp_ctx ctx, int64_t n, const double *pos, const double *radius, int32_t max_deg,
                        sgp_graph g, int64_t n_inst, const int64_t *h_off)
{
    if (!ctx || !g) return set_err(ctx, SGP_EINVAL, "collide: null handle");
    if (n < 0 || (n > 0 && (!pos || !radius))) return set_err(ctx, SGP_EINVAL, "collide: bad arguments");
    if (max_deg <= 0 || max_deg > MAXD_LIMIT)
        return set_err(ctx, SGP_EINVAL, "collide: max_deg must be in [1, %d]", MAXD_LIMIT);
    if (n >= (int64_t)1 << 30) return set_err(ctx, SGP_EINVAL, "collide: n too large");
    hipStream_t st = ctx->stream;
    g->n = n;
    g->version = next_graph_version();
    g->n_inst = n_inst;
    g->h_inst_off.assign(h_off, h_off + n_inst + 1);
    int32_t *rowptr;
    SGP_TRY(ensure_t(ctx, g->rowptr, n + 1, &rowptr));
    int64_t *d_off;
    SGP_TRY(ensure_t(ctx, g->inst_off, n_inst + 1, &d_off));
    SGP_TRY(upload(ctx, d_off, h_off, (n_inst + 1) * sizeof(int64_t)));
    int32_t *inst_of = nullptr;
    if (n_inst > 1) {
        SGP_TRY(ensure_t(ctx, g->inst_of, n + 1, &inst_of));
        k_inst_of<<<(unsigned)n_inst, 256, 0, st>>>(d_off, n_inst, inst_of);
        LAUNCH_CHECK(ctx);
    }
    if (n == 0) {
        g->m = 0;
        SGP_TRY(fill_i32(ctx, rowptr, 0, 1));
        return SGP_OK;
    }
    // 1. box
    double *part, *box;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PART], 8 * 256 + 16, &part));
    box = part + 8 * 256;
    k_bbox<<<256, 256, 0, st>>>(pos, radius, n, part, box, ctx->tickets);
    LAUNCH_CHECK(ctx);
    double hb[8];
    SGP_TRY(readback(ctx, hb, box, sizeof hb));
    if (hb[7] == 1.0) return set_err(ctx, SGP_ENONFINITE, "collide: non-finite position");
    if (hb[7] == 2.0) return set_err(ctx, SGP_EINVAL, "collide: negative or non-finite radius");
    Grid gr;
    double h = 2.0 * hb[6] * (1.0 + 0x1p-20);
    if (!(h > 0.0)) h = 1.0;
    gr.inv_h = 1.0 / h;
    int64_t ncell = 1;
    for (int a = 0; a < 3; a++) {
        gr.lo[a] = hb[a];
        double span = (hb[3 + a] - hb[a]) * gr.inv_h;
        int64_t d = (int64_t)floor(span) + 1;
        // a huge, sparse domain would need too many cells: coarsen uniformly
        gr.dim[a] = (int32_t)std::min<int64_t>(d, 1 << 20);
        ncell *= gr.dim[a];
    }
    int64_t budget = std::max<int64_t>(4 * n / std::max<int64_t>(n_inst, 1), 64);
    while (ncell > budget || (double)ncell * n_inst > 4.0e9) {
        // enlarge cells: still a correct cell list (side >= 2 max R)
        h *= 1.25;
        gr.inv_h = 1.0 / h;
        ncell = 1;
        for (int a = 0; a < 3; a++) {
            gr.dim[a] = (int32_t)floor((hb[3 + a] - hb[a]) * gr.inv_h) + 1;
            ncell *= gr.dim[a];
        }
    }
    gr.ncell = ncell;
    int64_t nkeys = ncell * n_inst;
    int key_bits = 1;
    while (((int64_t)1 << key_bits) < nkeys) key_bits++;
    // 2. keys + sort
    uint32_t *ka, *kb;
    int32_t *va, *vb, *cstart, *cend;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_A], n, &ka));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_B], n, &kb));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_A], n, &va));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_B], n, &vb));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP0], nkeys, &cstart));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP1], nkeys, &cend));
    k_cell_keys<<<grid_for(n, 256), 256, 0, st>>>(pos, n, gr, inst_of, ka, va);
    LAUNCH_CHECK(ctx);
    SGP_TRY(radix_sort_pairs(ctx, ka, va, kb, vb, n, key_bits));
    SGP_TRY(fill_i32(ctx, cstart, 0, nkeys));
    SGP_TRY(fill_i32(ctx, cend, 0, nkeys));
    k_cell_ranges<<<grid_for(n, 256), 256, 0, st>>>(ka, n, cstart, cend);
    double4 *sp;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP2], n, &sp));
    k_gather_sorted<<<grid_for(n, 256), 256, 0, st>>>(pos, radius, va, n, sp);
    LAUNCH_CHECK(ctx);
    // the cell-list order becomes the library's internal vertex order
    int32_t *gperm, *ginv;
    SGP_TRY(ensure_t(ctx, g->perm, n + 1, &gperm));
    SGP_TRY(ensure_t(ctx, g->inv, n + 1, &ginv));
    HIP_TRY(ctx, hipMemcpyAsync(gperm, va, n * 4, hipMemcpyDeviceToDevice, st));
    k_inverse<<<grid_for(n, 256), 256, 0, st>>>(va, n, ginv);
    LAUNCH_CHECK(ctx);
    // 3. contacts
    int32_t *slots, *deg, *upc, *flags;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_SLOTS], (size_t)n * max_deg, &slots));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_DEG], n + 1, &deg));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], n + 1, &upc));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], 4, &flags));
    SGP_TRY(fill_i32(ctx, flags, 0, 4));
    const size_t nb_lds = sizeof(int32_t) * NB_THREADS * (size_t)(max_deg | 1);
    k_neighbors<<<grid_for(n, NB_THREADS), NB_THREADS, nb_lds, st>>>(sp, va, ka, n, gr, cstart, cend, max_deg,
                                                                     slots, deg, upc, flags);
    LAUNCH_CHECK(ctx);
    // 4. rows and edge numbering
    SGP_TRY(scan_exclusive(ctx, deg, rowptr, n));
    SGP_TRY(scan_exclusive(ctx, upc, upc, n));   // upc becomes eoff [n+1]
    int32_t hs[4];
    k_copy_count<<<1, 1, 0, st>>>(upc + n, flags + 2);   // the edge count beside the two flags: one readback
    LAUNCH_CHECK(ctx);
    SGP_TRY(readback(ctx, hs, flags, 3 * sizeof(int32_t)));
    if (hs[0]) return set_err(ctx, SGP_ECAPACITY, "collide: a cell has more than max_deg=%d contacts", max_deg);
    if (hs[1]) return set_err(ctx, SGP_EINVAL, "collide: coincident centres in contact");
    int64_t m = hs[2];
    g->m = m;
    int32_t *col, *ee, *ei, *ej;
    double4 *wu;
    double *wv;
    SGP_TRY(ensure_t(ctx, g->col, 2 * m + 1, &col));
    SGP_TRY(ensure_t(ctx, g->ent_edge, 2 * m + 1, &ee));
    SGP_TRY(ensure_t(ctx, g->ei, m + 1, &ei));
    SGP_TRY(ensure_t(ctx, g->ej, m + 1, &ej));
    SGP_TRY(ensure_t(ctx, g->wu, m + 1, &wu));
    SGP_TRY(ensure_t(ctx, g->w, m + 1, &wv));
    k_compact_rows<<<grid_for(ROW_LANES * n, 256), 256, 0, st>>>(slots, max_deg, rowptr, n, col);
    k_edges<<<grid_for(ROW_LANES * n, 256), 256, 0, st>>>(pos, radius, rowptr, col, upc, n,
                                                          ctx->contact_model == SGP_CONTACT_HERTZ, ei, ej, wu, wv);
    k_entry_edges<<<grid_for(ROW_LANES * n, 256), 256, 0, st>>>(rowptr, col, upc, n, ee);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

extern "C" int sgp_collide(sgp_ctx ctx, int64_t n, const double *pos, const double *radius, int32_t max_deg,
                           sgp_graph g)
{
    int64_t off[2] = {0, n};
    phase_begin(ctx, 0);
    int s = collide_impl(ctx, n, pos, radius, max_deg, g, 1, off);
    if (s == SGP_OK) phase_end(ctx, 0);
    return s;
}

extern "C" int sgp_collide_batched(sgp_ctx ctx, int64_t n_inst, const int64_t *offsets, const double *pos,
                                   const double *radius, int32_t max_deg, sgp_graph g)
{
    if (!ctx || !offsets || n_inst <= 0) return set_err(ctx, SGP_EINVAL, "collide_batched: bad arguments");
    if (offsets[0] != 0) return set_err(ctx, SGP_EINVAL, "collide_batched: offsets[0] must be 0");
    for (int64_t k = 0; k < n_inst; k++)
        if (offsets[k + 1] < offsets[k]) return set_err(ctx, SGP_EINVAL, "collide_batched: offsets decrease");
    phase_begin(ctx, 0);
    int s = collide_impl(ctx, offsets[n_inst], pos, radius, max_deg, g, n_inst, offsets);
    if (s == SGP_OK) phase_end(ctx, 0);
    return s;
}

// --------------------------------------------------------------- clusters of the local forest
//
// Clusters for the local-MST forest (Section 6, Discussion: a spatial
// subdivision into clusters of a few hundred cells, each with a spanning tree
// of its own): the cells of every instance in the Z-order of a uniform grid,
// cut into runs of K.  Grid: cubes of side h = 2 max R (1 if all radii are
// 0), anchored at the bounding box's minimum corner (over all instances);
// cell coordinates c_a = floor((x_a - lo_a) / h); Z-order = the Morton code
// interleaving the bits of (c_x, c_y, c_z) from the lowest (x lowest), ties
// by cell id.  Cluster ids run instance by instance; an instance's last run
// may be shorter than K.

SGP_DEV uint32_t spread3(uint32_t v)
{
    uint32_t r = 0;
    for (int b = 0; b < 10; b++) r |= ((v >> b) & 1u) << (3 * b);
    return r;
}

__global__ void k_zkeys(const double *pos, int64_t n, double lox, double loy, double loz, double h, int bits,
                        const int32_t *inst_of, uint32_t *key, int32_t *val)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {lox, loy, loz};
    uint32_t m = 0;
    for (int a = 0; a < 3; a++) {
        const double c = floor((pos[3 * i + a] - lo[a]) / h);
        const uint32_t ci = c > 0.0 ? (uint32_t)c : 0u;
        m |= spread3(ci) << a;
    }
    const uint32_t inst = inst_of ? (uint32_t)inst_of[i] : 0u;
    key[i] = (inst << (3 * bits)) | m;
    val[i] = (int32_t)i;
}

// sorted position p -> cluster of its cell
__global__ void k_zclusters(int64_t n, const int32_t *sorted, const int32_t *inst_of, const int64_t *off,
                            const int32_t *cbase, int32_t K, int32_t *cluster)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t i = sorted[p];
    const int32_t k = inst_of ? inst_of[i] : 0;
    cluster[i] = cbase[k] + (int32_t)((p - off[k]) / K);
}

int forest_partition(sgp_ctx ctx, sgp_graph g, const double *pos, const double *radius, int32_t K,
                     int32_t *cluster, int64_t *n_clusters)
{
    hipStream_t st = ctx->stream;
    const int64_t n = g->n, n_inst = g->n_inst;
    *n_clusters = 0;
    if (n == 0) return SGP_OK;
    double *part, *box;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PART], 8 * 256 + 16, &part));
    box = part + 8 * 256;
    k_bbox<<<256, 256, 0, st>>>(pos, radius, n, part, box, ctx->tickets);
    LAUNCH_CHECK(ctx);
    double hb[8];
    SGP_TRY(readback(ctx, hb, box, sizeof hb));
    if (hb[7] == 1.0) return set_err(ctx, SGP_ENONFINITE, "build_forest: non-finite position");
    if (hb[7] == 2.0) return set_err(ctx, SGP_EINVAL, "build_forest: negative or non-finite radius");
    const double h = hb[6] > 0.0 ? 2.0 * hb[6] : 1.0;
    int bits = 1;
    for (int a = 0; a < 3; a++)
        while (bits < 10 && floor((hb[3 + a] - hb[a]) / h) >= (double)(1 << bits)) bits++;
    for (int a = 0; a < 3; a++)
        if (floor((hb[3 + a] - hb[a]) / h) >= (double)(1 << bits))
            return set_err(ctx, SGP_EINVAL, "build_forest: more than 1024 grid cells along an axis");
    int ibits = 0;
    while (((int64_t)1 << ibits) < n_inst) ibits++;
    if (3 * bits + ibits > 32) return set_err(ctx, SGP_EINVAL, "build_forest: Z-order keys exceed 32 bits");
    // first cluster of every instance
    std::vector<int32_t> cb(n_inst + 1, 0);
    for (int64_t k = 0; k < n_inst; k++)
        cb[k + 1] = cb[k] + (int32_t)((g->h_inst_off[k + 1] - g->h_inst_off[k] + K - 1) / K);
    int32_t *cbase;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PAIR], n_inst + 2, &cbase));
    SGP_TRY(upload(ctx, cbase, cb.data(), (n_inst + 1) * sizeof(int32_t)));
    uint32_t *ka, *kb;
    int32_t *va, *vb;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_A], n, &ka));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_B], n, &kb));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_A], n, &va));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_B], n, &vb));
    const int32_t *inst_of = n_inst > 1 ? (const int32_t *)g->inst_of.p : nullptr;
    k_zkeys<<<grid_for(n, 256), 256, 0, st>>>(pos, n, hb[0], hb[1], hb[2], h, bits, inst_of, ka, va);
    LAUNCH_CHECK(ctx);
    SGP_TRY(radix_sort_pairs(ctx, ka, va, kb, vb, n, std::max(3 * bits + ibits, 1)));
    k_zclusters<<<grid_for(n, 256), 256, 0, st>>>(n, va, inst_of, (const int64_t *)g->inst_off.p, cbase, K, cluster);
    LAUNCH_CHECK(ctx);
    *n_clusters = cb[n_inst];
    return SGP_OK;
}

extern "C" int sgp_set_contact_model(sgp_ctx ctx, int32_t model)
{
    if (!ctx) return SGP_EINVAL;
    if (model != SGP_CONTACT_OVERLAP && model != SGP_CONTACT_HERTZ)
        return set_err(ctx, SGP_EINVAL, "set_contact_model: unknown model %d", model);
    ctx->contact_model = model;
    return SGP_OK;
}

extern "C" int sgp_graph_size(sgp_graph g, int64_t *n, int64_t *m)
{
    if (!g) return SGP_EINVAL;
    if (n) *n = g->n;
    if (m) *m = g->m;
    return SGP_OK;
}

__global__ void k_split_wu(const double4 *wu, int64_t m, double *w, double *u)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    double4 v = wu[e];
    if (w) w[e] = v.x;
    if (u) {
        u[3 * e] = v.y;
        u[3 * e + 1] = v.z;
        u[3 * e + 2] = v.w;
    }
}

extern "C" int sgp_graph_export(sgp_ctx ctx, sgp_graph g, int32_t *rowptr, int32_t *col, int32_t *ei,
                                int32_t *ej, double *w, double *u)
{
    if (!ctx || !g) return set_err(ctx, SGP_EINVAL, "graph_export: null handle");
    hipStream_t st = ctx->stream;
    int64_t n = g->n, m = g->m;
    if (rowptr) HIP_TRY(ctx, hipMemcpyAsync(rowptr, g->rowptr.p, (n + 1) * 4, hipMemcpyDeviceToDevice, st));
    if (m > 0) {
        if (col) HIP_TRY(ctx, hipMemcpyAsync(col, g->col.p, 2 * m * 4, hipMemcpyDeviceToDevice, st));
        if (ei) HIP_TRY(ctx, hipMemcpyAsync(ei, g->ei.p, m * 4, hipMemcpyDeviceToDevice, st));
        if (ej) HIP_TRY(ctx, hipMemcpyAsync(ej, g->ej.p, m * 4, hipMemcpyDeviceToDevice, st));
        if (w || u) {
            k_split_wu<<<grid_for(m, 256), 256, 0, st>>>((const double4 *)g->wu.p, m, w, u);
            LAUNCH_CHECK(ctx);
        }
    }
    return SGP_OK;
}
