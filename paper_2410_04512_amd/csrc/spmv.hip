// The block-CSR product q = Gamma p that dominates every CG iteration.
//
// Storage (chosen for gfx950's 64-wide waves): every block of Gamma is
// symmetric -- W_e = w (g_par u u^T + g_perp (I - u u^T)) is, and so are the
// diagonal sums -- so a block is kept as its 6 distinct entries
// (00, 01, 02, 11, 12, 22).  Blocks are numbered as in block CSR (row by row,
// columns ascending) and laid out in groups of 64: entry t of block k lives at
//     val[(k / 64) * 6 * 64 + t * 64 + k % 64],
// so the 64 lanes of a wave that take 64 consecutive blocks read each entry
// with one fully coalesced 512-byte load (256 bytes in FP32).
//
// Work split (workgroups in XCD-contiguous order, see xcd_block): wave w owns
// the rows whose first block lies in
// [w * WAVE_BLOCKS, (w + 1) * WAVE_BLOCKS); it walks their blocks 64 at a time
// (one block per lane), multiplies against the gathered x, parks the three
// products per block in LDS, and then one lane per row adds the row's products
// in storage order.  A row is never split between waves, so every row sum has
// one fixed order and the product is bitwise reproducible.
//
// Edge form (the default for the CG): the same product from the contacts
// themselves, q_i = D_i p_i - sum_j W_ij p_j with
// W_ij p = w (g_perp p + (g_par - g_perp) (u . p) u) (eq. cell_cell_friction),
// so an off-diagonal entry costs its (w, u) and column (36 bytes) instead of a
// 6-entry block and column (52 bytes); the diagonal blocks D_i sit in their
// own 64-row groups.  Same work split and fixed row-sum order as above; the
// rows' first entries decide the wave (one extra wave owns trailing rows
// without entries).
#include "sgp_internal.h"

#include <hip/hip_ext.h>

constexpr int WAVE_GROUPS = 2;                       // 64-block groups per wave
constexpr int WAVE_BLOCKS = 64 * WAVE_GROUPS;
constexpr int ROW_MAX = 65;                          // blocks per row at most (max_deg 64 + diagonal)
constexpr int ACC_SLOTS = WAVE_BLOCKS + ROW_MAX;     // product slots per wave
constexpr int EDGE_GROUPS = 5;                       // 64-entry groups per wave, edge form
constexpr int EDGE_BLOCKS = 64 * EDGE_GROUPS;
constexpr int EDGE_SLOTS = EDGE_BLOCKS + ROW_MAX;

// first row of every wave: wrow[w] = first row whose first block is >= w * WAVE_BLOCKS
__global__ void k_wave_rows(const int32_t *rowptr, int64_t n, int64_t nwaves, int32_t *wrow)
{
    int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w > nwaves) return;
    int64_t b0 = w * WAVE_BLOCKS;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (rowptr[mid] < b0) lo = mid + 1; else hi = mid;
    }
    wrow[w] = (int32_t)lo;
}

// the same for the edge form: row i's first entry is rowptr[i] - i
__global__ void k_wave_rows_edge(const int32_t *rowptr, int64_t n, int64_t nwaves, int32_t *wrow)
{
    int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w > nwaves) return;
    int64_t b0 = w * EDGE_BLOCKS;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rowptr[mid] - mid < b0) lo = mid + 1; else hi = mid;
    }
    wrow[w] = (int32_t)lo;
}

int bsr_prepare(sgp_ctx ctx, sgp_bsr A)
{
    int64_t nw = (A->nnzb + WAVE_BLOCKS - 1) / WAVE_BLOCKS;
    int32_t *wrow;
    SGP_TRY(ensure_t(ctx, A->wrow, nw + 2, &wrow));
    A->nwaves = nw;
    const int64_t ne = A->nnzb - A->n;
    const int64_t enw = ne / EDGE_BLOCKS + 1;   // the last wave also owns rows whose first entry is ne
    int32_t *ewrow;
    SGP_TRY(ensure_t(ctx, A->ewrow, enw + 2, &ewrow));
    A->enwaves = A->n > 0 ? enw : 0;
    if (A->n > 0) {
        k_wave_rows<<<grid_for(nw + 1, 256), 256, 0, ctx->stream>>>((const int32_t *)A->rowptr.p, A->n, nw, wrow);
        k_wave_rows_edge<<<grid_for(enw + 1, 256), 256, 0, ctx->stream>>>((const int32_t *)A->rowptr.p, A->n, enw,
                                                                         ewrow);
        LAUNCH_CHECK(ctx);
    }
    return SGP_OK;
}

// one block's three products, parked in LDS
template <class T>
SGP_DEV void block_product(T *a, int s, const T *v, T x0, T x1, T x2)
{
    a[3 * s] = v[0] * x0 + v[1] * x1 + v[2] * x2;
    a[3 * s + 1] = v[1] * x0 + v[3] * x1 + v[4] * x2;
    a[3 * s + 2] = v[2] * x0 + v[4] * x1 + v[5] * x2;
}

template <class T, int SPMV_WAVES>
__global__ __launch_bounds__(64 * SPMV_WAVES) void k_spmv_sym(const int32_t *__restrict__ rowptr,
                                                              const int32_t *__restrict__ bcol,
                                                              const T *__restrict__ val, const T *__restrict__ x,
                                                              T *__restrict__ y, const int32_t *__restrict__ wrow,
                                                              int64_t nwaves, const PcgScalars *S, double *part,
                                                              int mode)
{
    __shared__ T acc[SPMV_WAVES][3 * ACC_SLOTS];
    __shared__ double sh[SPMV_WAVES];
    if (S && S->done) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);   // contiguous rows per XCD
    const int64_t w = lb * SPMV_WAVES + wv;
    int32_t r_lo = 0, r_hi = 0, kb = 0, ke = 0;
    const int64_t base = w * WAVE_BLOCKS;
    if (w < nwaves) {
        r_lo = wrow[w];
        r_hi = wrow[w + 1];
        kb = rowptr[r_lo];
        ke = rowptr[r_hi];
    }
    T *a = acc[wv];
    // the wave's two 64-block groups: all loads first, then the gathers
    const int64_t k0 = base + lane, k1 = base + 64 + lane;
    const bool on0 = k0 >= kb && k0 < ke, on1 = k1 >= kb && k1 < ke;
    T v0[6], v1[6];
    int64_t j0 = 0, j1 = 0;
    const T *g0 = val + (base >> 6) * 384 + lane;
    if (on0) {
        for (int t = 0; t < 6; t++) v0[t] = g0[64 * t];
        j0 = bcol[k0];
    }
    if (on1) {
        for (int t = 0; t < 6; t++) v1[t] = g0[384 + 64 * t];
        j1 = bcol[k1];
    }
    T x00 = 0, x01 = 0, x02 = 0, x10 = 0, x11 = 0, x12 = 0;
    if (on0) {
        x00 = x[3 * j0];
        x01 = x[3 * j0 + 1];
        x02 = x[3 * j0 + 2];
    }
    if (on1) {
        x10 = x[3 * j1];
        x11 = x[3 * j1 + 1];
        x12 = x[3 * j1 + 2];
    }
    if (on0) block_product(a, lane, v0, x00, x01, x02);
    if (on1) block_product(a, 64 + lane, v1, x10, x11, x12);
    // blocks of the last row that run past the two groups
    for (int64_t c = base + WAVE_BLOCKS; c < ke; c += 64) {
        const int64_t k = c + lane;
        if (k < ke) {
            const T *g = val + (c >> 6) * 384 + lane;
            T v[6];
            for (int t = 0; t < 6; t++) v[t] = g[64 * t];
            const int64_t j = bcol[k];
            block_product(a, (int)(k - base), v, x[3 * j], x[3 * j + 1], x[3 * j + 2]);
        }
    }
    // a wave reads back only what it wrote itself: a wave-scope LDS fence
    // suffices (the other waves of the workgroup need not wait)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    double d = 0.0;
    for (int32_t row = r_lo + lane; row < r_hi; row += 64) {
        const int s0 = (int)(rowptr[row] - base), s1 = (int)(rowptr[row + 1] - base);
        T y0 = 0, y1 = 0, y2 = 0;
        for (int s = s0; s < s1; s++) {
            y0 += a[3 * s];
            y1 += a[3 * s + 1];
            y2 += a[3 * s + 2];
        }
        y[3 * (int64_t)row] = y0;
        y[3 * (int64_t)row + 1] = y1;
        y[3 * (int64_t)row + 2] = y2;
        if (mode)
            d = d + ((double)x[3 * (int64_t)row] * (double)y0 + (double)x[3 * (int64_t)row + 1] * (double)y1 +
                     (double)x[3 * (int64_t)row + 2] * (double)y2);
    }
    if (mode) {
        // fixed-order sum of the p.q shares: butterfly within each wave, then the waves in order
        for (int o = 32; o > 0; o >>= 1) d = d + __shfl_xor(d, o, 64);
        if (lane == 0) sh[wv] = d;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = sh[0];
            for (int k = 1; k < SPMV_WAVES; k++) t = t + sh[k];
            part[lb] = t;
        }
    }
}

template <class T>
SGP_DEV void edge_product(T *a, int s, const T *e, T x0, T x1, T x2, T gpar, T gperp)
{
    edge_wp(e[0], e[1], e[2], x0, x1, x2, gpar, gperp, a[3 * s], a[3 * s + 1], a[3 * s + 2]);
}

template <class T, int SPMV_WAVES, bool EDGES>
__global__ __launch_bounds__(64 * SPMV_WAVES) void k_spmv_edge(const int32_t *__restrict__ rowptr,
                                                               const int32_t *__restrict__ ecol,
                                                               const T *__restrict__ ew, const T *__restrict__ dg,
                                                               T gpar, T gperp, const T *__restrict__ x,
                                                               T *__restrict__ y, const int32_t *__restrict__ wrow,
                                                               int64_t nwaves, int64_t ne, const PcgScalars *S,
                                                               double *part, int mode)
{
    __shared__ T acc[SPMV_WAVES][3 * EDGE_SLOTS];
    __shared__ double sh[SPMV_WAVES];
    if (S && S->done) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t w = lb * SPMV_WAVES + wv;
    const int64_t base = w * EDGE_BLOCKS;
    // Loads in two rounds, with no branch around any of them (a load's wait
    // counter is in order, and at a branch the compiler waits for everything
    // issued before it): the wave's row range (a wave past the last reads
    // the last one's and owns no rows), then (w, u) and column of every
    // entry in [base, base + EDGE_BLOCKS) (lanes past the last entry reload
    // it), whatever rows they belong to -- entries below kb belong to the
    // previous wave's last row and are loaded, not used.  Then the row
    // bounds, the first row's diagonal block, x and row pointers, and the
    // gathers.
    // EDGES = false: a product without entries (ne = 0), diagonal blocks only.
    // The entries, columns and diagonal blocks are read once per product,
    // and each load instruction takes whole cache lines of them (64-wide
    // planes), so they are loaded non-temporally: the ~340 MB they stream
    // then no longer pushes out of the caches the vectors that the next
    // kernels read (q just written, r).  Data read by a thread as several
    // short loads of one line loses from it (the line leaves before its
    // other loads come), so the sweeps' constants keep ordinary loads.
    const int64_t wc = min(w, nwaves - 1);
    int32_t r_lo = wrow[wc], r_hi = wrow[wc + 1];
    T e[EDGE_GROUPS][EDGE_PLANES], xv[EDGE_GROUPS][3];
    int64_t j[EDGE_GROUPS];
    if (EDGES) {
#pragma unroll
        for (int q = 0; q < EDGE_GROUPS; q++) {
            const int64_t k = min(base + 64 * q + lane, ne - 1);
            const T *g = ew + (k >> 6) * (64 * EDGE_PLANES) + (k & 63);
            for (int t = 0; t < EDGE_PLANES; t++) e[q][t] = __builtin_nontemporal_load(g + 64 * t);
            j[q] = __builtin_nontemporal_load(ecol + k);
        }
    }
    if (w >= nwaves) r_hi = r_lo;
    const int64_t kb = (int64_t)rowptr[r_lo] - r_lo, ke = (int64_t)rowptr[r_hi] - r_hi;
    T *a = acc[wv];
    // a lane's first row (lanes past the wave's rows reload a valid one)
    const int32_t row0 = r_lo + lane;
    T dr[6], pr[3];
    int32_t rp0, rp1;
    {
        const int32_t rc = max(min(row0, r_hi - 1), 0);
        const T *dgr = dg + ((int64_t)rc >> 6) * 384 + (rc & 63);
        for (int t = 0; t < 6; t++) dr[t] = __builtin_nontemporal_load(dgr + 64 * t);
        for (int t = 0; t < 3; t++) pr[t] = x[3 * (int64_t)rc + t];
        rp0 = rowptr[rc];
        rp1 = rowptr[rc + 1];
    }
    if (EDGES) {
#pragma unroll
        for (int q = 0; q < EDGE_GROUPS; q++)
            for (int t = 0; t < 3; t++) xv[q][t] = x[3 * j[q] + t];
        // every lane parks its products; slots of entries outside the wave's
        // rows (below kb, or past the last entry) are never read back (a
        // condition here would let the compiler sink the loads into it)
#pragma unroll
        for (int q = 0; q < EDGE_GROUPS; q++)
            edge_product(a, 64 * q + lane, e[q], xv[q][0], xv[q][1], xv[q][2], gpar, gperp);
    }
    // entries of the last row that run past the groups
    for (int64_t c = base + EDGE_BLOCKS; c < ke; c += 64) {
        const int64_t k = c + lane;
        if (k < ke) {
            const T *g = ew + (c >> 6) * (64 * EDGE_PLANES) + lane;
            T ee[EDGE_PLANES];
            for (int t = 0; t < EDGE_PLANES; t++) ee[t] = g[64 * t];
            const int64_t jj = ecol[k];
            edge_product(a, (int)(k - base), ee, x[3 * jj], x[3 * jj + 1], x[3 * jj + 2], gpar, gperp);
        }
    }
    // a wave reads back only what it wrote itself
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    double d = 0.0;
    for (int32_t row = row0; row < r_hi; row += 64) {
        if (row != row0) {
            const T *dgr = dg + ((int64_t)row >> 6) * 384 + (row & 63);
            for (int t = 0; t < 6; t++) dr[t] = __builtin_nontemporal_load(dgr + 64 * t);
            for (int t = 0; t < 3; t++) pr[t] = x[3 * (int64_t)row + t];
            rp0 = rowptr[row];
            rp1 = rowptr[row + 1];
        }
        const int s0 = (int)((int64_t)rp0 - row - base), s1 = (int)((int64_t)rp1 - (row + 1) - base);
        const T p0 = pr[0], p1 = pr[1], p2 = pr[2];
        T y0 = dr[0] * p0 + dr[1] * p1 + dr[2] * p2;
        T y1 = dr[1] * p0 + dr[3] * p1 + dr[4] * p2;
        T y2 = dr[2] * p0 + dr[4] * p1 + dr[5] * p2;
        for (int s = s0; s < s1; s++) {
            y0 -= a[3 * s];
            y1 -= a[3 * s + 1];
            y2 -= a[3 * s + 2];
        }
        y[3 * (int64_t)row] = y0;
        y[3 * (int64_t)row + 1] = y1;
        y[3 * (int64_t)row + 2] = y2;
        if (mode) d = d + ((double)p0 * (double)y0 + (double)p1 * (double)y1 + (double)p2 * (double)y2);
    }
    if (mode) {
        for (int o = 32; o > 0; o >>= 1) d = d + __shfl_xor(d, o, 64);
        if (lane == 0) sh[wv] = d;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = sh[0];
            for (int k = 1; k < SPMV_WAVES; k++) t = t + sh[k];
            part[lb] = t;
        }
    }
}

int spmv_blocks(sgp_ctx ctx, sgp_bsr A)
{
    const int64_t nw = ctx->spmv_form ? A->enwaves : A->nwaves;
    return (int)((nw + ctx->spmv_waves - 1) / ctx->spmv_waves);
}

template <class T>
static int spmv_launch(sgp_ctx ctx, sgp_bsr A, const T *val, const T *ew, const T *dg, const T *x, T *y,
                       const PcgScalars *S, double *part, int mode)
{
    const int64_t nw = ctx->spmv_form ? A->enwaves : A->nwaves;
    if (nw == 0) return SGP_OK;
    // the block form reads blocks its caller built (spmv_f64 / spmv_f32)
    if (!ctx->spmv_form && (!val || !A->have_blocks))
        return set_err(ctx, SGP_EINVAL, "spmv: the block-CSR product without its blocks");
    const int nb = spmv_blocks(ctx, A);
    hipStream_t st = ctx->stream;
    const int32_t *rp = (const int32_t *)A->rowptr.p, *bc = (const int32_t *)A->bcol.p, *wr = (const int32_t *)A->wrow.p;
    if (ctx->spmv_form) {
        const int32_t *ec = (const int32_t *)A->ecol.p, *ewr = (const int32_t *)A->ewrow.p;
        const T gp = (T)A->gpar, gq = (T)A->gperp;
        const int64_t ne = A->nnzb - A->n;
// a timed launch carries the kernel timer's events (ktimer_begin)
#define SGP_EDGE_LAUNCH(W, E)                                                                                 \
    if (ctx->kt_start) {                                                                                      \
        hipExtLaunchKernelGGL(k_spmv_edge<T, W, E>, dim3(nb), dim3(64 * W), 0, st, ctx->kt_start, ctx->kt_stop, \
                              0, rp, ec, ew, dg, gp, gq, x, y, ewr, nw, ne, S, part, mode);                   \
        ctx->kt_used = true;                                                                                  \
    } else                                                                                                    \
        k_spmv_edge<T, W, E><<<nb, 64 * W, 0, st>>>(rp, ec, ew, dg, gp, gq, x, y, ewr, nw, ne, S, part, mode)
        switch (ctx->spmv_waves * 2 + (ne > 0)) {
        case 4: SGP_EDGE_LAUNCH(2, false); break;
        case 5: SGP_EDGE_LAUNCH(2, true); break;
        case 8: SGP_EDGE_LAUNCH(4, false); break;
        case 9: SGP_EDGE_LAUNCH(4, true); break;
        case 16: SGP_EDGE_LAUNCH(8, false); break;
        case 17: SGP_EDGE_LAUNCH(8, true); break;
        default: return set_err(ctx, SGP_EINVAL, "spmv: unsupported waves per workgroup %d", ctx->spmv_waves);
        }
#undef SGP_EDGE_LAUNCH
    } else {
#define SGP_SYM_LAUNCH(W)                                                                                     \
    if (ctx->kt_start) {                                                                                      \
        hipExtLaunchKernelGGL(k_spmv_sym<T, W>, dim3(nb), dim3(64 * W), 0, st, ctx->kt_start, ctx->kt_stop, 0,  \
                              rp, bc, val, x, y, wr, nw, S, part, mode);                                      \
        ctx->kt_used = true;                                                                                  \
    } else                                                                                                    \
        k_spmv_sym<T, W><<<nb, 64 * W, 0, st>>>(rp, bc, val, x, y, wr, nw, S, part, mode)
        switch (ctx->spmv_waves) {
        case 2: SGP_SYM_LAUNCH(2); break;
        case 4: SGP_SYM_LAUNCH(4); break;
        case 8: SGP_SYM_LAUNCH(8); break;
        default: return set_err(ctx, SGP_EINVAL, "spmv: unsupported waves per workgroup %d", ctx->spmv_waves);
        }
#undef SGP_SYM_LAUNCH
    }
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

int spmv_f64(sgp_ctx ctx, sgp_bsr A, const double *x, double *y, const PcgScalars *S, double *part, int mode)
{
    // the blocks are assembled on first use: before their pointer is taken
    if (!ctx->spmv_form && A->n > 0) SGP_TRY(bsr_blocks(ctx, A));
    return spmv_launch<double>(ctx, A, (const double *)A->val.p, (const double *)A->ew.p, (const double *)A->dg.p,
                               x, y, S, part, mode);
}

int spmv_f32(sgp_ctx ctx, sgp_bsr A, const float *x, float *y, const PcgScalars *S, double *part, int mode)
{
    // the FP32 copies (and the blocks they round) before their pointers are taken
    if (A->n > 0) SGP_TRY(bsr_make32(ctx, A));
    return spmv_launch<float>(ctx, A, (const float *)A->val32.p, (const float *)A->ew32.p, (const float *)A->dg32.p,
                              x, y, S, part, mode);
}

// caller's numbering in and out; the product runs in the internal order
extern "C" int sgp_spmv(sgp_ctx ctx, sgp_bsr A, const double *x, double *y)
{
    if (!ctx || !A || (A->n > 0 && (!x || !y))) return set_err(ctx, SGP_EINVAL, "spmv: bad arguments");
    const int64_t n = A->n;
    if (n == 0) return SGP_OK;
    double *xi, *yi;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP0], 3 * n + 3, &xi));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP1], 3 * n + 3, &yi));
    const int32_t *perm = (const int32_t *)A->perm.p;
    SGP_TRY(permute_rows(ctx, perm, x, xi, n, 0));
    SGP_TRY(spmv_f64(ctx, A, xi, yi, nullptr, nullptr, 0));
    return permute_rows(ctx, perm, yi, y, n, 1);
}
