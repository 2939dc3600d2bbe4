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
// Work split: wave w owns the rows whose first block lies in
// [w * WAVE_BLOCKS, (w + 1) * WAVE_BLOCKS); it walks their blocks 64 at a time
// (one block per lane), multiplies against the gathered x, parks the three
// products per block in LDS, and then one lane per row adds the row's products
// in column order.  A row is never split between waves, so every row sum has
// one fixed order and the product is bitwise reproducible.
#include "sgp_internal.h"

constexpr int WAVE_GROUPS = 2;                       // 64-block groups per wave
constexpr int WAVE_BLOCKS = 64 * WAVE_GROUPS;
constexpr int SPMV_WAVES = 4;                        // waves per workgroup
constexpr int ROW_MAX = 65;                          // blocks per row at most (max_deg 64 + diagonal)
constexpr int ACC_SLOTS = WAVE_BLOCKS + ROW_MAX;     // product slots per wave

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

int bsr_prepare(sgp_ctx ctx, sgp_bsr A)
{
    int64_t nw = (A->nnzb + WAVE_BLOCKS - 1) / WAVE_BLOCKS;
    int32_t *wrow;
    SGP_TRY(ensure_t(ctx, A->wrow, nw + 2, &wrow));
    A->nwaves = nw;
    if (A->n > 0) {
        k_wave_rows<<<grid_for(nw + 1, 256), 256, 0, ctx->stream>>>((const int32_t *)A->rowptr.p, A->n, nw, wrow);
        LAUNCH_CHECK(ctx);
    }
    return SGP_OK;
}

template <class T>
__global__ __launch_bounds__(64 * SPMV_WAVES) void k_spmv_sym(const int32_t *__restrict__ rowptr,
                                                              const int32_t *__restrict__ bcol,
                                                              const T *__restrict__ val, const T *__restrict__ x,
                                                              T *__restrict__ y, const int32_t *__restrict__ wrow,
                                                              int64_t nwaves, const PcgScalars *S, double *part,
                                                              int mode)
{
    __shared__ T acc[SPMV_WAVES][3 * ACC_SLOTS];
    __shared__ double sh[64 * SPMV_WAVES];
    if (S && S->done) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t w = (int64_t)blockIdx.x * SPMV_WAVES + wv;
    int32_t r_lo = 0, r_hi = 0, kb = 0, ke = 0;
    int64_t base = w * WAVE_BLOCKS;
    if (w < nwaves) {
        r_lo = wrow[w];
        r_hi = wrow[w + 1];
        kb = rowptr[r_lo];
        ke = rowptr[r_hi];
    }
    T *a = acc[wv];
    for (int64_t c = base; c < ke; c += 64) {
        const int64_t k = c + lane;
        if (k >= kb && k < ke) {
            const T *g = val + (c >> 6) * 384 + lane;
            const T b00 = g[0], b01 = g[64], b02 = g[128], b11 = g[192], b12 = g[256], b22 = g[320];
            const int64_t j = bcol[k];
            const T x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
            const int s = (int)(k - base);
            a[3 * s] = b00 * x0 + b01 * x1 + b02 * x2;
            a[3 * s + 1] = b01 * x0 + b11 * x1 + b12 * x2;
            a[3 * s + 2] = b02 * x0 + b12 * x1 + b22 * x2;
        }
    }
    __syncthreads();
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
        // fixed-order workgroup sum of the p.q shares
        sh[threadIdx.x] = d;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
    }
}

int spmv_blocks(sgp_bsr A) { return (int)((A->nwaves + SPMV_WAVES - 1) / SPMV_WAVES); }

int spmv_f64(sgp_ctx ctx, sgp_bsr A, const double *x, double *y, const PcgScalars *S, double *part, int mode)
{
    if (A->nwaves == 0) return SGP_OK;
    k_spmv_sym<double><<<spmv_blocks(A), 64 * SPMV_WAVES, 0, ctx->stream>>>(
        (const int32_t *)A->rowptr.p, (const int32_t *)A->bcol.p, (const double *)A->val.p, x, y,
        (const int32_t *)A->wrow.p, A->nwaves, S, part, mode);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

int spmv_f32(sgp_ctx ctx, sgp_bsr A, const float *x, float *y, const PcgScalars *S, double *part, int mode)
{
    if (A->nwaves == 0) return SGP_OK;
    k_spmv_sym<float><<<spmv_blocks(A), 64 * SPMV_WAVES, 0, ctx->stream>>>(
        (const int32_t *)A->rowptr.p, (const int32_t *)A->bcol.p, (const float *)A->val32.p, x, y,
        (const int32_t *)A->wrow.p, A->nwaves, S, part, mode);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

extern "C" int sgp_spmv(sgp_ctx ctx, sgp_bsr A, const double *x, double *y)
{
    if (!ctx || !A || (A->n > 0 && (!x || !y))) return set_err(ctx, SGP_EINVAL, "spmv: bad arguments");
    if (A->n == 0) return SGP_OK;
    return spmv_f64(ctx, A, x, y, nullptr, nullptr, 0);
}
