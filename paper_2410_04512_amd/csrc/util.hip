// Integer primitives of libsgp: prefix sums, a stable LSD radix sort, fills,
// plus the context's buffer and error plumbing.  All integer work, hence
// deterministic; no floating-point atomics anywhere.
#include "sgp_internal.h"

#include <atomic>

#include <algorithm>
#include <cstring>

uint64_t next_graph_version()
{
    static std::atomic<uint64_t> counter{0};
    return ++counter;
}

int set_err(sgp_ctx ctx, int code, const char *fmt, ...)
{
    if (!ctx) return code;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
    return code;
}

int ensure(sgp_ctx ctx, DevBuf &b, size_t bytes)
{
    if (bytes <= b.bytes && b.p) return SGP_OK;
    if (ctx && ctx->plan_mode == PLAN_CAPTURE)   // the recorded run sized every buffer of the step
        return set_err(ctx, SGP_EINVAL, "step capture: a buffer would grow (%zu bytes)", bytes);
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        if (e != hipSuccess) return set_err(ctx, SGP_EHIP, "hipFree: %s", hipGetErrorString(e));
    }
    size_t want = std::max<size_t>(bytes + bytes / 8, 256);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return set_err(ctx, SGP_ENOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    }
    b.bytes = want;
    return SGP_OK;
}

void release(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

// flag = 1 if the live bytes differ from the recorded ones
__global__ void k_plan_check(const uint8_t *live, const uint8_t *rec, int64_t bytes, int32_t *flag)
{
    int differ = 0;
    for (int64_t t = threadIdx.x; t < bytes; t += blockDim.x) differ |= live[t] != rec[t];
    if (__syncthreads_or(differ) && threadIdx.x == 0) *flag = 1;
}

static int plan_entry(sgp_ctx ctx, size_t bytes, uint8_t kind, size_t &off)
{
    StepPlan &P = *ctx->plan;
    if (P.pos >= P.len.size() || P.len[P.pos] != bytes || P.kind[P.pos] != kind)
        return set_err(ctx, SGP_EINVAL, "step capture: the host read %zu bytes where the recorded run read %zu",
                       bytes, P.pos < P.len.size() ? P.len[P.pos] : (size_t)0);
    off = P.off[P.pos++];
    return SGP_OK;
}

static void plan_append(sgp_ctx ctx, const void *host, size_t bytes, uint8_t kind)
{
    StepPlan &P = *ctx->plan;
    P.off.push_back(P.bytes.size());
    P.len.push_back(bytes);
    P.kind.push_back(kind);
    P.bytes.insert(P.bytes.end(), (const uint8_t *)host, (const uint8_t *)host + bytes);
}

int readback(sgp_ctx ctx, void *host, const void *dev, size_t bytes)
{
    if (ctx->plan_mode == PLAN_CAPTURE) {
        size_t off;
        SGP_TRY(plan_entry(ctx, bytes, 0, off));
        memcpy(host, ctx->plan->bytes.data() + off, bytes);
        k_plan_check<<<1, 256, 0, ctx->stream>>>((const uint8_t *)dev, (const uint8_t *)ctx->plan->arena.p + off,
                                                 (int64_t)bytes, (int32_t *)ctx->plan->flag.p);
        LAUNCH_CHECK(ctx);
        return SGP_OK;
    }
    HIP_TRY(ctx, hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->plan_mode == PLAN_RECORD) plan_append(ctx, host, bytes, 0);
    return SGP_OK;
}

int upload(sgp_ctx ctx, void *dev, const void *host, size_t bytes)
{
    if (bytes == 0) return SGP_OK;
    if (ctx->plan_mode == PLAN_CAPTURE) {
        size_t off;
        SGP_TRY(plan_entry(ctx, bytes, 1, off));
        if (memcmp(host, ctx->plan->bytes.data() + off, bytes) != 0)
            return set_err(ctx, SGP_EINVAL, "step capture: host data differs from the recorded run");
        HIP_TRY(ctx, hipMemcpyAsync(dev, (const uint8_t *)ctx->plan->arena.p + off, bytes, hipMemcpyDeviceToDevice,
                                    ctx->stream));
        return SGP_OK;
    }
    HIP_TRY(ctx, hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, ctx->stream));
    if (ctx->plan_mode == PLAN_RECORD) plan_append(ctx, host, bytes, 1);
    return SGP_OK;
}

// ---------------------------------------------------------------- fills

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_iota(int32_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

int fill_i32(sgp_ctx ctx, int32_t *p, int32_t v, int64_t n)
{
    if (n <= 0) return SGP_OK;
    k_fill_i32<<<grid_for(n, 256), 256, 0, ctx->stream>>>(p, v, n);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}
int fill_f64(sgp_ctx ctx, double *p, double v, int64_t n)
{
    if (n <= 0) return SGP_OK;
    k_fill_f64<<<grid_for(n, 256), 256, 0, ctx->stream>>>(p, v, n);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}
int iota_i32(sgp_ctx ctx, int32_t *p, int64_t n)
{
    if (n <= 0) return SGP_OK;
    k_iota<<<grid_for(n, 256), 256, 0, ctx->stream>>>(p, n);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

// ---------------------------------------------------------------- scan

constexpr int SCAN_T = 256, SCAN_I = 8, SCAN_TILE = SCAN_T * SCAN_I;

// Exclusive scan of one value per thread over a 256-thread block.
__device__ int32_t block_exscan_256(int32_t v, int32_t *total, int32_t *sh)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t incl = v;
    for (int d = 1; d < 64; d <<= 1) {
        int32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    int32_t off = 0;
    for (int k = 0; k < w; k++) off += sh[k];
    *total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return off + incl - v;
}

__global__ void k_scan_tiles(const int32_t *in, int64_t n, int32_t *tile_sum)
{
    __shared__ int32_t sh[4];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
    int32_t s = 0;
    for (int k = 0; k < SCAN_I; k++)
        if (base + k < n) s += in[base + k];
    int32_t tot;
    block_exscan_256(s, &tot, sh);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// Exclusive scan of tile sums by one block, in place; writes the grand total.
__global__ void k_scan_tile_sums(int32_t *tile, int ntiles, int32_t *total_out)
{
    __shared__ int32_t sh[4];
    int32_t carry = 0;
    for (int base = 0; base < ntiles; base += SCAN_T) {
        int k = base + threadIdx.x;
        int32_t v = k < ntiles ? tile[k] : 0;
        int32_t tot;
        int32_t ex = block_exscan_256(v, &tot, sh);
        if (k < ntiles) tile[k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_apply(const int32_t *in, int32_t *out, int64_t n, const int32_t *tile_off)
{
    __shared__ int32_t sh[4];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
    int32_t v[SCAN_I];
    int32_t s = 0;
    for (int k = 0; k < SCAN_I; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int32_t tot;
    int32_t ex = block_exscan_256(s, &tot, sh) + tile_off[blockIdx.x];
    for (int k = 0; k < SCAN_I; k++) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
}

int scan_exclusive(sgp_ctx ctx, const int32_t *in, int32_t *out, int64_t n)
{
    int ntiles = (int)((n + SCAN_TILE - 1) / SCAN_TILE);
    if (ntiles == 0) ntiles = 1;
    int32_t *tiles;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TILES], (size_t)ntiles + 1, &tiles));
    k_scan_tiles<<<ntiles, SCAN_T, 0, ctx->stream>>>(in, n, tiles);
    k_scan_tile_sums<<<1, SCAN_T, 0, ctx->stream>>>(tiles, ntiles, out + n);
    k_scan_apply<<<ntiles, SCAN_T, 0, ctx->stream>>>(in, out, n, tiles);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

// ---------------------------------------------------------------- radix sort

constexpr int RS_T = 256, RS_I = 8, RS_TILE = RS_T * RS_I;

__global__ void k_rs_hist(const uint32_t *keys, int64_t n, int shift, int32_t *hist, int ntiles)
{
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_I; k++) {
        int64_t idx = base + (int64_t)k * RS_T + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: the tile is walked in element order, 256 elements per
// round; within a round the rank of an element among equal digits is the
// number of equal digits in lower lanes of its wave plus those of lower waves.
__global__ void k_rs_scatter(const uint32_t *kin, const int32_t *vin, uint32_t *kout, int32_t *vout,
                             int64_t n, int shift, const int32_t *offs, int ntiles)
{
    __shared__ int32_t run[256];
    __shared__ int32_t wcnt[4][256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    run[t] = offs[(int64_t)t * ntiles + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_I; k++) {
        int64_t idx = base + (int64_t)k * RS_T + t;
        bool valid = idx < n;
        uint32_t key = valid ? kin[idx] : 0u;
        int32_t val = valid ? vin[idx] : 0;
        uint32_t d = (key >> shift) & 255u;
        uint64_t mask = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            bool bit = (d >> b) & 1u;
            uint64_t bm = __ballot(bit);
            mask &= bit ? bm : ~bm;
        }
        int rank = __popcll(mask & lt);
        int cnt = __popcll(mask);
        wcnt[0][t] = 0; wcnt[1][t] = 0; wcnt[2][t] = 0; wcnt[3][t] = 0;
        __syncthreads();
        if (valid && rank == 0) wcnt[w][d] = cnt;
        __syncthreads();
        if (valid) {
            int32_t p = run[d] + rank;
            for (int q = 0; q < w; q++) p += wcnt[q][d];
            kout[p] = key;
            vout[p] = val;
        }
        __syncthreads();
        run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
        __syncthreads();
    }
}

int radix_sort_pairs(sgp_ctx ctx, uint32_t *keys, int32_t *vals, uint32_t *ktmp, int32_t *vtmp,
                     int64_t n, int key_bits)
{
    if (n <= 1) return SGP_OK;
    int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
    int32_t *hist;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_HIST], (size_t)256 * ntiles + 1, &hist));
    uint32_t *ka = keys, *kb = ktmp;
    int32_t *va = vals, *vb = vtmp;
    int passes = 0;
    for (int shift = 0; shift < key_bits; shift += 8) {
        k_rs_hist<<<ntiles, RS_T, 0, ctx->stream>>>(ka, n, shift, hist, ntiles);
        LAUNCH_CHECK(ctx);
        SGP_TRY(scan_exclusive(ctx, hist, hist, (int64_t)256 * ntiles));
        k_rs_scatter<<<ntiles, RS_T, 0, ctx->stream>>>(ka, va, kb, vb, n, shift, hist, ntiles);
        LAUNCH_CHECK(ctx);
        std::swap(ka, kb);
        std::swap(va, vb);
        passes++;
    }
    if (passes & 1) {
        HIP_TRY(ctx, hipMemcpyAsync(keys, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(vals, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream));
    }
    return SGP_OK;
}

// ---------------------------------------------------------------- permutations

// gather: dst[i] = src[idx[i]]; scatter: dst[idx[i]] = src[i] (3-vectors)
// one thread per component (3 n of them): the contiguous side is accessed
// with consecutive addresses across the wave, the permuted side in 24-byte runs
__global__ void k_permute_rows(const int32_t *idx, const double *src, double *dst, int64_t n, int scatter)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 3 * n) return;
    const int64_t i = e / 3, c = e - 3 * i;
    const int64_t j = idx[i];
    const int64_t a = scatter ? i : j, b = scatter ? j : i;
    dst[3 * b + c] = src[3 * a + c];
}

int permute_rows(sgp_ctx ctx, const int32_t *idx, const double *src, double *dst, int64_t n, int scatter)
{
    if (n <= 0) return SGP_OK;
    k_permute_rows<<<grid_for(3 * n, 256), 256, 0, ctx->stream>>>(idx, src, dst, n, scatter);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

int copy_order(sgp_ctx ctx, DevBuf &dperm, DevBuf &dinv, const DevBuf &sperm, const DevBuf &sinv, int64_t n)
{
    int32_t *a, *b;
    SGP_TRY(ensure_t(ctx, dperm, n + 1, &a));
    SGP_TRY(ensure_t(ctx, dinv, n + 1, &b));
    if (n > 0) {
        HIP_TRY(ctx, hipMemcpyAsync(a, sperm.p, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(b, sinv.p, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
    }
    return SGP_OK;
}

uint64_t next_gen()
{
    static std::atomic<uint64_t> counter{0};
    return ++counter;
}
