// Learned warm start: a message-passing network over the collision graph,
// (F, v_prev) -> v_hat, used as the CG's initial guess (CG to the same
// tolerance still decides; the previous velocity is the fallback).
//
// Network (hidden width 64, three message-passing layers; the same
// definition as the FP64 oracle):
//   x_i = [F_i/sF, v_prev,i/sV],  e_p = [w/sW, n_ij] for CSR entry p = (i, j)
//   h = relu(x W_in + b_in)
//   per layer: z_p = h_i W_a + b_m + h_j W_b + e_p W_c; m_p = relu(z_p)
//              a_i = sum over row i of m_p;  h = h + relu([h, a] W_u + b_u)
//   out = h W_out + b_out,  v_hat = sV out
// The message MLP on [h_i, h_j, e_p] is split into the node products h W_a,
// h W_b (one node-level GEMM) and the per-edge gather-add, so the dense
// contractions run on MFMA and the per-edge part stays a bandwidth-bound
// gather instead of a 2m x 132 GEMM.
//
// Precision: FP32 master weights; every GEMM takes BF16 weights and BF16
// activations with FP32 accumulation (v_mfma_f32_16x16x16_bf16); the per-edge
// arithmetic uses the BF16-rounded W_c and b_m in FP32.  All reductions (row
// sums, column sums, split-K weight gradients) have a fixed order, so a step
// is bitwise reproducible.
#include "sgp_internal.h"

#include <cmath>
#include <cstring>

namespace {

constexpr int HID = 64, NL = 3;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

SGP_DEV unsigned short f2bf(float f)
{
    unsigned int b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);   // round to nearest even
    return (unsigned short)(b >> 16);
}
SGP_DEV float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// flat parameter offsets (same order as the oracle's layout)
struct Layout {
    int64_t W_in, b_in, W_a[NL], W_b[NL], W_c[NL], b_m[NL], W_u[NL], b_u[NL], W_out, b_out, total;
};

Layout make_layout()
{
    Layout L;
    int64_t k = 0;
    L.W_in = k; k += 6 * HID;
    L.b_in = k; k += HID;
    for (int l = 0; l < NL; l++) {
        L.W_a[l] = k; k += HID * HID;
        L.W_b[l] = k; k += HID * HID;
        L.W_c[l] = k; k += 4 * HID;
        L.b_m[l] = k; k += HID;
        L.W_u[l] = k; k += 2 * HID * HID;
        L.b_u[l] = k; k += HID;
    }
    L.W_out = k; k += HID * 3;
    L.b_out = k; k += 3;
    L.total = k;
    return L;
}

// BF16 GEMM operands built from the master weights (K x N row-major, padded)
struct Packed {
    int64_t in16;           // W_in padded to 16 x 64
    int64_t ab[NL];         // [W_a | W_b]   64 x 128
    int64_t u[NL];          // W_u           128 x 64
    int64_t out16;          // W_out padded  64 x 16
    int64_t abT[NL];        // [W_a | W_b]^T 128 x 64
    int64_t uT[NL];         // W_u^T         64 x 128
    int64_t out16T;         // W_out^T pad   16 x 64
    int64_t total;
};

Packed make_packed()
{
    Packed p;
    int64_t k = 0;
    p.in16 = k; k += 16 * 64;
    for (int l = 0; l < NL; l++) { p.ab[l] = k; k += 64 * 128; }
    for (int l = 0; l < NL; l++) { p.u[l] = k; k += 128 * 64; }
    p.out16 = k; k += 64 * 16;
    for (int l = 0; l < NL; l++) { p.abT[l] = k; k += 128 * 64; }
    for (int l = 0; l < NL; l++) { p.uT[l] = k; k += 64 * 128; }
    p.out16T = k; k += 16 * 64;
    p.total = k;
    return p;
}

}   // namespace

struct sgp_mpnn_ {
    Layout L = make_layout();
    Packed PK = make_packed();
    DevBuf theta, m1, m2, grad, wbf, wrow;   // wrow: BF16-rounded master weights as FP32 (edge arithmetic)
    DevBuf act, efeat, part;
    double sF = 1, sV = 1, sW = 1;
    int64_t adam_t = 0;
    int64_t cap_n = 0, cap_e = 0;
};

namespace {

// ---------------------------------------------------------------- weight packing

__global__ void k_pack(const float *theta, Layout L, Packed P, unsigned short *wbf, float *wr)
{
    // one thread per packed element; wr receives every master weight rounded to BF16
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < L.total) wr[t] = bf2f(f2bf(theta[t]));
    if (t >= P.total) return;
    float v = 0.f;
    int64_t o = t;
    if (o < P.ab[0]) {   // in16: 16 x 64
        int r = (int)(o / 64), c = (int)(o % 64);
        v = r < 6 ? theta[L.W_in + r * 64 + c] : 0.f;
    } else if (o < P.u[0]) {
        int l = (int)((o - P.ab[0]) / (64 * 128));
        int64_t q = (o - P.ab[0]) % (64 * 128);
        int r = (int)(q / 128), c = (int)(q % 128);
        v = c < 64 ? theta[L.W_a[l] + r * 64 + c] : theta[L.W_b[l] + r * 64 + (c - 64)];
    } else if (o < P.out16) {
        int l = (int)((o - P.u[0]) / (128 * 64));
        int64_t q = (o - P.u[0]) % (128 * 64);
        v = theta[L.W_u[l] + q];
    } else if (o < P.abT[0]) {   // out16: 64 x 16
        int64_t q = o - P.out16;
        int r = (int)(q / 16), c = (int)(q % 16);
        v = c < 3 ? theta[L.W_out + r * 3 + c] : 0.f;
    } else if (o < P.uT[0]) {   // abT: 128 x 64
        int l = (int)((o - P.abT[0]) / (128 * 64));
        int64_t q = (o - P.abT[0]) % (128 * 64);
        int r = (int)(q / 64), c = (int)(q % 64);   // (r, c) of the transpose = (c, r) of [W_a | W_b]
        v = r < 64 ? theta[L.W_a[l] + c * 64 + r] : theta[L.W_b[l] + c * 64 + (r - 64)];
    } else if (o < P.out16T) {   // uT: 64 x 128
        int l = (int)((o - P.uT[0]) / (64 * 128));
        int64_t q = (o - P.uT[0]) % (64 * 128);
        int r = (int)(q / 128), c = (int)(q % 128);
        v = theta[L.W_u[l] + c * 64 + r];
    } else {   // out16T: 16 x 64
        int64_t q = o - P.out16T;
        int r = (int)(q / 64), c = (int)(q % 64);
        v = r < 3 ? theta[L.W_out + c * 3 + r] : 0.f;
    }
    wbf[o] = f2bf(v);
}

// ---------------------------------------------------------------- MFMA GEMM
//
// C[M x N] (=|+=) A[M x K] B[K x N] (+ bias): A FP32 row-major (lda), B BF16
// row-major K x N, K and N multiples of 16 (<= 128).  A workgroup of 4 waves
// takes 64 rows; wave w takes rows [16w, 16w+16) and every 16-wide column
// tile.  v_mfma_f32_16x16x16_bf16 lane layout (wave64): lane l holds
//   A[l % 16][4 (l / 16) + t], B[4 (l / 16) + t][l % 16], D[4 (l / 16) + t][l % 16], t = 0..3.

__global__ __launch_bounds__(256) void k_gemm(const float *A, int64_t lda, const unsigned short *B, float *C,
                                              int64_t ldc, int64_t M, int K, int N, const float *bias,
                                              int accumulate)
{
    __shared__ unsigned short sB[128 * 128];
    for (int t = threadIdx.x; t < K * N; t += 256) sB[t] = B[t];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + 16 * wv;
    const int lr = lane & 15, lg = lane >> 4;
    const int64_t arow = r0 + lr;
    const bool arow_ok = arow < M;
    for (int n0 = 0; n0 < N; n0 += 16) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < K; k0 += 16) {
            bf16x4 a, b;
            for (int t = 0; t < 4; t++) {
                float av = arow_ok ? A[arow * lda + k0 + 4 * lg + t] : 0.f;
                a[t] = (short)f2bf(av);
                b[t] = (short)sB[(k0 + 4 * lg + t) * N + n0 + lr];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        for (int t = 0; t < 4; t++) {
            const int64_t row = r0 + 4 * lg + t;
            if (row >= M) continue;
            float v = acc[t];
            if (bias) v += bias[n0 + lr];
            float *c = C + row * ldc + n0 + lr;
            *c = accumulate ? *c + v : v;
        }
    }
}

// Weight gradient G[K x N] = A^T D over M rows, split into chunks of CH rows:
// partial p holds the chunk's product (MFMA, reduction dimension = rows);
// k_sum_parts adds the partials in chunk order.
constexpr int CH = 2048;

__global__ __launch_bounds__(256) void k_gemm_at(const float *A, int64_t lda, const float *D, int64_t ldd, int64_t M,
                                                 int K, int N, float *part)
{
    __shared__ float sA[16][128];
    __shared__ float sD[16][128];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * CH;
    const int tiles = (K / 16) * (N / 16);
    f32x4 acc[8];
    for (int q = 0; q < 8; q++) acc[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int64_t rs = m0; rs < m0 + CH && rs < M; rs += 16) {
        __syncthreads();
        for (int t = threadIdx.x; t < 16 * K; t += 256) {
            int r = t / K, c = t % K;
            sA[r][c] = (rs + r < M) ? A[(rs + r) * lda + c] : 0.f;
        }
        for (int t = threadIdx.x; t < 16 * N; t += 256) {
            int r = t / N, c = t % N;
            sD[r][c] = (rs + r < M) ? D[(rs + r) * ldd + c] : 0.f;
        }
        __syncthreads();
        for (int q = 0; q < 8; q++) {
            int tile = wv + 4 * q;
            if (tile >= tiles) break;
            int kt = tile / (N / 16), nt = tile % (N / 16);
            bf16x4 a, b;
            for (int t = 0; t < 4; t++) {
                a[t] = (short)f2bf(sA[4 * lg + t][16 * kt + lr]);   // (A^T)[row][k] = A[k][row]
                b[t] = (short)f2bf(sD[4 * lg + t][16 * nt + lr]);
            }
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[q], 0, 0, 0);
        }
    }
    float *P = part + (int64_t)blockIdx.x * K * N;
    for (int q = 0; q < 8; q++) {
        int tile = wv + 4 * q;
        if (tile >= tiles) break;
        int kt = tile / (N / 16), nt = tile % (N / 16);
        for (int t = 0; t < 4; t++) P[(16 * kt + 4 * lg + t) * N + 16 * nt + lr] = acc[q][t];
    }
}

// out[r][c] (in the flat gradient, with row stride ld and column window
// [c0, c1)) = sum over chunks of part[chunk][r][c]
__global__ void k_sum_parts(const float *part, int nparts, int K, int N, int r1, int c0, int c1, float *out,
                            int64_t ld)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= r1 * (c1 - c0)) return;
    int r = t / (c1 - c0), c = c0 + t % (c1 - c0);
    float s = 0.f;
    for (int p = 0; p < nparts; p++) s += part[(int64_t)p * K * N + r * N + c];
    out[(int64_t)r * ld + (c - c0)] = s;
}

// column sums of A[M x N] (first nc columns) in chunks of CH rows, then in chunk order
__global__ void k_colsum_part(const float *A, int64_t lda, int64_t M, int nc, float *part)
{
    int c = threadIdx.x;
    if (c >= nc) return;
    int64_t m0 = (int64_t)blockIdx.x * CH;
    float s = 0.f;
    for (int64_t r = m0; r < m0 + CH && r < M; r++) s += A[r * lda + c];
    part[(int64_t)blockIdx.x * nc + c] = s;
}

__global__ void k_colsum_final(const float *part, int nparts, int nc, float *out)
{
    int c = threadIdx.x;
    if (c >= nc) return;
    float s = 0.f;
    for (int p = 0; p < nparts; p++) s += part[(int64_t)p * nc + c];
    out[c] = s;
}

// ---------------------------------------------------------------- elementwise

__global__ void k_input(int64_t n, const double *F, const double *vp, float sF, float sV, float *x16)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float *x = x16 + 16 * i;
    for (int a = 0; a < 3; a++) {
        x[a] = (float)(F[3 * i + a] / sF);
        x[3 + a] = (float)(vp[3 * i + a] / sV);
    }
    for (int a = 6; a < 16; a++) x[a] = 0.f;
}

// e_p = [w/sW, n], n = (r_i - r_j)/d = -u_e for i < j, +u_e otherwise
__global__ void k_edge_feat(int64_t n, const int32_t *rowptr, const int32_t *col, const int32_t *ent_edge,
                            const double4 *wu, float sW, float4 *ef)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
        double4 q = wu[ent_edge[p]];
        float s = (i < col[p]) ? -1.f : 1.f;
        ef[p] = make_float4((float)(q.x / sW), s * (float)q.y, s * (float)q.z, s * (float)q.w);
    }
}

__global__ void k_relu(int64_t len, const float *a, float *b)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) b[t] = fmaxf(a[t], 0.f);
}

// h_next = h + relu(U)
__global__ void k_residual(int64_t len, const float *h, const float *U, float *hn)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) hn[t] = h[t] + fmaxf(U[t], 0.f);
}

// dst = src * (mask > 0)
__global__ void k_mask(int64_t len, const float *src, const float *mask, float *dst)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) dst[t] = mask[t] > 0.f ? src[t] : 0.f;
}

// dst (row stride ldd) = a (row stride lda) + b (row stride ldb), 64 columns
__global__ void k_add64(int64_t n, const float *a, int64_t lda, const float *b, int64_t ldb, float *dst, int64_t ldd)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 64) return;
    int64_t i = t / 64;
    int c = (int)(t % 64);
    dst[i * ldd + c] = a[i * lda + c] + b[i * ldb + c];
}

// ---------------------------------------------------------------- messages (one wave per row, lane = feature)

__global__ __launch_bounds__(256) void k_msg_fwd(int64_t n, const int32_t *rowptr, const int32_t *col,
                                                 const float4 *ef, const float *PQ, const float *bm,
                                                 const float *Wc, float *agg)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int f = threadIdx.x & 63;
    if (i >= n) return;
    const float Pi = PQ[i * 128 + f] + bm[f];
    const float w0 = Wc[f], w1 = Wc[64 + f], w2 = Wc[128 + f], w3 = Wc[192 + f];
    float acc = 0.f;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
        const int64_t j = col[p];
        const float4 e = ef[p];
        const float z = Pi + PQ[j * 128 + 64 + f] + (e.x * w0 + e.y * w1 + e.z * w2 + e.w * w3);
        acc += fmaxf(z, 0.f);
    }
    agg[i * 64 + f] = acc;
}

// dP_i = sum over row i of dz_p, dz_p = da_i [z_p > 0]; per-workgroup partials of e_p^T dz_p
__global__ __launch_bounds__(256) void k_msg_bwd_p(int64_t n, const int32_t *rowptr, const int32_t *col,
                                                   const float4 *ef, const float *PQ, const float *bm,
                                                   const float *Wc, const float *da, int64_t ldda, float *dPQ,
                                                   float *wc_part)
{
    __shared__ float sw[4][256];
    const int wv = threadIdx.x >> 6, f = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + wv;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
    if (i < n) {
        const float Pi = PQ[i * 128 + f] + bm[f];
        const float w0 = Wc[f], w1 = Wc[64 + f], w2 = Wc[128 + f], w3 = Wc[192 + f];
        const float dai = da[i * ldda + f];
        float dp = 0.f;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            const int64_t j = col[p];
            const float4 e = ef[p];
            const float z = Pi + PQ[j * 128 + 64 + f] + (e.x * w0 + e.y * w1 + e.z * w2 + e.w * w3);
            const float dz = z > 0.f ? dai : 0.f;
            dp += dz;
            g0 += e.x * dz;
            g1 += e.y * dz;
            g2 += e.z * dz;
            g3 += e.w * dz;
        }
        dPQ[i * 128 + f] = dp;
    }
    sw[wv][f] = g0;
    sw[wv][64 + f] = g1;
    sw[wv][128 + f] = g2;
    sw[wv][192 + f] = g3;
    __syncthreads();
    const int t = threadIdx.x;   // 256 = 4 x 64 outputs
    wc_part[(int64_t)blockIdx.x * 256 + t] = (sw[0][t] + sw[1][t]) + (sw[2][t] + sw[3][t]);
}

// dQ_j = sum over the entries (i, j) of column j of dz: walked as row j's
// entries (j, i) with the twin's features e = [w, -n]
__global__ __launch_bounds__(256) void k_msg_bwd_q(int64_t n, const int32_t *rowptr, const int32_t *col,
                                                   const float4 *ef, const float *PQ, const float *bm,
                                                   const float *Wc, const float *da, int64_t ldda, float *dPQ)
{
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int f = threadIdx.x & 63;
    if (j >= n) return;
    const float Qj = PQ[j * 128 + 64 + f];
    const float w0 = Wc[f], w1 = Wc[64 + f], w2 = Wc[128 + f], w3 = Wc[192 + f];
    float dq = 0.f;
    for (int32_t p = rowptr[j]; p < rowptr[j + 1]; p++) {
        const int64_t i = col[p];
        const float4 e = ef[p];
        const float z = (PQ[i * 128 + f] + bm[f]) + Qj + (e.x * w0 - e.y * w1 - e.z * w2 - e.w * w3);
        dq += z > 0.f ? da[i * ldda + f] : 0.f;
    }
    dPQ[j * 128 + 64 + f] = dq;
}

// loss = mean (out - v/sV)^2 over 3n values; dout16 = 2 (out - v/sV)/(3n) in columns 0..2
__global__ __launch_bounds__(256) void k_loss(int64_t n, const float *out16, const double *v, float sV, float *dout16,
                                              double *part)
{
    __shared__ double sh[256];
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (i < n) {
        for (int a = 0; a < 16; a++) {
            float d = 0.f;
            if (a < 3) {
                d = out16[16 * i + a] - (float)(v[3 * i + a] / sV);
                s += (double)d * (double)d;
                d = 2.f * d / (float)(3 * n);
            }
            dout16[16 * i + a] = d;
        }
    }
    s = block_sum_256(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_double(const double *part, int np, double *out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < np; k += 256) s += part[k];
    s = block_sum_256(s, sh);
    if (threadIdx.x == 0) *out = s;
}

__global__ void k_output(int64_t n, const float *out16, double sV, double *vhat)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int a = 0; a < 3; a++) vhat[3 * i + a] = sV * (double)out16[16 * i + a];
}

__global__ void k_adam(int64_t np, float *theta, const float *g, float *m1, float *m2, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np) return;
    float gt = g[t];
    float a = b1 * m1[t] + (1.f - b1) * gt;
    float b = b2 * m2[t] + (1.f - b2) * gt * gt;
    m1[t] = a;
    m2[t] = b;
    theta[t] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// b_out added to the first three output columns
__global__ void k_add_bias3(int64_t n, float *out16, const float *b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out16[16 * i] += b[0];
    out16[16 * i + 1] += b[1];
    out16[16 * i + 2] += b[2];
}

// ---------------------------------------------------------------- host drivers

struct Act {
    float *x16, *pre0, *h[NL + 1], *PQ, *a[NL], *U[NL], *out16;   // forward
    float *dout16, *dh, *dU, *dcat, *dPQ, *tmp;                    // backward
};

int64_t act_floats(int64_t n) { return n * (16 + 64 + 64 * (NL + 1) + 128 + 64 * NL + 64 * NL + 16 + 16 + 64 + 64 + 128 + 128 + 64); }

Act carve(float *base, int64_t n)
{
    Act A;
    float *p = base;
    auto take = [&](int64_t cnt) { float *q = p; p += cnt; return q; };
    A.x16 = take(16 * n);
    A.pre0 = take(64 * n);
    for (int l = 0; l <= NL; l++) A.h[l] = take(64 * n);
    A.PQ = take(128 * n);
    for (int l = 0; l < NL; l++) A.a[l] = take(64 * n);
    for (int l = 0; l < NL; l++) A.U[l] = take(64 * n);
    A.out16 = take(16 * n);
    A.dout16 = take(16 * n);
    A.dh = take(64 * n);
    A.dU = take(64 * n);
    A.dcat = take(128 * n);
    A.dPQ = take(128 * n);
    A.tmp = take(64 * n);
    return A;
}

int gemm(sgp_ctx ctx, const float *A, int64_t lda, const unsigned short *B, float *C, int64_t ldc, int64_t M, int K,
         int N, const float *bias, int acc)
{
    if (M <= 0) return SGP_OK;
    k_gemm<<<grid_for(M, 64), 256, 0, ctx->stream>>>(A, lda, B, C, ldc, M, K, N, bias, acc);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

// out (flat gradient at off, row stride ld) = A^T D restricted to rows [0, r1), columns [c0, c1)
int gemm_at(sgp_ctx ctx, sgp_mpnn M, const float *A, int64_t lda, const float *D, int64_t ldd, int64_t m, int K, int N,
            int r1, int c0, int c1, float *out, int64_t ld)
{
    int nparts = (int)((m + CH - 1) / CH);
    if (nparts == 0) nparts = 1;
    float *part;
    SGP_TRY(ensure_t(ctx, M->part, (size_t)nparts * K * N + 64, &part));
    k_gemm_at<<<nparts, 256, 0, ctx->stream>>>(A, lda, D, ldd, m, K, N, part);
    k_sum_parts<<<grid_for(r1 * (c1 - c0), 256), 256, 0, ctx->stream>>>(part, nparts, K, N, r1, c0, c1, out, ld);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

int colsum(sgp_ctx ctx, sgp_mpnn M, const float *A, int64_t lda, int64_t m, int nc, float *out)
{
    int nparts = (int)((m + CH - 1) / CH);
    if (nparts == 0) nparts = 1;
    float *part;
    SGP_TRY(ensure_t(ctx, M->part, (size_t)nparts * nc + 64, &part));
    k_colsum_part<<<nparts, 128, 0, ctx->stream>>>(A, lda, m, nc, part);
    k_colsum_final<<<1, 128, 0, ctx->stream>>>(part, nparts, nc, out);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

int prepare(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, const double *F, const double *vp, Act &A)
{
    const int64_t n = g->n, ne = 2 * g->m;
    float *base;
    float4 *ef;
    SGP_TRY(ensure_t(ctx, M->act, (size_t)act_floats(n) + 64, &base));
    SGP_TRY(ensure_t(ctx, M->efeat, (size_t)ne + 1, &ef));
    A = carve(base, n);
    hipStream_t st = ctx->stream;
    k_input<<<grid_for(n, 256), 256, 0, st>>>(n, F, vp, (float)M->sF, (float)M->sV, A.x16);
    k_edge_feat<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)g->rowptr.p, (const int32_t *)g->col.p,
                                                  (const int32_t *)g->ent_edge.p, (const double4 *)g->wu.p,
                                                  (float)M->sW, ef);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

int forward(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, Act &A)
{
    hipStream_t st = ctx->stream;
    const int64_t n = g->n;
    const unsigned short *W = (const unsigned short *)M->wbf.p;
    const float *wr = (const float *)M->wrow.p;
    const Layout &L = M->L;
    const Packed &PK = M->PK;
    const int32_t *rowptr = (const int32_t *)g->rowptr.p, *col = (const int32_t *)g->col.p;
    const float4 *ef = (const float4 *)M->efeat.p;
    SGP_TRY(gemm(ctx, A.x16, 16, W + PK.in16, A.pre0, 64, n, 16, 64, wr + L.b_in, 0));
    k_relu<<<grid_for(64 * n, 256), 256, 0, st>>>(64 * n, A.pre0, A.h[0]);
    for (int l = 0; l < NL; l++) {
        SGP_TRY(gemm(ctx, A.h[l], 64, W + PK.ab[l], A.PQ, 128, n, 64, 128, nullptr, 0));
        k_msg_fwd<<<grid_for(n, 4), 256, 0, st>>>(n, rowptr, col, ef, A.PQ, wr + L.b_m[l], wr + L.W_c[l], A.a[l]);
        SGP_TRY(gemm(ctx, A.h[l], 64, W + PK.u[l], A.U[l], 64, n, 64, 64, wr + L.b_u[l], 0));
        SGP_TRY(gemm(ctx, A.a[l], 64, W + PK.u[l] + 64 * 64, A.U[l], 64, n, 64, 64, nullptr, 1));
        k_residual<<<grid_for(64 * n, 256), 256, 0, st>>>(64 * n, A.h[l], A.U[l], A.h[l + 1]);
    }
    SGP_TRY(gemm(ctx, A.h[NL], 64, W + PK.out16, A.out16, 16, n, 64, 16, nullptr, 0));
    // b_out (3 entries) added by a tiny pass
    k_add_bias3<<<grid_for(n, 256), 256, 0, st>>>(n, A.out16, wr + L.b_out);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

int backward(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, Act &A)
{
    hipStream_t st = ctx->stream;
    const int64_t n = g->n;
    const unsigned short *W = (const unsigned short *)M->wbf.p;
    const float *wr = (const float *)M->wrow.p;
    const Layout &L = M->L;
    const Packed &PK = M->PK;
    float *G = (float *)M->grad.p;
    const int32_t *rowptr = (const int32_t *)g->rowptr.p, *col = (const int32_t *)g->col.p;
    const float4 *ef = (const float4 *)M->efeat.p;
    // output layer
    SGP_TRY(gemm_at(ctx, M, A.h[NL], 64, A.dout16, 16, n, 64, 16, 64, 0, 3, G + L.W_out, 3));
    SGP_TRY(colsum(ctx, M, A.dout16, 16, n, 3, G + L.b_out));
    SGP_TRY(gemm(ctx, A.dout16, 16, W + PK.out16T, A.dh, 64, n, 16, 64, nullptr, 0));
    for (int l = NL - 1; l >= 0; l--) {
        k_mask<<<grid_for(64 * n, 256), 256, 0, st>>>(64 * n, A.dh, A.U[l], A.dU);
        SGP_TRY(gemm_at(ctx, M, A.h[l], 64, A.dU, 64, n, 64, 64, 64, 0, 64, G + L.W_u[l], 64));
        SGP_TRY(gemm_at(ctx, M, A.a[l], 64, A.dU, 64, n, 64, 64, 64, 0, 64, G + L.W_u[l] + 64 * 64, 64));
        SGP_TRY(colsum(ctx, M, A.dU, 64, n, 64, G + L.b_u[l]));
        SGP_TRY(gemm(ctx, A.dU, 64, W + PK.uT[l], A.dcat, 128, n, 64, 128, nullptr, 0));   // [dh part | da]
        // messages: recompute PQ of this layer from h[l]
        SGP_TRY(gemm(ctx, A.h[l], 64, W + PK.ab[l], A.PQ, 128, n, 64, 128, nullptr, 0));
        int nb = (int)grid_for(n, 4);
        float *wcp;
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP9], (size_t)nb * 256 + 64, &wcp));
        k_msg_bwd_p<<<nb, 256, 0, st>>>(n, rowptr, col, ef, A.PQ, wr + L.b_m[l], wr + L.W_c[l], A.dcat + 64, 128,
                                        A.dPQ, wcp);
        k_msg_bwd_q<<<nb, 256, 0, st>>>(n, rowptr, col, ef, A.PQ, wr + L.b_m[l], wr + L.W_c[l], A.dcat + 64, 128,
                                        A.dPQ);
        k_colsum_final<<<1, 256, 0, st>>>(wcp, nb, 256, G + L.W_c[l]);   // partials in block order
        LAUNCH_CHECK(ctx);
        SGP_TRY(colsum(ctx, M, A.dPQ, 128, n, 64, G + L.b_m[l]));
        SGP_TRY(gemm_at(ctx, M, A.h[l], 64, A.dPQ, 128, n, 64, 128, 64, 0, 64, G + L.W_a[l], 64));
        SGP_TRY(gemm_at(ctx, M, A.h[l], 64, A.dPQ, 128, n, 64, 128, 64, 64, 128, G + L.W_b[l], 64));
        // dh_l = dh (residual) + dcat[:, :64] + dPQ W_ab^T
        k_add64<<<grid_for(64 * n, 256), 256, 0, st>>>(n, A.dh, 64, A.dcat, 128, A.tmp, 64);
        LAUNCH_CHECK(ctx);
        SGP_TRY(gemm(ctx, A.dPQ, 128, W + PK.abT[l], A.tmp, 64, n, 128, 64, nullptr, 1));
        std::swap(A.dh, A.tmp);
    }
    k_mask<<<grid_for(64 * n, 256), 256, 0, st>>>(64 * n, A.dh, A.pre0, A.dU);
    SGP_TRY(gemm_at(ctx, M, A.x16, 16, A.dU, 64, n, 16, 64, 6, 0, 64, G + L.W_in, 64));
    SGP_TRY(colsum(ctx, M, A.dU, 64, n, 64, G + L.b_in));
    return SGP_OK;
}

int repack(sgp_ctx ctx, sgp_mpnn M)
{
    unsigned short *wbf;
    float *wr;
    SGP_TRY(ensure_t(ctx, M->wbf, (size_t)M->PK.total + 8, &wbf));
    SGP_TRY(ensure_t(ctx, M->wrow, (size_t)M->L.total + 8, &wr));
    int64_t cnt = std::max<int64_t>(M->PK.total, M->L.total);
    k_pack<<<grid_for(cnt, 256), 256, 0, ctx->stream>>>((const float *)M->theta.p, M->L, M->PK, wbf, wr);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

}   // namespace

// ---------------------------------------------------------------- C ABI

extern "C" int sgp_mpnn_param_count(int64_t *count)
{
    if (!count) return SGP_EINVAL;
    *count = make_layout().total;
    return SGP_OK;
}

extern "C" int sgp_mpnn_create(sgp_ctx ctx, sgp_mpnn *out)
{
    if (!ctx || !out) return set_err(ctx, SGP_EINVAL, "mpnn_create: null");
    *out = new (std::nothrow) sgp_mpnn_();
    return *out ? SGP_OK : set_err(ctx, SGP_ENOMEM, "mpnn_create: out of memory");
}

extern "C" void sgp_mpnn_free(sgp_mpnn M)
{
    if (!M) return;
    (void)hipDeviceSynchronize();
    release(M->theta); release(M->m1); release(M->m2); release(M->grad); release(M->wbf); release(M->wrow);
    release(M->act); release(M->efeat); release(M->part);
    delete M;
}

extern "C" int sgp_mpnn_set_params(sgp_ctx ctx, sgp_mpnn M, const float *theta, double sF, double sV, double sW)
{
    if (!ctx || !M || !theta || !(sF > 0) || !(sV > 0) || !(sW > 0))
        return set_err(ctx, SGP_EINVAL, "mpnn_set_params: bad arguments");
    const int64_t np = M->L.total;
    float *t, *a, *b, *gr;
    SGP_TRY(ensure_t(ctx, M->theta, np + 8, &t));
    SGP_TRY(ensure_t(ctx, M->m1, np + 8, &a));
    SGP_TRY(ensure_t(ctx, M->m2, np + 8, &b));
    SGP_TRY(ensure_t(ctx, M->grad, np + 8, &gr));
    HIP_TRY(ctx, hipMemcpyAsync(t, theta, np * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(a, 0, np * sizeof(float), ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(b, 0, np * sizeof(float), ctx->stream));
    M->sF = sF;
    M->sV = sV;
    M->sW = sW;
    M->adam_t = 0;
    return repack(ctx, M);
}

extern "C" int sgp_mpnn_get_params(sgp_ctx ctx, sgp_mpnn M, float *theta)
{
    if (!ctx || !M || !theta || !M->theta.p) return set_err(ctx, SGP_EINVAL, "mpnn_get_params: bad arguments");
    HIP_TRY(ctx, hipMemcpyAsync(theta, M->theta.p, M->L.total * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
    return SGP_OK;
}

static int check_common(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, const double *F, const double *vp)
{
    if (!ctx || !M || !g || !M->theta.p) return set_err(ctx, SGP_EINVAL, "mpnn: missing handle or parameters");
    if (g->n > 0 && (!F || !vp)) return set_err(ctx, SGP_EINVAL, "mpnn: null input");
    return SGP_OK;
}

extern "C" int sgp_mpnn_forward(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, const double *F, const double *vprev,
                                double *vhat)
{
    SGP_TRY(check_common(ctx, M, g, F, vprev));
    if (g->n == 0) return SGP_OK;
    if (!vhat) return set_err(ctx, SGP_EINVAL, "mpnn_forward: null output");
    Act A;
    SGP_TRY(prepare(ctx, M, g, F, vprev, A));
    SGP_TRY(forward(ctx, M, g, A));
    k_output<<<grid_for(g->n, 256), 256, 0, ctx->stream>>>(g->n, A.out16, M->sV, vhat);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

static int loss_grad(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, const double *F, const double *vprev, const double *v,
                     double *loss)
{
    Act A;
    const int64_t n = g->n;
    SGP_TRY(prepare(ctx, M, g, F, vprev, A));
    SGP_TRY(forward(ctx, M, g, A));
    double *part;
    int nb = (int)grid_for(n, 256);
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PART], (size_t)nb + 8, &part));
    k_loss<<<nb, 256, 0, ctx->stream>>>(n, A.out16, v, (float)M->sV, A.dout16, part);
    k_sum_double<<<1, 256, 0, ctx->stream>>>(part, nb, part + nb);
    LAUNCH_CHECK(ctx);
    SGP_TRY(backward(ctx, M, g, A));
    double s;
    SGP_TRY(readback(ctx, &s, part + nb, sizeof s));
    if (loss) *loss = s / (3.0 * (double)n);
    return SGP_OK;
}

extern "C" int sgp_mpnn_grad(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, const double *F, const double *vprev,
                             const double *v, float *grad, double *loss)
{
    SGP_TRY(check_common(ctx, M, g, F, vprev));
    if (!v || !grad || g->n == 0) return set_err(ctx, SGP_EINVAL, "mpnn_grad: bad arguments");
    SGP_TRY(loss_grad(ctx, M, g, F, vprev, v, loss));
    HIP_TRY(ctx, hipMemcpyAsync(grad, M->grad.p, M->L.total * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
    return SGP_OK;
}

extern "C" int sgp_mpnn_train_step(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, const double *F, const double *vprev,
                                   const double *v, double lr, double *loss)
{
    SGP_TRY(check_common(ctx, M, g, F, vprev));
    if (!v || g->n == 0 || !(lr > 0)) return set_err(ctx, SGP_EINVAL, "mpnn_train_step: bad arguments");
    SGP_TRY(loss_grad(ctx, M, g, F, vprev, v, loss));
    M->adam_t++;
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = 1.f - powf(b1, (float)M->adam_t), c2 = 1.f - powf(b2, (float)M->adam_t);
    k_adam<<<grid_for(M->L.total, 256), 256, 0, ctx->stream>>>(M->L.total, (float *)M->theta.p, (const float *)M->grad.p,
                                                              (float *)M->m1.p, (float *)M->m2.p, (float)lr, b1, b2,
                                                              1e-8f, c1, c2);
    LAUNCH_CHECK(ctx);
    return repack(ctx, M);
}
