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
// Order: the network runs in the graph's internal (cell-list) vertex order,
// so a row's neighbours sit close in memory and the per-edge gathers mostly
// hit in L2; inputs are gathered and outputs scattered through the graph's
// permutation at the boundary.  The network is permutation-equivariant, so
// this changes only the order of roundings in its sums.
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
    DevBuf act, efeat, part, red, sum, vq;   // vq: v_hat and Gamma v_hat (FP64, canonical order)
    DevBuf irow, icol;                      // neighbour lists in the internal order (with efeat)
    const void *lists_of = nullptr;         // graph and version they were built for
    uint64_t lists_version = 0;
    double lists_sW = 0;
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
// row-major K x N, K = 16 KT and N multiples of 16 (<= 128).
// v_mfma_f32_16x16x16_bf16 lane layout (wave64): lane l holds
//   A[l % 16][4 (l / 16) + t], B[4 (l / 16) + t][l % 16], D[4 (l / 16) + t][l % 16], t = 0..3.
// B is staged in LDS in fragment order (a lane's four k-values adjacent, one
// 8-byte read); a wave converts the A fragments of its 16-row tile to BF16
// once and reuses them for every column tile.  A workgroup (4 waves) covers
// GEMM_ROWS rows (one 16-row tile per wave: more waves in flight than
// several tiles per wave, whose loads would wait for the previous tile).
constexpr int GEMM_ROWS = 64;

template <int KT>
__global__ __launch_bounds__(256) void k_gemm(const float *A, int64_t lda, const unsigned short *B, float *C,
                                              int64_t ldc, int64_t M, int N, const float *bias, int accumulate,
                                              float *R)
{
    __shared__ bf16x4 sB[KT * 8 * 64];
    const int NT = N >> 4;
    for (int e = threadIdx.x; e < KT * NT * 64; e += 256) {
        const int ln = e & 63, tile = e >> 6, kt = tile / NT, nt = tile % NT;
        bf16x4 b;
        for (int t = 0; t < 4; t++) b[t] = (short)B[(16 * kt + 4 * (ln >> 4) + t) * N + 16 * nt + (ln & 15)];
        sB[e] = b;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    for (int it = 0; it < GEMM_ROWS / 64; it++) {
        const int64_t r0 = (int64_t)blockIdx.x * GEMM_ROWS + 64 * it + 16 * wv;
        if (r0 >= M) break;
        // every load of the tile before any store, unconditional (rows past
        // M read row M-1 and are not stored): a load behind a store, or in a
        // branch, would wait for it
        const int64_t arow = min(r0 + lr, M - 1);
        float4 av[KT];
#pragma unroll
        for (int kt = 0; kt < KT; kt++) av[kt] = *(const float4 *)(A + arow * lda + 16 * kt + 4 * lg);
        float bv[8], cv[8][4];
#pragma unroll
        for (int nt = 0; nt < 8; nt++) {
            bv[nt] = bias && nt < NT ? bias[16 * nt + lr] : 0.f;
            if (accumulate && nt < NT)
                for (int t = 0; t < 4; t++) cv[nt][t] = C[min(r0 + 4 * lg + t, M - 1) * ldc + 16 * nt + lr];
        }
        keep_loads_above();
        bf16x4 a[KT];
#pragma unroll
        for (int kt = 0; kt < KT; kt++) {
            a[kt][0] = (short)f2bf(av[kt].x);
            a[kt][1] = (short)f2bf(av[kt].y);
            a[kt][2] = (short)f2bf(av[kt].z);
            a[kt][3] = (short)f2bf(av[kt].w);
        }
#pragma unroll
        for (int nt = 0; nt < 8; nt++) {
            if (nt >= NT) break;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < KT; kt++)
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[kt], sB[(kt * NT + nt) * 64 + lane], acc, 0, 0, 0);
            for (int t = 0; t < 4; t++) {
                const int64_t row = r0 + 4 * lg + t;
                if (row >= M) continue;
                const float v = acc[t] + bv[nt];
                const float o = accumulate ? cv[nt][t] + v : v;
                C[row * ldc + 16 * nt + lr] = o;
                if (R) R[row * ldc + 16 * nt + lr] = fmaxf(o, 0.f);
            }
        }
    }
}

// One layer's node update in one pass: U = [h, a] W_u + b_u as the two
// K = 64 products of the unfused form (h against rows 0..63 of W_u plus the
// bias, then a against rows 64..127, added in that order), kept for the
// backward pass, and h' = h + relu(U).  The operations and their order are
// those of two k_gemm launches and the residual pass, so the results are
// the same bit for bit; h and a are read once and U is not read back.
__global__ __launch_bounds__(256) void k_gemm_update(const float *H, const float *Ag, const unsigned short *B,
                                                     const float *bias, float *U, float *Hn, int64_t M)
{
    constexpr int KT = 4, NT = 4, N = 64;
    __shared__ bf16x4 sB[2 * KT * NT * 64];
    for (int e = threadIdx.x; e < 2 * KT * NT * 64; e += 256) {
        const int half = e / (KT * NT * 64), f = e % (KT * NT * 64);
        const int ln = f & 63, tile = f >> 6, kt = tile / NT, nt = tile % NT;
        bf16x4 b;
        for (int t = 0; t < 4; t++)
            b[t] = (short)B[(64 * half + 16 * kt + 4 * (ln >> 4) + t) * N + 16 * nt + (ln & 15)];
        sB[e] = b;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    for (int it = 0; it < GEMM_ROWS / 64; it++) {
        const int64_t r0 = (int64_t)blockIdx.x * GEMM_ROWS + 64 * it + 16 * wv;
        if (r0 >= M) break;
        // Every load of the tile before any store, unconditional (rows past
        // M read row M-1; their results are not stored): the fragments of h
        // and a, and h at the lane's output positions for the residual.  A
        // load behind a store, or in a branch, would wait for it.
        const int64_t arow = min(r0 + lr, M - 1);
        float hv[NT][4];
#pragma unroll
        for (int nt = 0; nt < NT; nt++)
#pragma unroll
            for (int t = 0; t < 4; t++) hv[nt][t] = H[min(r0 + 4 * lg + t, M - 1) * N + 16 * nt + lr];
        float4 vh[KT], va[KT];
#pragma unroll
        for (int kt = 0; kt < KT; kt++) {
            vh[kt] = *(const float4 *)(H + arow * 64 + 16 * kt + 4 * lg);
            va[kt] = *(const float4 *)(Ag + arow * 64 + 16 * kt + 4 * lg);
        }
        float bv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; nt++) bv[nt] = bias[16 * nt + lr];
        keep_loads_above();
        bf16x4 ah[KT], aa[KT];
#pragma unroll
        for (int kt = 0; kt < KT; kt++) {
            ah[kt][0] = (short)f2bf(vh[kt].x);
            ah[kt][1] = (short)f2bf(vh[kt].y);
            ah[kt][2] = (short)f2bf(vh[kt].z);
            ah[kt][3] = (short)f2bf(vh[kt].w);
            aa[kt][0] = (short)f2bf(va[kt].x);
            aa[kt][1] = (short)f2bf(va[kt].y);
            aa[kt][2] = (short)f2bf(va[kt].z);
            aa[kt][3] = (short)f2bf(va[kt].w);
        }
        for (int nt = 0; nt < NT; nt++) {
            f32x4 acc1 = {0.f, 0.f, 0.f, 0.f}, acc2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < KT; kt++) {
                acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[kt], sB[(kt * NT + nt) * 64 + lane], acc1, 0, 0, 0);
                acc2 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aa[kt], sB[KT * NT * 64 + (kt * NT + nt) * 64 + lane],
                                                                 acc2, 0, 0, 0);
            }
            for (int t = 0; t < 4; t++) {
                const int64_t row = r0 + 4 * lg + t;
                if (row >= M) continue;
                const int64_t o = row * N + 16 * nt + lr;
                const float u = (acc1[t] + bv[nt]) + (acc2[t] + 0.f);
                U[o] = u;
                Hn[o] = hv[nt][t] + fmaxf(u, 0.f);
            }
        }
    }
}

// Weight-gradient partials over chunks of AT_ROWS rows: part[g] holds the
// chunk's A^T D (K x N, MFMA with the row index as the reduction dimension)
// followed by the chunk's column sums of D (N values, FP32).  A 64-row slab is
// staged in LDS transposed and in BF16, so a lane's four reduction-index
// values are adjacent; wave w owns the output tiles w, w + 4, ...  Every sum
// has a fixed order.
constexpr int AT_ROWS = 512;

template <int KT>
__global__ __launch_bounds__(256) void k_gemm_at(const float *A, int64_t lda, const float *D, int64_t ldd, int N,
                                                 int64_t M, float *part)
{
    constexpr int K = 16 * KT;
    __shared__ __attribute__((aligned(16))) unsigned short sAT[K][68];
    __shared__ __attribute__((aligned(16))) unsigned short sDT[128][68];
    __shared__ float scs[256];
    const int NT = N >> 4, tiles = KT * NT;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * AT_ROWS;
    const int64_t m1 = m0 + AT_ROWS < M ? m0 + AT_ROWS : M;
    f32x4 acc[8];
    for (int q = 0; q < 8; q++) acc[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
    float cs = 0.f;   // column threadIdx.x % N (256 is a multiple of N)
    for (int64_t rs = m0; rs < m1; rs += 64) {
        __syncthreads();
        for (int t = threadIdx.x; t < 64 * K; t += 256) {
            const int r = t / K, c = t % K;
            sAT[c][r] = f2bf(rs + r < m1 ? A[(rs + r) * lda + c] : 0.f);
        }
        for (int t = threadIdx.x; t < 64 * N; t += 256) {
            const int r = t / N, c = t % N;
            const float v = rs + r < m1 ? D[(rs + r) * ldd + c] : 0.f;
            cs += v;
            sDT[c][r] = f2bf(v);
        }
        __syncthreads();
        for (int sub = 0; sub < 4; sub++) {
            for (int q = 0; q < 8; q++) {
                const int tile = wv + 4 * q;
                if (tile >= tiles) break;
                const int kt = tile / NT, nt = tile % NT;
                const bf16x4 a = *(const bf16x4 *)&sAT[16 * kt + lr][16 * sub + 4 * lg];
                const bf16x4 b = *(const bf16x4 *)&sDT[16 * nt + lr][16 * sub + 4 * lg];
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[q], 0, 0, 0);
            }
        }
    }
    float *P = part + (int64_t)blockIdx.x * (K * N + N);
    for (int q = 0; q < 8; q++) {
        const int tile = wv + 4 * q;
        if (tile >= tiles) break;
        const int kt = tile / NT, nt = tile % NT;
        for (int t = 0; t < 4; t++) P[(16 * kt + 4 * lg + t) * N + 16 * nt + lr] = acc[q][t];
    }
    scs[threadIdx.x] = cs;
    __syncthreads();
    if (threadIdx.x < N) {
        float s = 0.f;
        for (int k = threadIdx.x; k < 256; k += N) s += scs[k];
        P[K * N + threadIdx.x] = s;
    }
}

// Fixed-order reduction of G partial vectors of length L: stage 1 sums a
// contiguous run of `per` partials per segment, stage 2 the segments in order.
__global__ void k_red1(const float *part, int G, int L, int per, float *tmp)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= L) return;
    const int p0 = blockIdx.y * per, p1 = p0 + per < G ? p0 + per : G;
    float acc = 0.f;
    for (int p = p0; p < p1; p++) acc += part[(int64_t)p * L + c];
    tmp[(int64_t)blockIdx.y * L + c] = acc;
}

__global__ void k_red2(const float *tmp, int S, int L, float *out)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= L) return;
    float acc = 0.f;
    for (int s = 0; s < S; s++) acc += tmp[(int64_t)s * L + c];
    out[c] = acc;
}

// out[r * ld + (c - c0)] = red[off + r * N + c] for r < r1, c0 <= c < c1
__global__ void k_window(const float *red, int off, int N, int r1, int c0, int c1, float *out, int64_t ld)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= r1 * (c1 - c0)) return;
    const int r = t / (c1 - c0), c = c0 + t % (c1 - c0);
    out[(int64_t)r * ld + (c - c0)] = red[off + r * N + c];
}

// ---------------------------------------------------------------- elementwise

// node features of internal vertex i = graph vertex perm[i]
__global__ void k_input(int64_t n, const int32_t *perm, const double *F, const double *vp, float sF, float sV,
                        float *x16)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    float *x = x16 + 16 * i;
    for (int a = 0; a < 3; a++) {
        x[a] = (float)(F[3 * u + a] / sF);
        x[3 + a] = (float)(vp[3 * u + a] / sV);
    }
    for (int a = 6; a < 16; a++) x[a] = 0.f;
}

// neighbour count of internal row i
__global__ void k_int_deg(int64_t n, const int32_t *perm, const int32_t *rowptr, int32_t *deg)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t u = perm[i];
    deg[i] = rowptr[u + 1] - rowptr[u];
}

// internal neighbour lists (the graph's row order kept within a row) and the
// edge features e_p = [w/sW, n], n = (r_i - r_j)/d = -u_e when i < j in the
// graph's numbering, +u_e otherwise.  16 threads per row, one entry each.
__global__ void k_int_entries(int64_t n, const int32_t *perm, const int32_t *inv, const int32_t *rowptr,
                              const int32_t *col, const int32_t *ent_edge, const double4 *wu, float sW,
                              const int32_t *irow, int32_t *icol, float4 *ef)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t >> 4;
    if (i >= n) return;
    const int32_t u = perm[i];
    const int32_t b = rowptr[u], e = rowptr[u + 1], k0 = irow[i];
    for (int32_t c = (int32_t)(t & 15); c < e - b; c += 16) {
        const int32_t j = col[b + c];
        const double4 q = wu[ent_edge[b + c]];
        const float sg = (u < j) ? -1.f : 1.f;
        icol[k0 + c] = inv[j];
        ef[k0 + c] = make_float4((float)(q.x / sW), sg * (float)q.y, sg * (float)q.z, sg * (float)q.w);
    }
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

// ---------------------------------------------------------------- messages (forward: 16 lanes per row, four
// features per lane; backward: one wave per row, lane = feature)

// A row's entries are taken MSG_BATCH at a time: their column ids and edge
// features first, then all their neighbour gathers, then the arithmetic in
// entry order -- so a wave waits for memory twice per batch instead of twice
// per entry.  The summation order is the entry order, as in a plain loop.
constexpr int MSG_BATCH = 8;

__global__ __launch_bounds__(256) void k_msg_fwd(int64_t n, const int32_t *rowptr, const int32_t *col,
                                                 const float4 *ef, const float *PQ, const float *bm,
                                                 const float *Wc, float *agg)
{
    // 16 lanes per node, four features per lane (one 16-byte load of a
    // neighbour's 64 features per 16 lanes), 16 nodes per workgroup
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * 16 + (threadIdx.x >> 4);
    const int f = 4 * (threadIdx.x & 15);
    if (i >= n) return;
    const float4 pq = *(const float4 *)(PQ + i * 128 + f), b4 = *(const float4 *)(bm + f);
    const float P0 = pq.x + b4.x, P1 = pq.y + b4.y, P2 = pq.z + b4.z, P3 = pq.w + b4.w;
    const float4 w0 = *(const float4 *)(Wc + f), w1 = *(const float4 *)(Wc + 64 + f);
    const float4 w2 = *(const float4 *)(Wc + 128 + f), w3 = *(const float4 *)(Wc + 192 + f);
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    const int32_t re = rowptr[i + 1];
    for (int32_t p = rowptr[i]; p < re; p += MSG_BATCH) {
        // a batch's loads are unconditional (entries past the row's end
        // reload its last one and are not summed) and precede every use: a
        // load in a branch makes the compiler wait for it there
        const int cnt = re - p < MSG_BATCH ? re - p : MSG_BATCH;
        int32_t jj[MSG_BATCH];
        float4 ee[MSG_BATCH], qv[MSG_BATCH];
#pragma unroll
        for (int u = 0; u < MSG_BATCH; u++) {
            const int32_t pc = min(p + u, re - 1);
            jj[u] = col[pc];
            ee[u] = ef[pc];
        }
#pragma unroll
        for (int u = 0; u < MSG_BATCH; u++) qv[u] = *(const float4 *)(PQ + (int64_t)jj[u] * 128 + 64 + f);
        keep_loads_above();
#pragma unroll
        for (int u = 0; u < MSG_BATCH; u++)
            if (u < cnt) {
                const float4 e = ee[u], q = qv[u];
                a0 += fmaxf(P0 + q.x + (e.x * w0.x + e.y * w1.x + e.z * w2.x + e.w * w3.x), 0.f);
                a1 += fmaxf(P1 + q.y + (e.x * w0.y + e.y * w1.y + e.z * w2.y + e.w * w3.y), 0.f);
                a2 += fmaxf(P2 + q.z + (e.x * w0.z + e.y * w1.z + e.z * w2.z + e.w * w3.z), 0.f);
                a3 += fmaxf(P3 + q.w + (e.x * w0.w + e.y * w1.w + e.z * w2.w + e.w * w3.w), 0.f);
            }
    }
    *(float4 *)(agg + i * 64 + f) = make_float4(a0, a1, a2, a3);
}

// dP_i = sum over row i of dz_p, dz_p = da_i [z_p > 0]; per-workgroup partials
// of e_p^T dz_p (4 x 64).  The grid is fixed (at most MSG_BWD_GRID workgroups);
// workgroup b (in XCD-contiguous order) walks its own contiguous run of 4-row
// blocks in order.
constexpr int MSG_BWD_GRID = 1024;

__global__ __launch_bounds__(256) void k_msg_bwd_p(int64_t n, const int32_t *rowptr, const int32_t *col,
                                                   const float4 *ef, const float *PQ, const float *bm,
                                                   const float *Wc, const float *da, int64_t ldda, float *dPQ,
                                                   float *wc_part)
{
    __shared__ float sw[4][256];
    const int wv = threadIdx.x >> 6, f = threadIdx.x & 63;
    const float w0 = Wc[f], w1 = Wc[64 + f], w2 = Wc[128 + f], w3 = Wc[192 + f];
    const float bmf = bm[f];
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
    const int64_t nblk = (n + 3) / 4, per = (nblk + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = xcd_block(blockIdx.x, gridDim.x) * per;
    const int64_t b1 = b0 + per < nblk ? b0 + per : nblk;
    for (int64_t blk = b0; blk < b1; blk++) {
        const int64_t i = blk * 4 + wv;
        if (i >= n) continue;
        const float Pi = PQ[i * 128 + f] + bmf;
        const float dai = da[i * ldda + f];
        float dp = 0.f;
        const int32_t re = rowptr[i + 1];
        for (int32_t p = rowptr[i]; p < re; p += MSG_BATCH) {
            const int cnt = re - p < MSG_BATCH ? re - p : MSG_BATCH;
            int64_t jj[MSG_BATCH];
            float4 ee[MSG_BATCH];
            float qv[MSG_BATCH];
#pragma unroll
            for (int u = 0; u < MSG_BATCH; u++)
                if (u < cnt) {
                    jj[u] = col[p + u];
                    ee[u] = ef[p + u];
                }
#pragma unroll
            for (int u = 0; u < MSG_BATCH; u++)
                if (u < cnt) qv[u] = PQ[jj[u] * 128 + 64 + f];
#pragma unroll
            for (int u = 0; u < MSG_BATCH; u++)
                if (u < cnt) {
                    const float4 e = ee[u];
                    const float z = Pi + qv[u] + (e.x * w0 + e.y * w1 + e.z * w2 + e.w * w3);
                    const float dz = z > 0.f ? dai : 0.f;
                    dp += dz;
                    g0 += e.x * dz;
                    g1 += e.y * dz;
                    g2 += e.z * dz;
                    g3 += e.w * dz;
                }
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
    const int64_t j = xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    const int f = threadIdx.x & 63;
    if (j >= n) return;
    const float Qj = PQ[j * 128 + 64 + f];
    const float w0 = Wc[f], w1 = Wc[64 + f], w2 = Wc[128 + f], w3 = Wc[192 + f];
    const float bmf = bm[f];
    float dq = 0.f;
    const int32_t re = rowptr[j + 1];
    for (int32_t p = rowptr[j]; p < re; p += MSG_BATCH) {
        const int cnt = re - p < MSG_BATCH ? re - p : MSG_BATCH;
        int64_t ii[MSG_BATCH];
        float4 ee[MSG_BATCH];
        float pv[MSG_BATCH], dv[MSG_BATCH];
#pragma unroll
        for (int u = 0; u < MSG_BATCH; u++)
            if (u < cnt) {
                ii[u] = col[p + u];
                ee[u] = ef[p + u];
            }
#pragma unroll
        for (int u = 0; u < MSG_BATCH; u++)
            if (u < cnt) {
                pv[u] = PQ[ii[u] * 128 + f];
                dv[u] = da[ii[u] * ldda + f];
            }
#pragma unroll
        for (int u = 0; u < MSG_BATCH; u++)
            if (u < cnt) {
                const float4 e = ee[u];
                const float z = (pv[u] + bmf) + Qj + (e.x * w0 - e.y * w1 - e.z * w2 - e.w * w3);
                dq += z > 0.f ? dv[u] : 0.f;
            }
    }
    dPQ[j * 128 + 64 + f] = dq;
}

// loss = mean (out - v/sV)^2 over 3n values; dout16 = 2 (out - v/sV)/(3n) in columns 0..2
__global__ __launch_bounds__(256) void k_loss(int64_t n, const int32_t *perm, const float *out16, const double *v,
                                              float sV, float *dout16, double *part)
{
    __shared__ double sh[256];
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (i < n) {
        for (int a = 0; a < 16; a++) {
            float d = 0.f;
            if (a < 3) {
                d = out16[16 * i + a] - (float)(v[3 * (int64_t)perm[i] + a] / sV);
                s += (double)d * (double)d;
                d = 2.f * d / (float)(3 * n);
            }
            dout16[16 * i + a] = d;
        }
    }
    s = block_sum_256(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// energy loss sums per block: (v_hat . Gamma v_hat, v_hat . F, v . F); v == nullptr
// leaves the third at zero (the warm-start energies need only the first two)
__global__ __launch_bounds__(256) void k_energy_parts(int64_t len, const double *vh, const double *q, const double *F,
                                                      const double *v, double *part)
{
    __shared__ double sh[256];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256) {
        a += vh[t] * q[t];
        b += vh[t] * F[t];
        if (v) c += v[t] * F[t];
    }
    a = block_sum_256(a, sh);
    b = block_sum_256(b, sh);
    c = block_sum_256(c, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = a;
        part[3 * blockIdx.x + 1] = b;
        part[3 * blockIdx.x + 2] = c;
    }
}

// s[k] = sum over blocks of part[3 b + k], in block order
__global__ void k_sum3(const double *part, int np, double *s)
{
    __shared__ double sh[256];
    for (int k = 0; k < 3; k++) {
        double a = 0.0;
        for (int b = threadIdx.x; b < np; b += 256) a += part[3 * b + k];
        a = block_sum_256(a, sh);
        if (threadIdx.x == 0) s[k] = a;
    }
}

// d loss / d out = 2 sV (Gamma v_hat - F) / (v . F) in columns 0..2
__global__ void k_energy_dout(int64_t n, const int32_t *perm, const double *q, const double *F, double sV,
                              const double *s, float *dout16)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    const double scale = 2.0 * sV / s[2];
    for (int a = 0; a < 16; a++)
        dout16[16 * i + a] = a < 3 ? (float)(scale * (q[3 * u + a] - F[3 * u + a])) : 0.f;
}

// The start of lowest energy E(x) = 0.5 x' Gamma x - x' F among v_prev, the
// network's guess and zero (E = 0), in that order of preference on ties
// (0: v_prev, 1: the network, 2: zero).  Lower energy is the smaller
// Gamma-norm error, since E(x) - E(v) = 0.5 ||x - v||^2_Gamma.
SGP_DEV int pick_start(double en, double ep)
{
    if (ep <= en && ep <= 0.0) return 0;
    return en <= 0.0 ? 1 : 2;
}

// x0 holds v_prev on entry
__global__ void k_pick(int64_t len, const double *s_net, const double *s_prev, const double *guess, double *x0)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= len) return;
    const double en = 0.5 * s_net[0] - s_net[1], ep = 0.5 * s_prev[0] - s_prev[1];
    const int k = pick_start(en, ep);
    if (k == 1) x0[t] = guess[t];
    if (k == 2) x0[t] = 0.0;
}

__global__ void k_sum_double(const double *part, int np, double *out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < np; k += 256) s += part[k];
    s = block_sum_256(s, sh);
    if (threadIdx.x == 0) *out = s;
}

__global__ void k_output(int64_t n, const int32_t *perm, const float *out16, double sV, double *vhat)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    for (int a = 0; a < 3; a++) vhat[3 * u + a] = sV * (double)out16[16 * i + a];
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
         int N, const float *bias, int acc, float *relu_out = nullptr)
{
    if (M <= 0) return SGP_OK;
    const int64_t nb = grid_for(M, GEMM_ROWS);
    hipStream_t st = ctx->stream;
    float *R = relu_out;
    switch (K) {
    case 16: k_gemm<1><<<nb, 256, 0, st>>>(A, lda, B, C, ldc, M, N, bias, acc, R); break;
    case 64: k_gemm<4><<<nb, 256, 0, st>>>(A, lda, B, C, ldc, M, N, bias, acc, R); break;
    case 128: k_gemm<8><<<nb, 256, 0, st>>>(A, lda, B, C, ldc, M, N, bias, acc, R); break;
    default: return set_err(ctx, SGP_EINVAL, "mpnn gemm: unsupported K");
    }
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

// out[0, L) = fixed-order sum of the G partial vectors part[g][0, L)
int reduce_parts(sgp_ctx ctx, sgp_mpnn M, const float *part, int G, int L, float *out)
{
    const int S = G < 32 ? G : 32;
    const int per = (G + S - 1) / S;
    const int segs = (G + per - 1) / per;
    float *tmp;
    SGP_TRY(ensure_t(ctx, M->red, (size_t)segs * L + 64, &tmp));
    k_red1<<<dim3((unsigned)grid_for(L, 256), (unsigned)segs), 256, 0, ctx->stream>>>(part, G, L, per, tmp);
    k_red2<<<grid_for(L, 256), 256, 0, ctx->stream>>>(tmp, segs, L, out);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

// A^T D (K x N) followed by the column sums of D (N), summed over all m rows,
// into M->sum; the caller copies windows of it into the gradient.
int gemm_at(sgp_ctx ctx, sgp_mpnn M, const float *A, int64_t lda, int K, const float *D, int64_t ldd, int N,
            int64_t m, float **sum)
{
    const int G = m > 0 ? (int)((m + AT_ROWS - 1) / AT_ROWS) : 1;
    const int L = K * N + N;
    float *part, *out;
    SGP_TRY(ensure_t(ctx, M->part, (size_t)G * L + 64, &part));
    SGP_TRY(ensure_t(ctx, M->sum, (size_t)L + 64, &out));
    hipStream_t st = ctx->stream;
    switch (K) {
    case 16: k_gemm_at<1><<<G, 256, 0, st>>>(A, lda, D, ldd, N, m, part); break;
    case 64: k_gemm_at<4><<<G, 256, 0, st>>>(A, lda, D, ldd, N, m, part); break;
    default: return set_err(ctx, SGP_EINVAL, "mpnn gemm_at: unsupported K");
    }
    LAUNCH_CHECK(ctx);
    SGP_TRY(reduce_parts(ctx, M, part, G, L, out));
    *sum = out;
    return SGP_OK;
}

int window(sgp_ctx ctx, const float *red, int off, int N, int r1, int c0, int c1, float *out, int64_t ld)
{
    k_window<<<grid_for((int64_t)r1 * (c1 - c0), 256), 256, 0, ctx->stream>>>(red, off, N, r1, c0, c1, out, ld);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

int prepare(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, const double *F, const double *vp, Act &A)
{
    const int64_t n = g->n, ne = 2 * g->m;
    float *base;
    float4 *ef;
    int32_t *irow, *icol, *deg;
    SGP_TRY(ensure_t(ctx, M->act, (size_t)act_floats(n) + 64, &base));
    SGP_TRY(ensure_t(ctx, M->efeat, (size_t)ne + 1, &ef));
    SGP_TRY(ensure_t(ctx, M->irow, (size_t)n + 2, &irow));
    SGP_TRY(ensure_t(ctx, M->icol, (size_t)ne + 1, &icol));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_DEG], (size_t)n + 2, &deg));
    A = carve(base, n);
    hipStream_t st = ctx->stream;
    const int32_t *perm = (const int32_t *)g->perm.p;
    k_input<<<grid_for(n, 256), 256, 0, st>>>(n, perm, F, vp, (float)M->sF, (float)M->sV, A.x16);
    LAUNCH_CHECK(ctx);
    // the internal neighbour lists depend only on the graph and sW: rebuilt
    // when either changed since the last call
    if (M->lists_of != g || M->lists_version != g->version || M->lists_sW != M->sW) {
        k_int_deg<<<grid_for(n, 256), 256, 0, st>>>(n, perm, (const int32_t *)g->rowptr.p, deg);
        LAUNCH_CHECK(ctx);
        SGP_TRY(scan_exclusive(ctx, deg, irow, n));
        k_int_entries<<<grid_for(16 * n, 256), 256, 0, st>>>(n, perm, (const int32_t *)g->inv.p,
                                                             (const int32_t *)g->rowptr.p, (const int32_t *)g->col.p,
                                                             (const int32_t *)g->ent_edge.p, (const double4 *)g->wu.p,
                                                             (float)M->sW, irow, icol, ef);
        LAUNCH_CHECK(ctx);
        M->lists_of = g;
        M->lists_version = g->version;
        M->lists_sW = M->sW;
    }
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
    const int32_t *rowptr = (const int32_t *)M->irow.p, *col = (const int32_t *)M->icol.p;   // internal order
    const float4 *ef = (const float4 *)M->efeat.p;
    // input layer: pre0 kept for the backward pass, h0 = relu(pre0) in the same pass
    SGP_TRY(gemm(ctx, A.x16, 16, W + PK.in16, A.pre0, 64, n, 16, 64, wr + L.b_in, 0, A.h[0]));
    for (int l = 0; l < NL; l++) {
        SGP_TRY(gemm(ctx, A.h[l], 64, W + PK.ab[l], A.PQ, 128, n, 64, 128, nullptr, 0));
        k_msg_fwd<<<grid_for(n, 16), 256, 0, st>>>(n, rowptr, col, ef, A.PQ, wr + L.b_m[l], wr + L.W_c[l], A.a[l]);
        if (n > 0)
            k_gemm_update<<<grid_for(n, GEMM_ROWS), 256, 0, st>>>(A.h[l], A.a[l], W + PK.u[l], wr + L.b_u[l], A.U[l],
                                                                  A.h[l + 1], n);
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
    const int32_t *rowptr = (const int32_t *)M->irow.p, *col = (const int32_t *)M->icol.p;   // internal order
    const float4 *ef = (const float4 *)M->efeat.p;
    float *S;
    // output layer: W_out rows 0..63 x columns 0..2 of h^T dout, b_out = column sums
    SGP_TRY(gemm_at(ctx, M, A.h[NL], 64, 64, A.dout16, 16, 16, n, &S));
    SGP_TRY(window(ctx, S, 0, 16, 64, 0, 3, G + L.W_out, 3));
    SGP_TRY(window(ctx, S, 64 * 16, 16, 1, 0, 3, G + L.b_out, 3));
    SGP_TRY(gemm(ctx, A.dout16, 16, W + PK.out16T, A.dh, 64, n, 16, 64, nullptr, 0));
    for (int l = NL - 1; l >= 0; l--) {
        k_mask<<<grid_for(64 * n, 256), 256, 0, st>>>(64 * n, A.dh, A.U[l], A.dU);
        SGP_TRY(gemm_at(ctx, M, A.h[l], 64, 64, A.dU, 64, 64, n, &S));
        SGP_TRY(window(ctx, S, 0, 64, 64, 0, 64, G + L.W_u[l], 64));
        SGP_TRY(window(ctx, S, 64 * 64, 64, 1, 0, 64, G + L.b_u[l], 64));
        SGP_TRY(gemm_at(ctx, M, A.a[l], 64, 64, A.dU, 64, 64, n, &S));
        SGP_TRY(window(ctx, S, 0, 64, 64, 0, 64, G + L.W_u[l] + 64 * 64, 64));
        SGP_TRY(gemm(ctx, A.dU, 64, W + PK.uT[l], A.dcat, 128, n, 64, 128, nullptr, 0));   // [dh part | da]
        // messages: recompute PQ of this layer from h[l]
        SGP_TRY(gemm(ctx, A.h[l], 64, W + PK.ab[l], A.PQ, 128, n, 64, 128, nullptr, 0));
        const int nb = (int)std::min<int64_t>(grid_for(n, 4), MSG_BWD_GRID);
        float *wcp;
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP9], (size_t)nb * 256 + 64, &wcp));
        k_msg_bwd_p<<<nb, 256, 0, st>>>(n, rowptr, col, ef, A.PQ, wr + L.b_m[l], wr + L.W_c[l], A.dcat + 64, 128,
                                        A.dPQ, wcp);
        k_msg_bwd_q<<<grid_for(n, 4), 256, 0, st>>>(n, rowptr, col, ef, A.PQ, wr + L.b_m[l], wr + L.W_c[l],
                                                    A.dcat + 64, 128, A.dPQ);
        LAUNCH_CHECK(ctx);
        SGP_TRY(reduce_parts(ctx, M, wcp, nb, 256, G + L.W_c[l]));   // W_c is 4 x 64 row-major
        // W_a, W_b = h^T dP, h^T dQ; b_m = column sums of dP
        SGP_TRY(gemm_at(ctx, M, A.h[l], 64, 64, A.dPQ, 128, 128, n, &S));
        SGP_TRY(window(ctx, S, 0, 128, 64, 0, 64, G + L.W_a[l], 64));
        SGP_TRY(window(ctx, S, 0, 128, 64, 64, 128, G + L.W_b[l], 64));
        SGP_TRY(window(ctx, S, 64 * 128, 128, 1, 0, 64, G + L.b_m[l], 64));
        // dh_l = dh (residual) + dcat[:, :64] + dPQ W_ab^T
        k_add64<<<grid_for(64 * n, 256), 256, 0, st>>>(n, A.dh, 64, A.dcat, 128, A.tmp, 64);
        LAUNCH_CHECK(ctx);
        SGP_TRY(gemm(ctx, A.dPQ, 128, W + PK.abT[l], A.tmp, 64, n, 128, 64, nullptr, 1));
        std::swap(A.dh, A.tmp);
    }
    k_mask<<<grid_for(64 * n, 256), 256, 0, st>>>(64 * n, A.dh, A.pre0, A.dU);
    SGP_TRY(gemm_at(ctx, M, A.x16, 16, 16, A.dU, 64, 64, n, &S));
    SGP_TRY(window(ctx, S, 0, 64, 6, 0, 64, G + L.W_in, 64));
    SGP_TRY(window(ctx, S, 16 * 64, 64, 1, 0, 64, G + L.b_in, 64));
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
    release(M->act); release(M->efeat); release(M->part); release(M->red); release(M->sum); release(M->vq);
    release(M->irow); release(M->icol);
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
    k_output<<<grid_for(g->n, 256), 256, 0, ctx->stream>>>(g->n, (const int32_t *)g->perm.p, A.out16, M->sV, vhat);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

// sums (x . Gamma x, x . F, v . F) of a canonical-order x into s[0..2]; q
// receives Gamma x.  Uses the library's product (workspaces of sgp_spmv).
static int energy_sums(sgp_ctx ctx, sgp_mpnn M, sgp_bsr A, const double *x, double *q, const double *F,
                       const double *v, double *s)
{
    const int64_t n = A->n;
    SGP_TRY(sgp_spmv(ctx, A, x, q));
    const int nb = (int)std::min<int64_t>(grid_for(3 * n, 256), 1024);
    double *part;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PART], (size_t)3 * nb + 8, &part));
    k_energy_parts<<<nb, 256, 0, ctx->stream>>>(3 * n, x, q, F, v, part);
    k_sum3<<<1, 256, 0, ctx->stream>>>(part, nb, s);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

static int loss_grad(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, sgp_bsr Gm, const double *F, const double *vprev,
                     const double *v, double *loss)
{
    Act A;
    const int64_t n = g->n;
    SGP_TRY(prepare(ctx, M, g, F, vprev, A));
    SGP_TRY(forward(ctx, M, g, A));
    double s[3];
    if (!Gm) {
        double *part;
        const int nb = (int)grid_for(n, 256);
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_PART], (size_t)nb + 8, &part));
        k_loss<<<nb, 256, 0, ctx->stream>>>(n, (const int32_t *)g->perm.p, A.out16, v, (float)M->sV, A.dout16, part);
        k_sum_double<<<1, 256, 0, ctx->stream>>>(part, nb, part + nb);
        LAUNCH_CHECK(ctx);
        SGP_TRY(backward(ctx, M, g, A));
        SGP_TRY(readback(ctx, s, part + nb, sizeof(double)));
        if (loss) *loss = s[0] / (3.0 * (double)n);
        return SGP_OK;
    }
    // energy loss (v_hat' G v_hat - 2 v_hat' F + v' F) / (v' F)
    double *vh, *ds;
    SGP_TRY(ensure_t(ctx, M->vq, (size_t)6 * n + 8, &vh));
    double *q = vh + 3 * n, *sd = vh + 6 * n;
    ds = sd;
    k_output<<<grid_for(n, 256), 256, 0, ctx->stream>>>(n, (const int32_t *)g->perm.p, A.out16, M->sV, vh);
    LAUNCH_CHECK(ctx);
    SGP_TRY(energy_sums(ctx, M, Gm, vh, q, F, v, ds));
    k_energy_dout<<<grid_for(n, 256), 256, 0, ctx->stream>>>(n, (const int32_t *)g->perm.p, q, F, M->sV, ds,
                                                            A.dout16);
    LAUNCH_CHECK(ctx);
    SGP_TRY(backward(ctx, M, g, A));
    SGP_TRY(readback(ctx, s, ds, sizeof s));
    if (loss) *loss = (s[0] - 2.0 * s[1] + s[2]) / s[2];
    return SGP_OK;
}

static int check_gamma(sgp_ctx ctx, sgp_graph g, sgp_bsr Gm)
{
    if (Gm && Gm->n != g->n) return set_err(ctx, SGP_EINVAL, "mpnn: Gamma and graph sizes differ");
    return SGP_OK;
}

extern "C" int sgp_mpnn_grad(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, sgp_bsr Gm, const double *F, const double *vprev,
                             const double *v, float *grad, double *loss)
{
    SGP_TRY(check_common(ctx, M, g, F, vprev));
    if (!v || !grad || g->n == 0) return set_err(ctx, SGP_EINVAL, "mpnn_grad: bad arguments");
    SGP_TRY(check_gamma(ctx, g, Gm));
    SGP_TRY(loss_grad(ctx, M, g, Gm, F, vprev, v, loss));
    HIP_TRY(ctx, hipMemcpyAsync(grad, M->grad.p, M->L.total * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
    return SGP_OK;
}

extern "C" int sgp_mpnn_train_step(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, sgp_bsr Gm, const double *F,
                                   const double *vprev, const double *v, double lr, double *loss)
{
    SGP_TRY(check_common(ctx, M, g, F, vprev));
    if (!v || g->n == 0 || !(lr > 0)) return set_err(ctx, SGP_EINVAL, "mpnn_train_step: bad arguments");
    SGP_TRY(check_gamma(ctx, g, Gm));
    SGP_TRY(loss_grad(ctx, M, g, Gm, F, vprev, v, loss));
    M->adam_t++;
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = 1.f - powf(b1, (float)M->adam_t), c2 = 1.f - powf(b2, (float)M->adam_t);
    k_adam<<<grid_for(M->L.total, 256), 256, 0, ctx->stream>>>(M->L.total, (float *)M->theta.p, (const float *)M->grad.p,
                                                              (float *)M->m1.p, (float *)M->m2.p, (float)lr, b1, b2,
                                                              1e-8f, c1, c2);
    LAUNCH_CHECK(ctx);
    return repack(ctx, M);
}

extern "C" int sgp_mpnn_warm_start(sgp_ctx ctx, sgp_mpnn M, sgp_graph g, sgp_bsr Gm, const double *F,
                                   const double *vprev, double *x0, int32_t *used_net, double *energy_net,
                                   double *energy_prev)
{
    SGP_TRY(check_common(ctx, M, g, F, vprev));
    if (!Gm || (g->n > 0 && !x0)) return set_err(ctx, SGP_EINVAL, "mpnn_warm_start: bad arguments");
    SGP_TRY(check_gamma(ctx, g, Gm));
    const int64_t n = g->n;
    if (n == 0) {
        if (used_net) *used_net = 0;
        if (energy_net) *energy_net = 0.0;
        if (energy_prev) *energy_prev = 0.0;
        return SGP_OK;
    }
    Act A;
    SGP_TRY(prepare(ctx, M, g, F, vprev, A));
    SGP_TRY(forward(ctx, M, g, A));
    double *vh;
    SGP_TRY(ensure_t(ctx, M->vq, (size_t)6 * n + 8, &vh));
    double *q = vh + 3 * n, *s = vh + 6 * n;   // s: 3 sums of the guess, 3 of v_prev (8 doubles reserved)
    k_output<<<grid_for(n, 256), 256, 0, ctx->stream>>>(n, (const int32_t *)g->perm.p, A.out16, M->sV, vh);
    LAUNCH_CHECK(ctx);
    SGP_TRY(energy_sums(ctx, M, Gm, vh, q, F, nullptr, s));
    SGP_TRY(energy_sums(ctx, M, Gm, vprev, q, F, nullptr, s + 3));
    if (x0 != vprev)
        HIP_TRY(ctx, hipMemcpyAsync(x0, vprev, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    k_pick<<<grid_for(3 * n, 256), 256, 0, ctx->stream>>>(3 * n, s, s + 3, vh, x0);
    LAUNCH_CHECK(ctx);
    double hs[6];
    SGP_TRY(readback(ctx, hs, s, sizeof hs));
    const double en = 0.5 * hs[0] - hs[1], ep = 0.5 * hs[3] - hs[4];
    // the host's choice repeats the kernel's comparisons on the same values
    if (used_net) *used_net = (ep <= en && ep <= 0.0) ? 0 : (en <= 0.0 ? 1 : 2);
    if (energy_net) *energy_net = en;
    if (energy_prev) *energy_prev = ep;
    return SGP_OK;
}
