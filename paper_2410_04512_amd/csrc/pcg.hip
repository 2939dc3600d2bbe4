// Section 1.1: preconditioned conjugate gradients on Gamma v = F, plus the
// 3x3-block CSR product that dominates each iteration.
//
// Left-preconditioned CG (the left form of the split preconditioning E^T
// Gamma E with H = E E^T = M^{-1}; Saad, Alg. 9.1):
//   r = F - Gamma x0, z = M^{-1} r, p = z, rho = r.z
//   repeat: q = Gamma p; alpha = rho / p.q; x += alpha p; r -= alpha q
//           stop if ||r|| / ||F|| <= rtol
//           z = M^{-1} r; rho' = r.z; p = z + (rho'/rho) p
//
// The launches of one iteration: the product (with the partials of p.q);
// alpha; r -= alpha q (with the partials of ||r||^2); z = M^{-1} r; the
// partials of r.z; one reduction for both ||r||^2 (the stopping rule) and
// rho' (beta); then x += alpha p and p = z + beta p in one pass, which reads
// p once for both.  The same values as the order above, bit for bit: x's
// update only moves later.  The stopping rule is thus applied after the
// sweeps of the last iteration instead of before them (one preconditioner
// application more per solve, for one reduction less per iteration).  A
// solve that stops normally is marked done = 3 ("finishing"): the last pass
// still adds alpha p to x but leaves p, and the next alpha reduction turns
// the mark into done = 1; every other kernel skips on any nonzero mark.
//
// Every scalar lives on the device.  Each dot product is a fixed-shape
// two-stage reduction (per-block partials in a fixed order, the last block of
// a cluster sums them in a fixed order), so results are bitwise reproducible.
// Clusters of a batched graph run independent CG recurrences: every launch
// covers all clusters, blocks never straddle two clusters, and a cluster that
// has converged skips its blocks.  The host only reads the "all done" state
// every few iterations.
#include "sgp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

// ---------------------------------------------------------------- block tables

struct BlockTab {
    const int32_t *row0, *row1, *inst;   // per block
    const int32_t *ifirst, *inb;         // per cluster: first block, number of blocks
};

// Vector kernels run 256 threads per block over VEC_ROWS rows, so a thread
// owns at most VEC_EPT of the block's 3 * VEC_ROWS elements (t, t+256, ...).
// Its loads are all issued before its first store (a store might alias a
// later element's load, so a plain loop would wait for every element in
// turn), unconditionally: a thread past the block's ne elements reloads
// element ne-1 (vec_idx) and drops the result.
constexpr int VEC_ROWS = 256;
constexpr int VEC_EPT = 3 * VEC_ROWS / 256;
// the tail's extra workgroups (SideX): at most one per CU but the tail's own
constexpr int SIDE_NWG = 255;
static_assert(3 * VEC_ROWS <= SIDE_BLOCK_VALUES, "a vector block must fit the tail's side update");

SGP_DEV int vec_idx(int u, int ne) { return min((int)threadIdx.x + 256 * u, ne - 1); }
SGP_DEV bool vec_own(int u, int ne) { return (int)threadIdx.x + 256 * u < ne; }

// host-side construction: clusters are cut into blocks of rows_per_block rows
static void build_tab(const std::vector<int64_t> &off, int rows_per_block, std::vector<int32_t> &buf,
                      int32_t &nblocks)
{
    int64_t K = (int64_t)off.size() - 1;
    std::vector<int32_t> r0, r1, in, f(K), nb(K);
    for (int64_t k = 0; k < K; k++) {
        f[k] = (int32_t)r0.size();
        int64_t a = off[k], b = off[k + 1];
        int32_t cnt = 0;
        for (int64_t s = a; s < b; s += rows_per_block) {
            r0.push_back((int32_t)s);
            r1.push_back((int32_t)std::min<int64_t>(s + rows_per_block, b));
            in.push_back((int32_t)k);
            cnt++;
        }
        if (cnt == 0) {   // empty cluster: one empty block keeps the reductions uniform
            r0.push_back((int32_t)a);
            r1.push_back((int32_t)a);
            in.push_back((int32_t)k);
            cnt = 1;
        }
        nb[k] = cnt;
    }
    nblocks = (int32_t)r0.size();
    buf.clear();
    buf.insert(buf.end(), r0.begin(), r0.end());
    buf.insert(buf.end(), r1.begin(), r1.end());
    buf.insert(buf.end(), in.begin(), in.end());
    buf.insert(buf.end(), f.begin(), f.end());
    buf.insert(buf.end(), nb.begin(), nb.end());
}

static BlockTab tab_ptrs(const int32_t *d, int32_t nblocks, int64_t K)
{
    BlockTab t;
    t.row0 = d;
    t.row1 = d + nblocks;
    t.inst = d + 2 * nblocks;
    t.ifirst = d + 3 * nblocks;
    t.inb = d + 3 * nblocks + K;
    return t;
}

// First stage of every reduction: the block's sum of one value per thread in
// a fixed order, stored as the block's partial.  The second stage is k_fin
// (one block per cluster, partials summed in block order), launched after the
// producer: the kernel boundary orders the two, so no fences or atomics.
SGP_DEV void block_partial(double v, int b, double *part, double *sh)
{
    double s = block_sum_256(v, sh);
    if (threadIdx.x == 0) part[b] = s;
}

enum { FIN_ALPHA, FIN_RR_BETA, FIN_RHO, FIN_INIT, FIN_TRUE, FIN_NORM2 };

// fixed-order sums of n partials by the FIN_THREADS threads of k_fin, for NA
// arrays (stride ns) at once: thread t owns the interleaved sequence t,
// t+FIN_THREADS, ...; position j of a pass of U * FIN_THREADS partials goes
// to running sum j mod U, and all U * NA loads of a pass are issued together
// (one pass covers the 1M-cell product's 10k partials), so the partials,
// just written by the producer, cost one round trip instead of one per
// FIN_THREADS.  Each thread adds its U sums pairwise, each wave folds its
// lanes by a butterfly and thread 0 adds the waves in order.  Results valid
// in thread 0.  sh holds NA * FIN_THREADS / 64 doubles.
constexpr int FIN_THREADS = 1024;

template <int NA>
SGP_DEV void sum_partials(const double *part, int64_t ns, int n, double *sh, double *res)
{
    constexpr int B = FIN_THREADS, U = NA == 1 ? 16 : NA == 2 ? 8 : 4;
    double acc[NA][U];
#pragma unroll
    for (int a = 0; a < NA; a++)
#pragma unroll
        for (int j = 0; j < U; j++) acc[a][j] = 0.0;
    for (int k = threadIdx.x; k < n; k += U * B) {
        double v[NA][U];
#pragma unroll
        for (int a = 0; a < NA; a++)
#pragma unroll
            for (int j = 0; j < U; j++) v[a][j] = k + j * B < n ? part[a * ns + k + j * B] : 0.0;
#pragma unroll
        for (int a = 0; a < NA; a++)
#pragma unroll
            for (int j = 0; j < U; j++) acc[a][j] = acc[a][j] + v[a][j];
    }
#pragma unroll
    for (int a = 0; a < NA; a++) {
#pragma unroll
        for (int h = U / 2; h > 0; h >>= 1)
#pragma unroll
            for (int j = 0; j < h; j++) acc[a][j] = acc[a][j] + acc[a][j + h];
        double v = acc[a][0];
        for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) sh[a * (B / 64) + (threadIdx.x >> 6)] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int a = 0; a < NA; a++) {
            double r = 0.0;
            for (int w = 0; w < B / 64; w++) r = r + sh[a * (B / 64) + w];
            res[a] = r;
        }
}

// Second stage: cluster k = blockIdx.x sums its partials (np values per block,
// stored as np arrays of stride nblk) and updates its scalars.
__global__ __launch_bounds__(FIN_THREADS) void k_fin(int op, const double *part, int nblk, const int32_t *ifirst,
                                                     const int32_t *inb, PcgScalars *S)
{
    __shared__ double sh[3 * FIN_THREADS / 64];
    const int k = blockIdx.x;
    PcgScalars *Sc = S + k;
    // the cluster's flag and its partials' range are loaded together (the
    // range does not depend on the flag), so the partials wait for one round
    // trip instead of two
    const int32_t dn = Sc->done;
    const int f = ifirst[k], nbk = inb[k];
    keep_loads_above();
    if (op != FIN_INIT && op != FIN_TRUE && op != FIN_NORM2 && dn) {
        // a finishing solve (its last x update has run): finished
        if (op == FIN_ALPHA && dn == 3 && threadIdx.x == 0) Sc->done = 1;
        return;
    }
    double t[3] = {0.0, 0.0, 0.0};
    if (op == FIN_INIT)
        sum_partials<3>(part + f, nblk, nbk, sh, t);
    else if (op == FIN_NORM2 || op == FIN_RR_BETA)
        sum_partials<2>(part + f, nblk, nbk, sh, t);
    else
        sum_partials<1>(part + f, nblk, nbk, sh, t);
    if (threadIdx.x != 0) return;
    const double t0 = t[0], t1 = t[1], t2 = t[2];
    switch (op) {
    case FIN_ALPHA:
        Sc->pq = t0;
        if (!(t0 > 0.0) || !isfinite(t0)) {
            Sc->status = SGP_EBREAKDOWN;
            Sc->done = 1;
        } else {
            Sc->alpha = Sc->rho / t0;
        }
        break;
    case FIN_RR_BETA: {   // t0 = ||r||^2, t1 = r.z
        Sc->rr = t0;
        Sc->iter = Sc->iter + 1;
        Sc->relres2 = t0 / Sc->nF2;
        if (!isfinite(t0)) {
            Sc->status = SGP_ENONFINITE;
            Sc->done = 1;
            break;
        }
        bool conv;
        if (Sc->stop == SGP_STOP_ERROR) {
            // the Gauss-Radau bound of the energy error after this step
            const double a = Sc->alpha, beta = t1 / Sc->rho;
            Sc->gs = Sc->gs + a * Sc->rho;
            Sc->phi = (Sc->phi - a) / (Sc->mu * (Sc->phi - a) + beta);
            Sc->gbound = Sc->phi * t1;
            conv = Sc->gbound <= Sc->tol2 * (Sc->gs + Sc->gbound);
        } else {
            conv = Sc->relres2 <= Sc->tol2;
        }
        bool stop = false;
        if (Sc->fixed) {
            stop = Sc->iter >= Sc->fixed;
        } else if (conv) {
            stop = true;
        } else if (Sc->iter >= Sc->max_iter) {
            Sc->status = SGP_ENOCONV;
            stop = true;
        }
        Sc->beta = t1 / Sc->rho;
        Sc->rho = t1;
        if (stop) Sc->done = 3;
        break;
    }
    case FIN_RHO:
        Sc->rho = t0;
        if (Sc->stop == SGP_STOP_ERROR) {
            Sc->phi = 1.0 / Sc->mu;
            Sc->gs = 0.0;
            Sc->gbound = Sc->phi * t0;
        }
        break;
    case FIN_INIT:   // t0 = ||F||^2, t1 = ||r||^2, t2 = bad-input count
        Sc->nF2 = t0;
        Sc->rr = t1;
        Sc->iter = 0;
        Sc->relres2 = t0 > 0.0 ? t1 / t0 : 0.0;
        if (t2 != 0.0 || !isfinite(t1)) {
            Sc->status = SGP_ENONFINITE;
            Sc->done = 1;
        } else if (t0 == 0.0) {
            Sc->done = 2;   // zero force: v = 0
        } else if (!Sc->fixed && (Sc->stop == SGP_STOP_ERROR ? Sc->tol2 >= 1.0 : Sc->relres2 <= Sc->tol2)) {
            Sc->done = 1;   // (from x0 = 0 the relative energy error is 1)
        }
        break;
    case FIN_TRUE:
        Sc->rz = t0;
        break;
    case FIN_NORM2:
        Sc->rz = t0;    // ||r||^2
        Sc->nF2 = t1;   // ||F||^2
        break;
    }
}

// ---------------------------------------------------------------- vector kernels

// rows of block b of a row table (blocks never straddle clusters)
SGP_DEV bool block_rows(const BlockTab &tab, int b, int64_t &row, int &inst)
{
    inst = tab.inst[b];
    row = tab.row0[b] + threadIdx.x;
    return row < tab.row1[b];
}

// r = F - q (q = Gamma x0) or r = F (x = 0); partials of ||F||^2, ||r||^2, #bad
template <class T>
__global__ __launch_bounds__(256) void k_init_res(const double *F, const T *q, T *x, T *r, int use_x0, BlockTab tab,
                                                  double *part)
{
    __shared__ double sh[256];
    int b = blockIdx.x, inst;
    int64_t row;
    bool ok = block_rows(tab, b, row, inst);
    double ff = 0.0, rr = 0.0, bad = 0.0;
    if (ok) {
        for (int a = 0; a < 3; a++) {
            double f = F[3 * row + a];
            T ri;
            if (use_x0) {
                ri = (T)f - q[3 * row + a];
                if (!isfinite((double)x[3 * row + a])) bad = 1.0;
            } else {
                ri = (T)f;
                x[3 * row + a] = 0;
            }
            r[3 * row + a] = ri;
            if (!isfinite(f)) bad = 1.0;
            ff = ff + f * f;
            rr = rr + (double)ri * (double)ri;
        }
    }
    block_partial(ff, b, part, sh);
    block_partial(rr, b, part + gridDim.x, sh);
    block_partial(bad, b, part + 2 * gridDim.x, sh);
}

// p = z; partial of r.z
template <class T>
__global__ __launch_bounds__(256) void k_init_p(const T *r, const T *z, T *p, BlockTab tab, const PcgScalars *S,
                                                double *part)
{
    __shared__ double sh[256];
    int b = blockIdx.x, inst;
    int64_t row;
    bool ok = block_rows(tab, b, row, inst);
    if (S[inst].done) return;
    double rz = 0.0;
    if (ok) {
        for (int a = 0; a < 3; a++) {
            T zi = z[3 * row + a];
            p[3 * row + a] = zi;
            rz = rz + (double)r[3 * row + a] * (double)zi;
        }
    }
    block_partial(rz, b, part, sh);
}

// Element range of a block: the 3 (row1 - row0) values of its rows, walked
// flat (thread t takes elements t, t + 256, t + 512 of the range), so every
// load instruction of a wave reads 512 contiguous bytes.
SGP_DEV int block_elems(const BlockTab &tab, int b, int64_t &e0, int &inst)
{
    inst = tab.inst[b];
    e0 = 3 * (int64_t)tab.row0[b];
    return 3 * (tab.row1[b] - tab.row0[b]);
}

// r -= alpha q; partial of ||r||^2
template <class T>
__global__ __launch_bounds__(256) void k_update_r(T *r, const T *q, BlockTab tab, const PcgScalars *S, double *part)
{
    __shared__ double sh[256];
    int inst;
    int64_t e0;
    const int ne = block_elems(tab, blockIdx.x, e0, inst);
    const PcgScalars *Sc = S + inst;
    if (Sc->done) return;
    const T alpha = (T)Sc->alpha;
    double rr = 0.0;
    if (ne > 0) {
        T rv[VEC_EPT], qv[VEC_EPT];
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++) {
            rv[u] = r[e0 + vec_idx(u, ne)];
            qv[u] = q[e0 + vec_idx(u, ne)];
        }
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++)
            if (vec_own(u, ne)) {
                const T ri = rv[u] - alpha * qv[u];
                r[e0 + vec_idx(u, ne)] = ri;
                rr = rr + (double)ri * (double)ri;
            }
    }
    block_partial(rr, blockIdx.x, part, sh);
}

// partial of p.q (batched solves: the product itself has no cluster split)
template <class T>
__global__ __launch_bounds__(256) void k_pq(const T *p, const T *q, BlockTab tab, const PcgScalars *S, double *part)
{
    __shared__ double sh[256];
    int inst;
    int64_t e0;
    const int ne = block_elems(tab, blockIdx.x, e0, inst);
    if (S[inst].done) return;
    double d = 0.0;
    if (ne > 0) {
        T pv[VEC_EPT], qv[VEC_EPT];
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++) {
            pv[u] = p[e0 + vec_idx(u, ne)];
            qv[u] = q[e0 + vec_idx(u, ne)];
        }
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++)
            if (vec_own(u, ne)) d = d + (double)pv[u] * (double)qv[u];
    }
    block_partial(d, blockIdx.x, part, sh);
}

// partial of r.z
template <class T>
__global__ __launch_bounds__(256) void k_rz(const T *r, const T *z, BlockTab tab, const PcgScalars *S, double *part)
{
    __shared__ double sh[256];
    int inst;
    int64_t e0;
    const int ne = block_elems(tab, blockIdx.x, e0, inst);
    if (S[inst].done) return;
    double rz = 0.0;
    if (ne > 0) {
        T rv[VEC_EPT], zv[VEC_EPT];
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++) {
            rv[u] = r[e0 + vec_idx(u, ne)];
            zv[u] = z[e0 + vec_idx(u, ne)];
        }
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++)
            if (vec_own(u, ne)) rz = rz + (double)rv[u] * (double)zv[u];
    }
    block_partial(rz, blockIdx.x, part, sh);
}

// The first elimination step of a tree preconditioner inside the two vector
// passes around the sweeps.  Its vertices are the elimination positions
// 0..q1-1, ascending in the internal order, so the block of rows of a vector
// kernel holds the positions qr[2b]..qr[2b+1]-1 (at most one per thread).
// r -= alpha q is followed by that step's forward substitution (the work of
// k_fwd_step0), and r.z is preceded by its backward substitution (that of
// k_bwd_step0), with r and z of the block's rows taken from LDS instead of
// gathered: the same operations on the same values as the separate launches,
// so results are bitwise unchanged.
template <class T>
struct Step0Tab {
    const int32_t *qr, *elim, *tout, *upq;
    const T *wu, *Dinv;
    T *y, *cs;
    int64_t ws;   // offset of the second (w, u) plane
    T gpar, gperp, gmed;
};

// the positions of block b: qr[2b] = first position whose vertex is >= row0,
// qr[2b + 1] the same for row1 (binary search over the ascending vertices)
__global__ void k_step0_ranges(int32_t nb, BlockTab tab, const int32_t *elim, int32_t q1, int32_t *qr)
{
    const int32_t b = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b >= nb) return;
    for (int k = 0; k < 2; k++) {
        const int32_t row = k == 0 ? tab.row0[b] : tab.row1[b];
        int32_t lo = 0, hi = q1;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (elim[mid] < row)
                lo = mid + 1;
            else
                hi = mid;
        }
        qr[2 * b + k] = lo;
    }
}

// r -= alpha q with the partial of ||r||^2, then the forward substitution of
// the block's first-step vertices: y = P_qq^{-1} r and its pushes (y itself
// is formed again by k_rz_s0)
template <class T>
__global__ __launch_bounds__(256) void k_update_r_s0(T *r, const T *q, BlockTab tab, const PcgScalars *S,
                                                     double *part, Step0Tab<T> t)
{
    __shared__ double sh[256];
    __shared__ T rl[3 * VEC_ROWS];
    int inst;
    int64_t e0;
    // XCD-contiguous rows: the pushes of an XCD's blocks land in one region
    const int b = (int)xcd_block(blockIdx.x, gridDim.x);
    const int ne = block_elems(tab, b, e0, inst);
    const PcgScalars *Sc = S + inst;
    if (Sc->done) return;
    const int32_t qa = t.qr[2 * b], qb = t.qr[2 * b + 1];
    T rv[VEC_EPT], qx[VEC_EPT];
    if (ne > 0) {
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++) {
            rv[u] = r[e0 + vec_idx(u, ne)];
            // q's last read (non-temporal: r and the sweeps' data stay cached)
            qx[u] = __builtin_nontemporal_load(q + e0 + vec_idx(u, ne));
        }
    }
    // this thread's first-step vertex (a thread without one reads position 0
    // and computes nothing)
    const int32_t qs = qa + (int32_t)threadIdx.x;
    const bool mine = qs < qb;
    const int32_t qc = mine ? qs : 0;
    const int64_t v = t.elim[qc];
    const int32_t to0 = t.tout[2 * qc], to1 = t.tout[2 * qc + 1];
    T w0[4], w1[4], d[6];
    for (int k = 0; k < 4; k++) w0[k] = t.wu[4 * (int64_t)qc + k];
    if (to1 >= 0) {   // a compressed vertex: second contact and stored pivot
        for (int k = 0; k < 4; k++) w1[k] = t.wu[t.ws + 4 * (int64_t)qc + k];
        for (int k = 0; k < 6; k++) d[k] = t.Dinv[6 * (int64_t)qc + k];
    }
    const T alpha = (T)Sc->alpha;
    double rr = 0.0;
    if (ne > 0) {
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++)
            if (vec_own(u, ne)) {
                const T ri = rv[u] - alpha * qx[u];
                r[e0 + vec_idx(u, ne)] = ri;
                rl[threadIdx.x + 256 * u] = ri;
                rr = rr + (double)ri * (double)ri;
            }
    }
    __syncthreads();
    if (mine) {
        const int64_t i = 3 * (v - e0 / 3);
        const T b0 = rl[i], b1 = rl[i + 1], b2 = rl[i + 2];
        T o0, o1, o2;
        if (to1 >= 0)
            sym_mv(d, b0, b1, b2, o0, o1, o2);
        else
            leaf_pivot_solve(w0, t.gpar, t.gperp, t.gmed, b0, b1, b2, o0, o1, o2);
        // y = P_qq^{-1} r is not stored: the backward pass forms it again
        // from the same r
        if (to0 >= 0) {
            T *c = t.cs + 3 * (int64_t)to0;
            neg_w_mv(w0, t.gpar, t.gperp, o0, o1, o2, c[0], c[1], c[2]);
        }
        if (to1 >= 0) {
            T *c = t.cs + 3 * (int64_t)to1;
            neg_w_mv(w1, t.gpar, t.gperp, o0, o1, o2, c[0], c[1], c[2]);
        }
    }
    block_partial(rr, b, part, sh);
}

// the backward substitution of the block's first-step vertices, x =
// y - P_qq^{-1} (sum over up-links of W x), written to z; then the partial of
// r.z over the block's rows
template <class T>
__global__ __launch_bounds__(256) void k_rz_s0(const T *r, T *z, BlockTab tab, const PcgScalars *S, double *part,
                                               Step0Tab<T> t)
{
    __shared__ double sh[256];
    __shared__ T zl[3 * VEC_ROWS], rl[3 * VEC_ROWS];
    int inst;
    int64_t e0;
    // XCD-contiguous rows: the up-links an XCD's blocks read stay in its L2
    const int b = (int)xcd_block(blockIdx.x, gridDim.x);
    const int ne = block_elems(tab, b, e0, inst);
    if (S[inst].done) return;
    const int32_t qa = t.qr[2 * b], qb = t.qr[2 * b + 1];
    T rv[VEC_EPT], zv[VEC_EPT];
    if (ne > 0) {
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++) {
            rv[u] = r[e0 + vec_idx(u, ne)];
            zv[u] = z[e0 + vec_idx(u, ne)];
        }
    }
    const int32_t qs = qa + (int32_t)threadIdx.x;
    const bool mine = qs < qb;
    const int32_t qc = mine ? qs : 0;
    const int32_t a0 = t.upq[2 * qc], a1 = t.upq[2 * qc + 1];
    const int64_t v = t.elim[qc];
    T w0[4], w1[4], d[6];
    for (int k = 0; k < 4; k++) w0[k] = t.wu[4 * (int64_t)qc + k];
    const int64_t u0 = a0 >= 0 ? a0 : qc, u1 = a1 >= 0 ? a1 : qc;
    const T p0 = t.y[3 * u0], p1 = t.y[3 * u0 + 1], p2 = t.y[3 * u0 + 2];
    const T x0 = t.y[3 * u1], x1 = t.y[3 * u1 + 1], x2 = t.y[3 * u1 + 2];
    if (a1 >= 0) {
        for (int k = 0; k < 4; k++) w1[k] = t.wu[t.ws + 4 * (int64_t)qc + k];
        for (int k = 0; k < 6; k++) d[k] = t.Dinv[6 * (int64_t)qc + k];
    }
    keep_loads_above();
    // z of the block's rows as the sweeps left them (the first-step rows are
    // overwritten below), and r
    if (ne > 0) {
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++)
            if (vec_own(u, ne)) {
                zl[threadIdx.x + 256 * u] = zv[u];
                rl[threadIdx.x + 256 * u] = rv[u];
            }
    }
    __syncthreads();
    if (mine) {
        // the forward substitution's y = P_qq^{-1} r again (a first-step
        // vertex has no in-slots), in the same operations
        const int64_t i = 3 * (v - e0 / 3);
        T y0, y1, y2;
        if (a1 >= 0)
            sym_mv(d, rl[i], rl[i + 1], rl[i + 2], y0, y1, y2);
        else
            leaf_pivot_solve(w0, t.gpar, t.gperp, t.gmed, rl[i], rl[i + 1], rl[i + 2], y0, y1, y2);
        T c0 = 0, c1 = 0, c2 = 0;
        if (a0 >= 0) {
            T e0_, e1_, e2_;
            neg_w_mv(w0, t.gpar, t.gperp, p0, p1, p2, e0_, e1_, e2_);
            c0 = c0 + e0_;
            c1 = c1 + e1_;
            c2 = c2 + e2_;
        }
        if (a1 >= 0) {
            T e0_, e1_, e2_;
            neg_w_mv(w1, t.gpar, t.gperp, x0, x1, x2, e0_, e1_, e2_);
            c0 = c0 + e0_;
            c1 = c1 + e1_;
            c2 = c2 + e2_;
        }
        T s0, s1, s2;
        if (a1 >= 0)
            sym_mv(d, c0, c1, c2, s0, s1, s2);
        else
            leaf_pivot_solve(w0, t.gpar, t.gperp, t.gmed, c0, c1, c2, s0, s1, s2);
        const T n0 = y0 - s0, n1 = y1 - s1, n2 = y2 - s2;
        z[3 * v] = n0;
        z[3 * v + 1] = n1;
        z[3 * v + 2] = n2;
        zl[i] = n0;
        zl[i + 1] = n1;
        zl[i + 2] = n2;
    }
    __syncthreads();
    double rz = 0.0;
    if (ne > 0) {
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++)
            if (vec_own(u, ne)) rz = rz + (double)rv[u] * (double)zl[threadIdx.x + 256 * u];
    }
    block_partial(rz, b, part, sh);
}

// x += alpha p, then p = z + beta p (p only while the solve goes on)
template <class T>
__global__ __launch_bounds__(256) void k_update_xp(T *x, T *p, const T *z, BlockTab tab, const PcgScalars *S)
{
    int inst;
    int64_t e0;
    const int ne = block_elems(tab, blockIdx.x, e0, inst);
    const PcgScalars *Sc = S + inst;
    const int32_t dn = Sc->done;
    if ((dn != 0 && dn != 3) || ne == 0) return;
    const T alpha = (T)Sc->alpha;
    T xv[VEC_EPT], pv[VEC_EPT];
#pragma unroll
    for (int u = 0; u < VEC_EPT; u++) {
        xv[u] = x[e0 + vec_idx(u, ne)];
        pv[u] = p[e0 + vec_idx(u, ne)];
    }
    if (dn == 3) {   // finishing: the last x update only
#pragma unroll
        for (int u = 0; u < VEC_EPT; u++)
            if (vec_own(u, ne)) x[e0 + vec_idx(u, ne)] = xv[u] + alpha * pv[u];
        return;
    }
    const T beta = (T)Sc->beta;
    T zv[VEC_EPT];
#pragma unroll
    for (int u = 0; u < VEC_EPT; u++) zv[u] = z[e0 + vec_idx(u, ne)];
#pragma unroll
    for (int u = 0; u < VEC_EPT; u++)
        if (vec_own(u, ne)) {
            x[e0 + vec_idx(u, ne)] = xv[u] + alpha * pv[u];
            p[e0 + vec_idx(u, ne)] = zv[u] + beta * pv[u];
        }
}

// p = z + beta p, where x += alpha p ran during the tree sweeps (SideX): a
// finishing solve has nothing left to do
template <class T>
__global__ __launch_bounds__(256) void k_update_p(T *p, const T *z, BlockTab tab, const PcgScalars *S)
{
    int inst;
    int64_t e0;
    const int ne = block_elems(tab, blockIdx.x, e0, inst);
    const PcgScalars *Sc = S + inst;
    T pv[VEC_EPT], zv[VEC_EPT];
#pragma unroll
    for (int u = 0; u < VEC_EPT; u++) {
        pv[u] = p[e0 + vec_idx(u, ne)];
        // z's last read in an iteration: non-temporal, so that it does not
        // displace p, which the product gathers next
        zv[u] = __builtin_nontemporal_load(z + e0 + vec_idx(u, ne));
    }
    if (Sc->done || ne == 0) return;
    const T beta = (T)Sc->beta;
#pragma unroll
    for (int u = 0; u < VEC_EPT; u++)
        if (vec_own(u, ne)) p[e0 + vec_idx(u, ne)] = zv[u] + beta * pv[u];
}

// partial of ||F - q||^2 (q = Gamma x)
__global__ __launch_bounds__(256) void k_true_res(const double *F, const double *q, BlockTab tab, double *part)
{
    __shared__ double sh[256];
    int b = blockIdx.x, inst;
    int64_t row;
    bool ok = block_rows(tab, b, row, inst);
    double rr = 0.0;
    if (ok)
        for (int a = 0; a < 3; a++) {
            double t = F[3 * row + a] - q[3 * row + a];
            rr = rr + t * t;
        }
    block_partial(rr, b, part, sh);
}

template <class T>
__global__ void k_zero_rows(T *x, BlockTab tab, const PcgScalars *S, int want_done)
{
    int b = blockIdx.x, inst;
    int64_t row;
    bool ok = block_rows(tab, b, row, inst);
    if (!ok || S[inst].done != want_done) return;
    x[3 * row] = 0;
    x[3 * row + 1] = 0;
    x[3 * row + 2] = 0;
}

__global__ void k_set_scalars(PcgScalars *S, int64_t K, double tol2, int fixed, int max_iter, int stop = 0,
                              double mu = 1.0)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    PcgScalars s = {};
    s.tol2 = tol2;
    s.fixed = fixed;
    s.max_iter = max_iter;
    s.stop = stop;
    s.mu = mu;
    S[k] = s;
}

// open[0]: clusters not done; open[1]: iterations of cluster 0; open[2..3]:
// the largest (||r||^2 / ||F||^2) / tol^2 of the open clusters, as the bits
// of a double (zeroed before the launch; positive doubles order as their
// bits, so an integer maximum picks the largest)
__global__ void k_any_open(const PcgScalars *S, int64_t K, int32_t *open)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K && !S[k].done) {
        atomicAdd(open, 1);
        // the stopping quantity over its target (squared)
        const double g = S[k].gs + S[k].gbound;
        const double e2 = S[k].stop == SGP_STOP_ERROR ? (g > 0.0 ? S[k].gbound / g : 1.0) : S[k].relres2;
        const double q = S[k].tol2 > 0.0 ? e2 / S[k].tol2 : 0.0;
        if (q > 0.0 && isfinite(q))
            atomicMax((unsigned long long *)(open + 2), (unsigned long long)__double_as_longlong(q));
    }
    if (k == 0) open[1] = S[0].iter;
}

// rowptr at the cluster offsets (block offsets of the clusters)
__global__ void k_gather_rowptr(const int32_t *rowptr, const int64_t *off, int64_t K1, int32_t *out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K1) out[k] = rowptr[off[k]];
}

// ---------------------------------------------------------------- the solver state

struct PcgWork {
    std::vector<int32_t> vec_buf;
    int32_t vec_nb = 0;
    BlockTab vec;
    int32_t mv_nb = 0;                   // product workgroups (one cluster: p.q partials)
    const int32_t *mv_first = nullptr;   // {0}
    const int32_t *mv_nb_dev = nullptr;  // {mv_nb}
    int64_t K = 1;
    int32_t s0_q1 = 0;               // > 0: the first elimination step runs in the vector passes
    const int32_t *s0_qr = nullptr;  // its positions per vector block
};

template <class T>
static int spmv_t(sgp_ctx ctx, sgp_bsr A, const T *x, T *y, const PcgScalars *S, double *part, int mode);
template <>
int spmv_t<double>(sgp_ctx ctx, sgp_bsr A, const double *x, double *y, const PcgScalars *S, double *part, int mode)
{
    return spmv_f64(ctx, A, x, y, S, part, mode);
}
template <>
int spmv_t<float>(sgp_ctx ctx, sgp_bsr A, const float *x, float *y, const PcgScalars *S, double *part, int mode)
{
    return spmv_f32(ctx, A, x, y, S, part, mode);
}


template <class T>
struct Vecs {
    T *x, *r, *z, *p, *q;
};

// the first step's tables of M in precision T
template <class T>
static Step0Tab<T> step0_tab(sgp_prec M, const PcgWork &w)
{
    const bool f64 = sizeof(T) == 8;
    Step0Tab<T> t;
    t.qr = w.s0_qr;
    t.elim = (const int32_t *)M->elim_int.p;
    t.tout = (const int32_t *)M->tout.p;
    t.upq = (const int32_t *)M->up.p;
    t.wu = (const T *)(f64 ? M->wu0.p : M->wu032.p);
    t.Dinv = (const T *)(f64 ? M->Dinv.p : M->Dinv32.p);
    t.y = (T *)(f64 ? M->y.p : M->y32.p);
    t.cs = (T *)(f64 ? M->cs.p : M->cs32.p);
    t.ws = 4 * (int64_t)w.s0_q1;
    t.gpar = (T)M->gpar;
    t.gperp = (T)M->gperp;
    t.gmed = (T)M->gmed;
    return t;
}

static int fin(sgp_ctx ctx, int op, const double *part, int nblk, const int32_t *ifirst, const int32_t *inb,
               PcgScalars *S, int64_t K)
{
    k_fin<<<(unsigned)K, FIN_THREADS, 0, ctx->stream>>>(op, part, nblk, ifirst, inb, S);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

// CG iterations per timed product (at most one per chunk)
constexpr int KT_STRIDE = 4;

// PCG iterations on prepared r, z (z = M r) and p, until every cluster is done.
// `count` CG iterations, launched on ctx->stream (no host synchronisation,
// allocation or memset inside, so the sequence can be captured into a graph).
// Every kernel returns at once for a converged cluster, so iterations issued
// past convergence change nothing.
template <class T>
static int pcg_chunk(sgp_ctx ctx, sgp_bsr A, sgp_prec M, Vecs<T> v, PcgWork &w, PcgScalars *S, double *part,
                     int count, int it0 = 0)
{
    hipStream_t st = ctx->stream;
    const int64_t K = w.K;
    // one cluster: the sweeps stop with it; several: every sweep runs
    PcgScalars *gate = K == 1 ? S : nullptr;
    for (int c = 0; c < count; c++) {
        // kernel timing: one product in every KT_STRIDE iterations carries a
        // pair of events on its own launch, the third of a chunk that starts
        // a new stride
        const bool timed = c == std::min(2, count - 1) && it0 % KT_STRIDE < count;
        if (timed) SGP_TRY(ktimer_begin(ctx, it0 + c));
        if (K == 1) {
            SGP_TRY(spmv_t<T>(ctx, A, v.p, v.q, S, part, 1));
            if (timed) SGP_TRY(ktimer_end(ctx));
            SGP_TRY(fin(ctx, FIN_ALPHA, part, w.mv_nb, w.mv_first, w.mv_nb_dev, S, 1));
        } else {
            SGP_TRY(spmv_t<T>(ctx, A, v.p, v.q, nullptr, nullptr, 0));
            if (timed) SGP_TRY(ktimer_end(ctx));
            k_pq<T><<<w.vec_nb, 256, 0, st>>>(v.p, v.q, w.vec, S, part);
            SGP_TRY(fin(ctx, FIN_ALPHA, part, w.vec_nb, w.vec.ifirst, w.vec.inb, S, K));
        }
        // partials: ||r||^2 in the first nb entries, r.z in the next nb
        const bool s0 = M && w.s0_q1 > 0;
        if (s0)
            k_update_r_s0<T><<<w.vec_nb, 256, 0, st>>>(v.r, v.q, w.vec, S, part, step0_tab<T>(M, w));
        else
            k_update_r<T><<<w.vec_nb, 256, 0, st>>>(v.r, v.q, w.vec, S, part);
        // x += alpha p by extra workgroups of the sweeps' one-workgroup tail
        // launch, when there is one (knob tail_side)
        SideX side = {v.x, v.p, w.vec.row0, w.vec.row1, w.vec.inst, S, w.vec_nb,
                      std::min(SIDE_NWG, (w.vec_nb + 3) / 4), false};
        SideX *sx = ctx->tail_side ? &side : nullptr;
        if (M) {
            if (sizeof(T) == 8)
                SGP_TRY(prec_apply_f64(ctx, M, (const double *)v.r, (double *)v.z, gate, s0, sx));
            else
                SGP_TRY(prec_apply_f32(ctx, M, (const float *)v.r, (float *)v.z, gate, s0, sx));
        }
        if (s0)
            k_rz_s0<T><<<w.vec_nb, 256, 0, st>>>(v.r, v.z, w.vec, S, part + w.vec_nb, step0_tab<T>(M, w));
        else
            k_rz<T><<<w.vec_nb, 256, 0, st>>>(v.r, v.z, w.vec, S, part + w.vec_nb);
        SGP_TRY(fin(ctx, FIN_RR_BETA, part, w.vec_nb, w.vec.ifirst, w.vec.inb, S, K));
        if (side.ran)
            k_update_p<T><<<w.vec_nb, 256, 0, st>>>(v.p, v.z, w.vec, S);
        else
            k_update_xp<T><<<w.vec_nb, 256, 0, st>>>(v.x, v.p, v.z, w.vec, S);
        LAUNCH_CHECK(ctx);
    }
    return SGP_OK;
}

// an instantiated graph of one chunk, destroyed with the solve
struct ChunkGraph {
    hipGraphExec_t exec = nullptr;
    ~ChunkGraph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

// capture `count` iterations on the context's private stream (capture only
// records; nothing runs until the graph is launched on ctx->stream)
template <class T>
static int capture_chunk(sgp_ctx ctx, sgp_bsr A, sgp_prec M, Vecs<T> v, PcgWork &w, PcgScalars *S, double *part,
                         int count, ChunkGraph &g)
{
    if (!ctx->cap_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    ctx->stream = ctx->cap_stream;
    hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? pcg_chunk<T>(ctx, A, M, v, w, S, part, count) : SGP_EHIP;
    hipGraph_t graph = nullptr;
    hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(ctx->cap_stream, &graph) : e;
    ctx->stream = saved;
    if (rc != SGP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e2 != hipSuccess) return set_err(ctx, SGP_EHIP, "graph capture failed: %s", hipGetErrorString(e2));
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        g.exec = nullptr;
        return set_err(ctx, SGP_EHIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    return SGP_OK;
}

template <class T>
static int pcg_iterate(sgp_ctx ctx, sgp_bsr A, sgp_prec M, Vecs<T> v, PcgWork &w, PcgScalars *S,
                       double *part, int32_t *open, int check_every, int max_iter, int fixed)
{
    hipStream_t st = ctx->stream;
    int32_t *hopen = (int32_t *)ctx->pinned;
    const int64_t K = w.K;
    const int limit = fixed > 0 ? fixed : max_iter;
    // graph replay of whole chunks (not while per-launch timing records events)
    const bool graph = ctx->use_graph && !ctx->ktiming && ctx->plan_mode == PLAN_OFF;
    ChunkGraph cg;
    // Chunks issued between two polls of the host.  A fixed iteration count
    // needs no poll before its end.  Otherwise, after two polls, the decay per
    // iteration of log(||r||^2 / (tol ||F||)^2) (or of the squared relative
    // error bound over tol^2, when that stops the solve) of the slowest open cluster
    // predicts the iterations it still needs, and the next poll comes after
    // half of them (whole chunks, at least one): polls thin out while the
    // solve is far from the tolerance, and iterations issued past
    // convergence stay within a chunk.  CG's residual is not monotone: where
    // it stalls, the prediction runs away, so a poll never waits for more
    // than a quarter of the iterations done so far (at least 8).
    int per_poll = fixed > 0 ? (limit + check_every - 1) / check_every : 1;
    int it_prev = -1;
    double lg_prev = 0.0;
    // Look-ahead: while the host waits for a poll's flags, the GPU runs one
    // more chunk, issued right after the poll (every kernel returns at once
    // for a cluster that has converged), so a poll leaves the GPU no idle
    // gap.  Not while a step is recorded or captured, whose readbacks are
    // replayed in order, nor for a fixed count (no poll before its end).
    const bool ahead = ctx->plan_mode == PLAN_OFF && fixed == 0;
    if (ahead && !ctx->poll_ev) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->poll_ev, hipEventDisableTiming));
    int it = 0;                // iterations issued
    bool issued_ahead = false;   // the current group's first chunk went out with the last poll
    auto issue = [&]() -> int {
        const int chunk = std::min(check_every, limit - it);
        if (graph && chunk == check_every) {
            if (!cg.exec) SGP_TRY(capture_chunk<T>(ctx, A, M, v, w, S, part, chunk, cg));
            HIP_TRY(ctx, hipGraphLaunch(cg.exec, st));
        } else {
            SGP_TRY(pcg_chunk<T>(ctx, A, M, v, w, S, part, chunk, it));
        }
        it += chunk;
        return SGP_OK;
    };
    int32_t iters_done = INT32_MAX;
    while (it < limit) {
        for (int b = issued_ahead ? 1 : 0; b < per_poll && it < limit; b++) SGP_TRY(issue());
        issued_ahead = false;
        const int it_poll = it;
        SGP_TRY(fill_i32(ctx, open, 0, 4));
        k_any_open<<<grid_for(K, 256), 256, 0, st>>>(S, K, open);
        if (ahead) {
            HIP_TRY(ctx, hipMemcpyAsync(hopen, open, 16, hipMemcpyDeviceToHost, st));
            HIP_TRY(ctx, hipEventRecord(ctx->poll_ev, st));
            if (it < limit) {
                SGP_TRY(issue());
                issued_ahead = true;
            }
            HIP_TRY(ctx, hipEventSynchronize(ctx->poll_ev));
        } else {
            SGP_TRY(readback(ctx, hopen, open, 16));
        }
        if (hopen[0] == 0) {
            // one cluster: its products past the final iteration were no-ops
            // (batched products always run for every cluster)
            if (K == 1) iters_done = hopen[1];
            break;
        }
        // timed pairs pile up only in long solves: fold in now and then those
        // of the iterations before this poll (all still open)
        if (ctx->kev_used >= 1024) SGP_TRY(ktimer_flush(ctx, it_poll));
        if (fixed > 0) continue;
        double worst;
        memcpy(&worst, hopen + 2, 8);
        per_poll = 1;
        if (worst > 1.0 && std::isfinite(worst)) {
            const double lg = log(worst);
            if (it_prev >= 0 && lg < lg_prev) {
                const double rem = -lg / ((lg - lg_prev) / (it_poll - it_prev));
                const double cap = std::max(8.0, 0.25 * it_poll) / check_every;
                per_poll = (int)std::max(1.0, std::min(cap, 0.5 * rem / check_every));
            }
            it_prev = it_poll;
            lg_prev = lg;
        }
    }
    SGP_TRY(ktimer_flush(ctx, iters_done));
    return SGP_OK;
}

// Note on the batched tree sweeps: converged clusters are not skipped inside
// the sweeps (their z is simply not used any more), only in the vector and
// matrix kernels, which carry the per-cluster test.

static int prepare_work(sgp_ctx ctx, sgp_bsr A, const std::vector<int64_t> &off, PcgWork &w,
                        sgp_prec M = nullptr)
{
    const int64_t K = (int64_t)off.size() - 1;
    w.K = K;
    build_tab(off, VEC_ROWS, w.vec_buf, w.vec_nb);
    w.mv_nb = spmv_blocks(ctx, A);
    w.vec_buf.push_back(0);
    w.vec_buf.push_back(w.mv_nb);
    int32_t *d;
    size_t nv = w.vec_buf.size();
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP6], nv + 2 + 2 * (size_t)w.vec_nb + 2, &d));
    SGP_TRY(upload(ctx, d, w.vec_buf.data(), nv * 4));
    w.vec = tab_ptrs(d, w.vec_nb, K);
    w.mv_first = d + nv - 2;
    w.mv_nb_dev = d + nv - 1;
    const int32_t q1 = ctx->fuse_step0 ? prec_step0_launch(M) : 0;
    if (q1 > 0 && M->n == A->n) {
        int32_t *qr = d + nv + 2;
        k_step0_ranges<<<grid_for(w.vec_nb, 256), 256, 0, ctx->stream>>>(w.vec_nb, w.vec,
                                                                         (const int32_t *)M->elim_int.p, q1, qr);
        LAUNCH_CHECK(ctx);
        w.s0_q1 = q1;
        w.s0_qr = qr;
    }
    return SGP_OK;
}

static int solve_f64(sgp_ctx ctx, sgp_bsr A, sgp_prec M, const std::vector<int64_t> &off, const double *F, double *x,
                     const sgp_solve_opts *o, sgp_solve_info *info)
{
    hipStream_t st = ctx->stream;
    const int64_t n = A->n, K = (int64_t)off.size() - 1;
    PcgWork w;
    SGP_TRY(prepare_work(ctx, A, off, w, M));
    double *r, *z, *p, *q, *part, *Fi, *xi;
    PcgScalars *S;
    int32_t *open;
    const int32_t *perm = (const int32_t *)A->perm.p;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP8], 6 * n + 6, &Fi));
    xi = Fi + 3 * n + 3;
    SGP_TRY(permute_rows(ctx, perm, F, Fi, n, 0));
    if (o->use_x0) SGP_TRY(permute_rows(ctx, perm, x, xi, n, 0));
    F = Fi;
    double *xuser = x;
    x = xi;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP0], 3 * n + 3, &r));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP1], 3 * n + 3, &p));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP2], 3 * n + 3, &q));
    if (M) SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], 3 * n + 3, &z));
    else z = r;   // no preconditioner: z is r
    int32_t nbmax = std::max(w.vec_nb, w.mv_nb);
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PART], 3 * (size_t)nbmax + 8, &part));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_SCAL], K + 1, &S));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], 8, &open));
    int fixed = std::max(0, o->fixed_iters);
    int max_iter = o->max_iter > 0 ? o->max_iter : 10000;
    const bool err_stop = o->stop == SGP_STOP_ERROR;
    double mu = o->mu;
    if (err_stop && !(mu > 0.0)) mu = M ? 1.0 : A->gmed;   // Section 4: lambda_min(P^-1 Gamma) >= 1; Gamma >= g_med I
    k_set_scalars<<<grid_for(K, 256), 256, 0, st>>>(S, K, o->rtol * o->rtol, fixed, max_iter, o->stop, mu);
    LAUNCH_CHECK(ctx);
    // a small single system: every iteration inside one workgroup, one
    // launch (bounded: at most 20,000 iterations in one launch)
    if (K == 1 && !err_stop && small_solve_fits(ctx, A, M) && std::max(fixed, max_iter) <= 20000) {
        SGP_TRY(solve_small(ctx, A, M, F, x, o, S));
    } else {
        if (o->use_x0) SGP_TRY(spmv_f64(ctx, A, x, q, nullptr, nullptr, 0));
        k_init_res<double><<<w.vec_nb, 256, 0, st>>>(F, q, x, r, o->use_x0, w.vec, part);
        LAUNCH_CHECK(ctx);
        SGP_TRY(fin(ctx, FIN_INIT, part, w.vec_nb, w.vec.ifirst, w.vec.inb, S, K));
        k_zero_rows<double><<<w.vec_nb, 256, 0, st>>>(x, w.vec, S, 2);
        if (M) SGP_TRY(prec_apply_f64(ctx, M, r, z, nullptr));
        k_init_p<double><<<w.vec_nb, 256, 0, st>>>(r, z, p, w.vec, S, part);
        LAUNCH_CHECK(ctx);
        SGP_TRY(fin(ctx, FIN_RHO, part, w.vec_nb, w.vec.ifirst, w.vec.inb, S, K));
        Vecs<double> v = {x, r, z, p, q};
        int ce = o->check_every > 0 ? o->check_every : ctx->check_every;
        SGP_TRY(pcg_iterate<double>(ctx, A, M, v, w, S, part, open, ce, max_iter, fixed));
    }
    // true residual
    SGP_TRY(spmv_f64(ctx, A, x, q, nullptr, nullptr, 0));
    k_true_res<<<w.vec_nb, 256, 0, st>>>(F, q, w.vec, part);
    LAUNCH_CHECK(ctx);
    SGP_TRY(fin(ctx, FIN_TRUE, part, w.vec_nb, w.vec.ifirst, w.vec.inb, S, K));
    SGP_TRY(permute_rows(ctx, perm, x, xuser, n, 1));
    std::vector<PcgScalars> hs(K);
    SGP_TRY(readback(ctx, hs.data(), S, K * sizeof(PcgScalars)));
    for (int64_t k = 0; k < K; k++) {
        const PcgScalars &s = hs[k];
        sgp_solve_info &I = info[k];
        memset(&I, 0, sizeof I);
        I.status = s.status;
        if (!s.done && !s.status) I.status = fixed > 0 ? SGP_OK : SGP_ENOCONV;
        I.iters = s.iter;
        I.relres_rec = s.nF2 > 0 ? sqrt(s.relres2) : 0.0;
        I.relres_true = s.nF2 > 0 ? sqrt(s.rz / s.nF2) : 0.0;
        if (err_stop && s.nF2 > 0) I.err_bound = s.gs + s.gbound > 0 ? sqrt(s.gbound / (s.gs + s.gbound)) : 1.0;
    }
    return SGP_OK;
}

// ---------------------------------------------------------------- FP32 inside FP64 refinement

__global__ void k_res64(int64_t len, const double *F, const double *q, double *r)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) r[i] = F[i] - q[i];
}

__global__ void k_axpy_f32_into_f64(int64_t len, const float *d, double *x)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) x[i] = x[i] + (double)d[i];
}

// partials of ||a||^2 and ||b||^2
__global__ __launch_bounds__(256) void k_norm2_pair(const double *a, const double *b, BlockTab tab, double *part)
{
    __shared__ double sh[256];
    int bl = blockIdx.x, inst;
    int64_t row;
    bool ok = block_rows(tab, bl, row, inst);
    double sa = 0.0, sb = 0.0;
    if (ok)
        for (int t = 0; t < 3; t++) {
            sa = sa + a[3 * row + t] * a[3 * row + t];
            sb = sb + b[3 * row + t] * b[3 * row + t];
        }
    block_partial(sa, bl, part, sh);
    block_partial(sb, bl, part + gridDim.x, sh);
}

static int solve_ir(sgp_ctx ctx, sgp_bsr A, sgp_prec M, const double *F, double *x, const sgp_solve_opts *o,
                    sgp_solve_info *info)
{
    hipStream_t st = ctx->stream;
    const int64_t n = A->n, len = 3 * n;
    if (!M || M->kind == PREC_NONE) return set_err(ctx, SGP_EINVAL, "IR solve needs a preconditioner");
    SGP_TRY(bsr_make32(ctx, A));
    SGP_TRY(prec_make32(ctx, M));
    std::vector<int64_t> off = {0, n};
    PcgWork w;
    SGP_TRY(prepare_work(ctx, A, off, w, M));
    double *r64, *q64, *part, *Fi, *xi;
    float *r, *z, *p, *q, *d;
    PcgScalars *S;
    int32_t *open;
    const int32_t *perm = (const int32_t *)A->perm.p;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP8], 2 * len + 6, &Fi));
    xi = Fi + len + 3;
    SGP_TRY(permute_rows(ctx, perm, F, Fi, n, 0));
    if (o->use_x0) SGP_TRY(permute_rows(ctx, perm, x, xi, n, 0));
    F = Fi;
    double *xuser = x;
    x = xi;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP0], len + 3, &r64));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP1], len + 3, &q64));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP2], 5 * len + 16, &r));
    z = r + len + 3;
    p = z + len + 3;
    q = p + len + 3;
    d = q + len + 3;
    int32_t nbmax = std::max(w.vec_nb, w.mv_nb);
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PART], 3 * (size_t)nbmax + 8, &part));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_SCAL], 2, &S));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], 8, &open));
    int max_outer = o->max_outer > 0 ? o->max_outer : 50;
    int max_inner = o->max_iter > 0 ? o->max_iter : 10000;
    double inner = o->inner_rtol > 0 ? o->inner_rtol : 1e-5;
    int ce = o->check_every > 0 ? o->check_every : ctx->check_every;
    if (!o->use_x0) SGP_TRY(fill_f64(ctx, x, 0.0, len));
    int total_inner = 0, outer = 0, status = SGP_OK;
    double relres = 0.0;
    PcgScalars hs;
    for (;;) {
        SGP_TRY(spmv_f64(ctx, A, x, q64, nullptr, nullptr, 0));
        k_res64<<<grid_for(len, 256), 256, 0, st>>>(len, F, q64, r64);
        k_norm2_pair<<<w.vec_nb, 256, 0, st>>>(r64, F, w.vec, part);
        LAUNCH_CHECK(ctx);
        SGP_TRY(fin(ctx, FIN_NORM2, part, w.vec_nb, w.vec.ifirst, w.vec.inb, S, 1));
        SGP_TRY(readback(ctx, &hs, S, sizeof hs));
        if (!std::isfinite(hs.rz) || !std::isfinite(hs.nF2)) {
            status = SGP_ENONFINITE;
            break;
        }
        if (hs.nF2 == 0.0) {
            SGP_TRY(fill_f64(ctx, x, 0.0, len));
            relres = 0.0;
            break;
        }
        relres = sqrt(hs.rz / hs.nF2);
        if (relres <= o->rtol) break;
        if (outer >= max_outer || total_inner >= max_inner) {
            status = SGP_ENOCONV;
            break;
        }
        // inner FP32 solve of Gamma d = r to relative tolerance `inner`
        k_set_scalars<<<1, 32, 0, st>>>(S, 1, inner * inner, 0, max_inner - total_inner);
        k_init_res<float><<<w.vec_nb, 256, 0, st>>>(r64, q, d, r, 0, w.vec, part);
        LAUNCH_CHECK(ctx);
        SGP_TRY(fin(ctx, FIN_INIT, part, w.vec_nb, w.vec.ifirst, w.vec.inb, S, 1));
        SGP_TRY(prec_apply_f32(ctx, M, r, z, nullptr));
        k_init_p<float><<<w.vec_nb, 256, 0, st>>>(r, z, p, w.vec, S, part);
        LAUNCH_CHECK(ctx);
        SGP_TRY(fin(ctx, FIN_RHO, part, w.vec_nb, w.vec.ifirst, w.vec.inb, S, 1));
        Vecs<float> v = {d, r, z, p, q};
        SGP_TRY(pcg_iterate<float>(ctx, A, M, v, w, S, part, open, ce, max_inner - total_inner, 0));
        SGP_TRY(readback(ctx, &hs, S, sizeof hs));
        total_inner += hs.iter;
        if (hs.status == SGP_EBREAKDOWN || hs.status == SGP_ENONFINITE) {
            status = hs.status;
            break;
        }
        k_axpy_f32_into_f64<<<grid_for(len, 256), 256, 0, st>>>(len, d, x);
        LAUNCH_CHECK(ctx);
        outer++;
    }
    SGP_TRY(permute_rows(ctx, perm, x, xuser, n, 1));
    memset(info, 0, sizeof *info);
    info->status = status;
    info->iters = total_inner;
    info->outer_iters = outer;
    info->relres_rec = relres;
    info->relres_true = relres;
    return SGP_OK;
}

// ---------------------------------------------------------------- entry points

static int solve_common(sgp_ctx ctx, sgp_bsr A, sgp_prec M, const std::vector<int64_t> &off, const double *F,
                        double *v, const sgp_solve_opts *opts, sgp_solve_info *info)
{
    if (!ctx || !A || !opts || !info) return set_err(ctx, SGP_EINVAL, "pcg_solve: null argument");
    if (A->n > 0 && (!F || !v)) return set_err(ctx, SGP_EINVAL, "pcg_solve: null vector");
    if (M && M->kind != PREC_NONE && M->n != A->n) return set_err(ctx, SGP_EINVAL, "pcg_solve: M and A differ in size");
    if (!(opts->rtol >= 0.0)) return set_err(ctx, SGP_EINVAL, "pcg_solve: rtol must be >= 0");
    if (M && M->kind == PREC_NONE) M = nullptr;
    // the block-CSR product's blocks, before any iteration is captured
    if (!ctx->spmv_form) SGP_TRY(bsr_blocks(ctx, A));
    if (opts->stop != SGP_STOP_RESIDUAL && opts->stop != SGP_STOP_ERROR)
        return set_err(ctx, SGP_EINVAL, "pcg_solve: unknown stopping rule %d", opts->stop);
    if (opts->stop == SGP_STOP_ERROR) {
        if (opts->use_x0 || opts->precision != SGP_PREC_F64 || (M && M->aug))
            return set_err(ctx, SGP_EINVAL, "pcg_solve: the error bound needs an FP64 solve from x0 = 0 (no augmented tree)");
        if (M && M->kind == PREC_JACOBI && !(opts->mu > 0.0))
            return set_err(ctx, SGP_EINVAL, "pcg_solve: the error bound with block Jacobi needs mu > 0");
    }
    const int64_t K = (int64_t)off.size() - 1;
    if (A->n == 0) {
        for (int64_t k = 0; k < K; k++) memset(&info[k], 0, sizeof info[k]);
        return SGP_OK;
    }
    hipStream_t st = ctx->stream;
    phase_begin(ctx, 4);
    int s;
    if (M && M->aug) {
        // the augmented tree (Section 3.1): flexible CG around an inner tree-PCG
        if (K != 1 || opts->precision != SGP_PREC_F64 || opts->fixed_iters > 0)
            return set_err(ctx, SGP_EINVAL, "pcg_solve: the augmented tree solves one FP64 system to rtol");
        const int64_t n = A->n;
        double *Fi, *xi;
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP8], 6 * n + 6, &Fi));
        xi = Fi + 3 * n + 3;
        const int32_t *perm = (const int32_t *)A->perm.p;
        SGP_TRY(permute_rows(ctx, perm, F, Fi, n, 0));
        if (opts->use_x0) SGP_TRY(permute_rows(ctx, perm, v, xi, n, 0));
        s = solve_augmented(ctx, A, M, Fi, xi, opts, info);
        if (s == SGP_OK || info->status != SGP_OK) SGP_TRY(permute_rows(ctx, perm, xi, v, n, 1));
    } else if (opts->precision == SGP_PREC_F32_IR) {
        if (K != 1) return set_err(ctx, SGP_EINVAL, "pcg_solve: FP32 refinement is single-cluster only");
        s = solve_ir(ctx, A, M, F, v, opts, info);
    } else {
        s = solve_f64(ctx, A, M, off, F, v, opts, info);
    }
    if (s == SGP_OK) phase_end(ctx, 4);
    if (s != SGP_OK) return s;
    int worst = SGP_OK;
    for (int64_t k = 0; k < K; k++)
        if (info[k].status != SGP_OK && worst == SGP_OK) worst = info[k].status;
    if (worst != SGP_OK) set_err(ctx, worst, "pcg_solve: status %d", worst);
    return worst;
}

extern "C" int sgp_pcg_solve(sgp_ctx ctx, sgp_bsr A, sgp_prec M, const double *F, double *v,
                             const sgp_solve_opts *opts, sgp_solve_info *info)
{
    if (!A) return set_err(ctx, SGP_EINVAL, "pcg_solve: null matrix");
    std::vector<int64_t> off = {0, A->n};
    return solve_common(ctx, A, M, off, F, v, opts, info);
}

extern "C" int sgp_pcg_solve_batched(sgp_ctx ctx, sgp_bsr A, sgp_prec M, int64_t n_inst, const int64_t *offsets,
                                     const double *F, double *v, const sgp_solve_opts *opts, sgp_solve_info *info)
{
    if (!A || !offsets || n_inst <= 0) return set_err(ctx, SGP_EINVAL, "pcg_solve_batched: bad arguments");
    if (offsets[0] != 0 || offsets[n_inst] != A->n)
        return set_err(ctx, SGP_EINVAL, "pcg_solve_batched: offsets must cover [0, n)");
    for (int64_t k = 0; k < n_inst; k++)
        if (offsets[k + 1] < offsets[k]) return set_err(ctx, SGP_EINVAL, "pcg_solve_batched: offsets decrease");
    std::vector<int64_t> off(offsets, offsets + n_inst + 1);
    return solve_common(ctx, A, M, off, F, v, opts, info);
}

extern "C" int sgp_residual_norm(sgp_ctx ctx, sgp_bsr A, const double *F, const double *x, double *relres)
{
    if (!ctx || !A || !relres || (A->n > 0 && (!F || !x))) return set_err(ctx, SGP_EINVAL, "residual_norm: bad arguments");
    const int64_t n = A->n;
    if (n == 0) {
        *relres = 0.0;
        return SGP_OK;
    }
    std::vector<int64_t> off = {0, n};
    PcgWork w;
    SGP_TRY(prepare_work(ctx, A, off, w));
    double *Fi, *xi, *q, *part;
    PcgScalars *S;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP8], 9 * n + 9, &Fi));
    xi = Fi + 3 * n + 3;
    q = xi + 3 * n + 3;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PART], 3 * (size_t)std::max(w.vec_nb, w.mv_nb) + 8, &part));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_SCAL], 2, &S));
    const int32_t *perm = (const int32_t *)A->perm.p;
    SGP_TRY(permute_rows(ctx, perm, F, Fi, n, 0));
    SGP_TRY(permute_rows(ctx, perm, x, xi, n, 0));
    SGP_TRY(spmv_f64(ctx, A, xi, q, nullptr, nullptr, 0));
    k_res64<<<grid_for(3 * n, 256), 256, 0, ctx->stream>>>(3 * n, Fi, q, q);
    k_norm2_pair<<<w.vec_nb, 256, 0, ctx->stream>>>(q, Fi, w.vec, part);
    LAUNCH_CHECK(ctx);
    SGP_TRY(fin(ctx, FIN_NORM2, part, w.vec_nb, w.vec.ifirst, w.vec.inb, S, 1));
    PcgScalars hs;
    SGP_TRY(readback(ctx, &hs, S, sizeof hs));
    *relres = hs.nF2 > 0 ? sqrt(hs.rz / hs.nF2) : 0.0;
    return SGP_OK;
}

extern "C" int sgp_tune(sgp_ctx ctx, const char *key, int32_t value)
{
    if (!ctx) return SGP_EINVAL;
    if (!key) return set_err(ctx, SGP_EINVAL, "tune: null key");
    if (!strcmp(key, "check_every")) {
        if (value < 1 || value > 1024) return set_err(ctx, SGP_EINVAL, "tune: check_every must be in [1, 1024]");
        ctx->check_every = value;
        return SGP_OK;
    }
    if (!strcmp(key, "tail_max")) {
        if (value < 0 || value > 65536) return set_err(ctx, SGP_EINVAL, "tune: tail_max must be in [0, 65536]");
        ctx->tail_max = value;
        return SGP_OK;
    }
    if (!strcmp(key, "graph")) {
        if (value != 0 && value != 1) return set_err(ctx, SGP_EINVAL, "tune: graph must be 0 or 1");
        ctx->use_graph = value;
        return SGP_OK;
    }
    if (!strcmp(key, "spmv_waves")) {
        if (value != 2 && value != 4 && value != 8) return set_err(ctx, SGP_EINVAL, "tune: spmv_waves must be 2, 4 or 8");
        ctx->spmv_waves = value;
        return SGP_OK;
    }
    if (!strcmp(key, "spmv_form")) {
        if (value != 0 && value != 1) return set_err(ctx, SGP_EINVAL, "tune: spmv_form must be 0 or 1");
        ctx->spmv_form = value;
        return SGP_OK;
    }
    if (!strcmp(key, "light_height")) {
        if (value < 0 || value > 1024) return set_err(ctx, SGP_EINVAL, "tune: light_height must be in [0, 1024]");
        ctx->light_height = value;
        return SGP_OK;
    }
    if (!strcmp(key, "light_cap")) {
        if (value < 1 || value > (1 << 20)) return set_err(ctx, SGP_EINVAL, "tune: light_cap must be in [1, 2^20]");
        ctx->light_cap = value;
        return SGP_OK;
    }
    if (!strcmp(key, "mid_lds")) {
        if (value < 0 || value > 1) return set_err(ctx, SGP_EINVAL, "tune: mid_lds must be 0 or 1");
        ctx->mid_lds = value;
        return SGP_OK;
    }
    if (!strcmp(key, "small_solve")) {
        if (value < 0 || value > 1) return set_err(ctx, SGP_EINVAL, "tune: small_solve must be 0 or 1");
        ctx->small_solve = value;
        return SGP_OK;
    }
    if (!strcmp(key, "fuse_step0")) {
        if (value < 0 || value > 1) return set_err(ctx, SGP_EINVAL, "tune: fuse_step0 must be 0 or 1");
        ctx->fuse_step0 = value;
        return SGP_OK;
    }
    if (!strcmp(key, "tail_side")) {
        if (value < 0 || value > 1) return set_err(ctx, SGP_EINVAL, "tune: tail_side must be 0 or 1");
        ctx->tail_side = value;
        return SGP_OK;
    }
    if (!strcmp(key, "prefetch")) {
        if (value < 0 || value > 1) return set_err(ctx, SGP_EINVAL, "tune: prefetch must be 0 or 1");
        ctx->prefetch = value;
        return SGP_OK;
    }
    return set_err(ctx, SGP_EINVAL, "tune: unknown key '%s'", key);
}

extern "C" int sgp_tune_get(sgp_ctx ctx, const char *key, int32_t *value)
{
    if (!ctx || !key || !value) return set_err(ctx, SGP_EINVAL, "tune_get: bad arguments");
    if (!strcmp(key, "check_every")) *value = ctx->check_every;
    else if (!strcmp(key, "tail_max")) *value = ctx->tail_max;
    else if (!strcmp(key, "graph")) *value = ctx->use_graph;
    else if (!strcmp(key, "spmv_waves")) *value = ctx->spmv_waves;
    else if (!strcmp(key, "light_height")) *value = ctx->light_height;
    else if (!strcmp(key, "spmv_form")) *value = ctx->spmv_form;
    else if (!strcmp(key, "light_cap")) *value = ctx->light_cap;
    else if (!strcmp(key, "fuse_step0")) *value = ctx->fuse_step0;
    else if (!strcmp(key, "small_solve")) *value = ctx->small_solve;
    else if (!strcmp(key, "mid_lds")) *value = ctx->mid_lds;
    else if (!strcmp(key, "tail_side")) *value = ctx->tail_side;
    else if (!strcmp(key, "prefetch")) *value = ctx->prefetch;
    else return set_err(ctx, SGP_EINVAL, "tune_get: unknown key '%s'", key);
    return SGP_OK;
}
