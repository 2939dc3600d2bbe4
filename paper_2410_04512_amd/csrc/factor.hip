// Section 3.3 (Alg. 2, TreeLDLT) and Appendix B.1 (tree solves) on the GPU.
//
// The factorisation is driven by an elimination schedule: a partition of the
// vertices into steps such that every vertex is eliminated after the
// vertices it is connected to from below.  Each vertex v records the (at most
// two) vertices it is still connected to when eliminated -- up0 (toward the
// root) and, for a chain vertex removed by compress, up1 (its one child).
// With the vertices renumbered in elimination order q, P = L D L^T where row
// q of L^T has the blocks L_{up_k(q), q} = A_{up_k, q} D_q^{-1}.  We store
//    Dinv[q]   = D_q^{-1}            (symmetric, packed 6)
//    F[q][k]   = A_{up_k(q), q}      (full 3x3, the coupling at elimination)
// and solve P x = b as
//    forward   y_q = D_q^{-1} (b_q - sum_{(u,k): up_k(u) = q} F[u][k] y_u)
//    backward  x_q = y_q - D_q^{-1} sum_k F[q][k]^T x_{up_k(q)}
// which is ForwardSolve, DiagSolve and BackwardSolve of Appendix B.1 with
// the pivot solve folded into each sweep.
//
// Schedules:
//  LEVEL     step = max depth - depth: Alg. 2's order (decreasing distance
//            to the root); up0 = parent.  One step per tree level.
//  CONTRACT  rake and compress (tree contraction): in one step every current
//            leaf is eliminated into its parent, and an independent set of
//            one-child vertices whose child is not a leaf is eliminated,
//            joining parent and child by the Schur block
//            A'_{p,c} = -A_{p,v} D_v^{-1} A_{v,c}.  The forest stays a forest
//            (no fill beyond one block per removed chain vertex) and the
//            number of steps is O(log n) instead of the tree depth.
#include "sgp_internal.h"

#include <algorithm>
#include <climits>

// ---------------------------------------------------------------- W and P_ii

SGP_DEV void friction_block_dev(double w, double ux, double uy, double uz, double gpar, double gperp,
                                double *W)
{
    const double u[3] = {ux, uy, uz};
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double uu = u[a] * u[b];
            double id = (a == b) ? 1.0 : 0.0;
            W[3 * a + b] = w * (gpar * uu + gperp * (id - uu));
        }
}

// P_vv = g_med I + sum of W_e over the tree edges at v, ascending edge id;
// E_v = A_{parent(v), v} = -W_{pedge(v)} (zero at roots).
__global__ void k_tree_blocks(int64_t n, const int32_t *tptr, const int32_t *tadje, const int32_t *pedge,
                              const double4 *wu, double gpar, double gperp, double gmed, double *Pd,
                              double *E)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double P[9];
    for (int t = 0; t < 9; t++) P[t] = (t % 4 == 0) ? gmed : 0.0;
    for (int32_t k = tptr[v]; k < tptr[v + 1]; k++) {
        double4 q = wu[tadje[k]];
        double W[9];
        friction_block_dev(q.x, q.y, q.z, q.w, gpar, gperp, W);
        for (int t = 0; t < 9; t++) P[t] = P[t] + W[t];
    }
    for (int t = 0; t < 9; t++) Pd[9 * v + t] = P[t];
    int32_t e = pedge[v];
    if (e >= 0) {
        double4 q = wu[e];
        double W[9];
        friction_block_dev(q.x, q.y, q.z, q.w, gpar, gperp, W);
        for (int t = 0; t < 9; t++) E[9 * v + t] = -W[t];
    } else {
        for (int t = 0; t < 9; t++) E[9 * v + t] = 0.0;
    }
}

// ---------------------------------------------------------------- schedules

__global__ void k_sched_level(int64_t n, const int32_t *depth, const int32_t *parent, int32_t maxd,
                              int32_t *stepv, int32_t *up0, int32_t *up1)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    stepv[v] = maxd - depth[v];
    up0[v] = parent[v];
    up1[v] = -1;
}

__global__ void k_contract_init(int64_t n, const int32_t *parent, int32_t *par, int32_t *nch, int32_t *xch,
                                int32_t *stepv)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t p = parent[v];
    par[v] = p;
    stepv[v] = -1;
    if (p >= 0) {
        atomicAdd(&nch[p], 1);
        atomicXor(&xch[p], (int32_t)v);
    }
}

SGP_DEV uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// priority of v in step s: a hash, ties by id (a strict order)
SGP_DEV bool beats(int32_t a, int32_t b, int32_t s)
{
    uint32_t ha = mix32((uint32_t)a * 0x9e3779b1u ^ (uint32_t)s * 0x85ebca77u);
    uint32_t hb = mix32((uint32_t)b * 0x9e3779b1u ^ (uint32_t)s * 0x85ebca77u);
    return ha != hb ? ha > hb : a > b;
}

__global__ void k_contract_select(int64_t n, int32_t s, const int32_t *par, const int32_t *nch,
                                  const int32_t *xch, int32_t *stepv, int32_t *up0, int32_t *up1)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || stepv[v] >= 0) return;
    int32_t p = par[v], c0 = nch[v];
    if (c0 == 0) {   // leaf (rake) or a lone root (final)
        stepv[v] = s;
        up0[v] = p;
        up1[v] = -1;
        return;
    }
    if (c0 != 1 || p < 0) return;
    int32_t c = xch[v];
    if (nch[c] == 0) return;   // its child is a leaf: it is raked first
    bool unary_p = nch[p] == 1 && par[p] >= 0;
    bool unary_c = nch[c] == 1 && par[c] >= 0;
    if (unary_p && !beats((int32_t)v, p, s)) return;
    if (unary_c && !beats((int32_t)v, c, s)) return;
    stepv[v] = s;
    up0[v] = p;
    up1[v] = c;
}

__global__ void k_contract_apply(int64_t n, int32_t s, const int32_t *stepv, const int32_t *up0,
                                 const int32_t *up1, int32_t *par, int32_t *nch, int32_t *xch, int32_t *cnt)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || stepv[v] != s) return;
    int32_t p = up0[v], c = up1[v];
    if (c >= 0) {
        par[c] = p;
        atomicXor(&xch[p], (int32_t)v ^ c);
    } else if (p >= 0) {
        atomicSub(&nch[p], 1);
        atomicXor(&xch[p], (int32_t)v);
    }
    atomicAdd(cnt, 1);
}

__global__ void k_step_count(int64_t n, const int32_t *stepv, int32_t *cnt)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) atomicAdd(&cnt[stepv[v]], 1);
}

__global__ void k_stepkeys(int64_t n, const int32_t *stepv, uint32_t *key, int32_t *val)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    key[v] = (uint32_t)stepv[v];
    val[v] = (int32_t)v;
}

__global__ void k_invperm(int64_t n, const int32_t *elim, int32_t *pos)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) pos[elim[q]] = (int32_t)q;
}

// up links in elimination numbering, and the in-list entries (target, source slot)
__global__ void k_uplinks(int64_t n, const int32_t *elim, const int32_t *pos, const int32_t *up0,
                          const int32_t *up1, int32_t *upq, uint32_t *ikey, int32_t *ival, int32_t *icnt)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int32_t v = elim[q];
    int32_t a = up0[v], b = up1[v];
    int32_t qa = a >= 0 ? pos[a] : -1, qb = b >= 0 ? pos[b] : -1;
    upq[2 * q] = qa;
    upq[2 * q + 1] = qb;
    ikey[2 * q] = qa >= 0 ? (uint32_t)qa : (uint32_t)n;
    ival[2 * q] = (int32_t)(2 * q);
    ikey[2 * q + 1] = qb >= 0 ? (uint32_t)qb : (uint32_t)n;
    ival[2 * q + 1] = (int32_t)(2 * q + 1);
    if (qa >= 0) atomicAdd(&icnt[qa], 1);
    if (qb >= 0) atomicAdd(&icnt[qb], 1);
}

// ---------------------------------------------------------------- numeric factor

// One elimination step: pivots of the step's vertices, their couplings F and
// their Schur contributions C[slot] (symmetric packed) to the vertices above.
__global__ void k_factor_step(int32_t q0, int32_t q1, const int32_t *elim, const int32_t *upq,
                              const int32_t *in_ptr, const int32_t *in_src, const double *Pd, double *E,
                              double *C, double *F, double *Dinv, int32_t *status)
{
    int32_t q = q0 + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= q1) return;
    int32_t v = elim[q];
    double D[9];
    for (int t = 0; t < 9; t++) D[t] = Pd[9 * (int64_t)v + t];
    for (int32_t t = in_ptr[q]; t < in_ptr[q + 1]; t++) {
        const double *c = C + 6 * (int64_t)in_src[t];
        D[0] = D[0] - c[0]; D[1] = D[1] - c[1]; D[2] = D[2] - c[2];
        D[3] = D[3] - c[1]; D[4] = D[4] - c[3]; D[5] = D[5] - c[4];
        D[6] = D[6] - c[2]; D[7] = D[7] - c[4]; D[8] = D[8] - c[5];
    }
    double inv[6];
    if (!spd_inverse3(D, inv)) {
        atomicOr(status, 1);
        for (int t = 0; t < 6; t++) inv[t] = 0.0;
    }
    for (int t = 0; t < 6; t++) Dinv[6 * (int64_t)q + t] = inv[t];
    double Di[9];
    sym_unpack(inv, Di);
    int32_t qa = upq[2 * q], qb = upq[2 * q + 1];
    double T0[9];
    if (qa >= 0) {
        double E0[9];
        for (int t = 0; t < 9; t++) E0[t] = E[9 * (int64_t)q + t];   // A_{p,v}
        for (int t = 0; t < 9; t++) F[18 * (int64_t)q + t] = E0[t];
        mm3(E0, Di, T0);                                                // A_{p,v} D^{-1}
        double *c = C + 6 * (2 * (int64_t)q);
        // A_{p,v} D^{-1} A_{v,p}: upper triangle of T0 E0^T
        c[0] = T0[0] * E0[0] + T0[1] * E0[1] + T0[2] * E0[2];
        c[1] = T0[0] * E0[3] + T0[1] * E0[4] + T0[2] * E0[5];
        c[2] = T0[0] * E0[6] + T0[1] * E0[7] + T0[2] * E0[8];
        c[3] = T0[3] * E0[3] + T0[4] * E0[4] + T0[5] * E0[5];
        c[4] = T0[3] * E0[6] + T0[4] * E0[7] + T0[5] * E0[8];
        c[5] = T0[6] * E0[6] + T0[7] * E0[7] + T0[8] * E0[8];
    }
    if (qb >= 0) {
        double E1[9], E1t[9], T1[9];
        for (int t = 0; t < 9; t++) E1[t] = E[9 * (int64_t)qb + t];   // A_{v,c}
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) E1t[3 * a + b] = E1[3 * b + a];
        for (int t = 0; t < 9; t++) F[18 * (int64_t)q + 9 + t] = E1t[t];   // A_{c,v}
        mm3(E1t, Di, T1);                                                   // A_{c,v} D^{-1}
        double *c = C + 6 * (2 * (int64_t)q + 1);
        // A_{c,v} D^{-1} A_{v,c}: upper triangle of T1 E1
        c[0] = T1[0] * E1[0] + T1[1] * E1[3] + T1[2] * E1[6];
        c[1] = T1[0] * E1[1] + T1[1] * E1[4] + T1[2] * E1[7];
        c[2] = T1[0] * E1[2] + T1[1] * E1[5] + T1[2] * E1[8];
        c[3] = T1[3] * E1[1] + T1[4] * E1[4] + T1[5] * E1[7];
        c[4] = T1[3] * E1[2] + T1[4] * E1[5] + T1[5] * E1[8];
        c[5] = T1[6] * E1[2] + T1[7] * E1[5] + T1[8] * E1[8];
        // new coupling of parent and child: -A_{p,v} D^{-1} A_{v,c}
        double Nw[9];
        mm3(T0, E1, Nw);
        for (int t = 0; t < 9; t++) E[9 * (int64_t)qb + t] = -Nw[t];
    }
}

// E is stored per vertex id for the initial blocks; the factor works in
// elimination numbering: permute once.
__global__ void k_permute9(int64_t n, const int32_t *elim, const double *src, double *dst)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int64_t v = elim[q];
    for (int t = 0; t < 9; t++) dst[9 * q + t] = src[9 * v + t];
}

// ---------------------------------------------------------------- sweeps

template <class T>
__global__ void k_fwd_step(int32_t q0, int32_t q1, const int32_t *elim, const int32_t *in_ptr,
                           const int32_t *in_src, const T *F, const T *Dinv, const T *r, T *y,
                           const PcgScalars *s)
{
    if (s && s->done) return;
    int32_t q = q0 + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= q1) return;
    int64_t v = elim[q];
    T b0 = r[3 * v], b1 = r[3 * v + 1], b2 = r[3 * v + 2];
    for (int32_t t = in_ptr[q]; t < in_ptr[q + 1]; t++) {
        int32_t src = in_src[t];
        const T *Fm = F + 9 * (int64_t)src;
        int64_t u = src >> 1;
        T y0 = y[3 * u], y1 = y[3 * u + 1], y2 = y[3 * u + 2];
        b0 = b0 - (Fm[0] * y0 + Fm[1] * y1 + Fm[2] * y2);
        b1 = b1 - (Fm[3] * y0 + Fm[4] * y1 + Fm[5] * y2);
        b2 = b2 - (Fm[6] * y0 + Fm[7] * y1 + Fm[8] * y2);
    }
    T o0, o1, o2;
    sym_mv(Dinv + 6 * (int64_t)q, b0, b1, b2, o0, o1, o2);
    y[3 * (int64_t)q] = o0;
    y[3 * (int64_t)q + 1] = o1;
    y[3 * (int64_t)q + 2] = o2;
}

template <class T>
__global__ void k_bwd_step(int32_t q0, int32_t q1, const int32_t *elim, const int32_t *upq, const T *F,
                           const T *Dinv, T *y, T *z, const PcgScalars *s)
{
    if (s && s->done) return;
    int32_t q = q0 + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= q1) return;
    T a0 = 0, a1 = 0, a2 = 0;
    for (int k = 0; k < 2; k++) {
        int32_t w = upq[2 * q + k];
        if (w < 0) continue;
        const T *Fm = F + 9 * (2 * (int64_t)q + k);
        T x0 = y[3 * (int64_t)w], x1 = y[3 * (int64_t)w + 1], x2 = y[3 * (int64_t)w + 2];
        a0 = a0 + (Fm[0] * x0 + Fm[3] * x1 + Fm[6] * x2);
        a1 = a1 + (Fm[1] * x0 + Fm[4] * x1 + Fm[7] * x2);
        a2 = a2 + (Fm[2] * x0 + Fm[5] * x1 + Fm[8] * x2);
    }
    T d0, d1, d2;
    sym_mv(Dinv + 6 * (int64_t)q, a0, a1, a2, d0, d1, d2);
    T x0 = y[3 * (int64_t)q] - d0, x1 = y[3 * (int64_t)q + 1] - d1, x2 = y[3 * (int64_t)q + 2] - d2;
    y[3 * (int64_t)q] = x0;
    y[3 * (int64_t)q + 1] = x1;
    y[3 * (int64_t)q + 2] = x2;
    int64_t v = elim[q];
    z[3 * v] = x0;
    z[3 * v + 1] = x1;
    z[3 * v + 2] = x2;
}

template <class T>
__global__ void k_jacobi_apply(int64_t n, const T *dinv, const T *r, T *z, const PcgScalars *s)
{
    if (s && s->done) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T o0, o1, o2;
    sym_mv(dinv + 6 * i, r[3 * i], r[3 * i + 1], r[3 * i + 2], o0, o1, o2);
    z[3 * i] = o0;
    z[3 * i + 1] = o1;
    z[3 * i + 2] = o2;
}

template <class T>
__global__ void k_copy_vec(int64_t len, const T *a, T *b, const PcgScalars *s)
{
    if (s && s->done) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) b[i] = a[i];
}

template <class T>
static int tree_sweeps(sgp_ctx ctx, sgp_prec M, const T *F, const T *Dinv, T *y, const T *r, T *z,
                       PcgScalars *s)
{
    hipStream_t st = ctx->stream;
    const int32_t *elim = (const int32_t *)M->elim.p, *in_ptr = (const int32_t *)M->in_ptr.p;
    const int32_t *in_src = (const int32_t *)M->in_src.p, *upq = (const int32_t *)M->up.p;
    const std::vector<int32_t> &sp = M->h_step_ptr;
    for (int k = 0; k < M->steps; k++) {
        int32_t q0 = sp[k], q1 = sp[k + 1];
        if (q1 > q0)
            k_fwd_step<T><<<grid_for(q1 - q0, 128), 128, 0, st>>>(q0, q1, elim, in_ptr, in_src, F, Dinv, r, y, s);
    }
    for (int k = M->steps - 1; k >= 0; k--) {
        int32_t q0 = sp[k], q1 = sp[k + 1];
        if (q1 > q0)
            k_bwd_step<T><<<grid_for(q1 - q0, 128), 128, 0, st>>>(q0, q1, elim, upq, F, Dinv, y, z, s);
    }
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

int prec_apply_f64(sgp_ctx ctx, sgp_prec M, const double *r, double *z, PcgScalars *s)
{
    hipStream_t st = ctx->stream;
    if (!M || M->kind == PREC_NONE) {
        int64_t len = 3 * (M ? M->n : 0);
        (void)len;
        return set_err(ctx, SGP_EINVAL, "prec_apply: identity handled by caller");
    }
    if (M->kind == PREC_JACOBI) {
        k_jacobi_apply<double><<<grid_for(M->n, 256), 256, 0, st>>>(M->n, (const double *)M->jdinv.p, r, z, s);
        LAUNCH_CHECK(ctx);
        return SGP_OK;
    }
    return tree_sweeps<double>(ctx, M, (const double *)M->F.p, (const double *)M->Dinv.p, (double *)M->y.p, r, z,
                               s);
}

int prec_apply_f32(sgp_ctx ctx, sgp_prec M, const float *r, float *z, PcgScalars *s)
{
    hipStream_t st = ctx->stream;
    if (M->kind == PREC_JACOBI) {
        k_jacobi_apply<float><<<grid_for(M->n, 256), 256, 0, st>>>(M->n, (const float *)M->Dinv32.p, r, z, s);
        LAUNCH_CHECK(ctx);
        return SGP_OK;
    }
    return tree_sweeps<float>(ctx, M, (const float *)M->F32.p, (const float *)M->Dinv32.p, (float *)M->y32.p, r, z,
                              s);
}

__global__ void k_to_f32(int64_t len, const double *a, float *b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) b[i] = (float)a[i];
}

// FP32 copies of the factors: computed in FP64, rounded once
int prec_make32(sgp_ctx ctx, sgp_prec M)
{
    if (M->have32) return SGP_OK;
    hipStream_t st = ctx->stream;
    int64_t n = M->n;
    float *F32, *D32, *y32;
    if (M->kind == PREC_TREE) {
        SGP_TRY(ensure_t(ctx, M->F32, 18 * n + 1, &F32));
        SGP_TRY(ensure_t(ctx, M->Dinv32, 6 * n + 1, &D32));
        SGP_TRY(ensure_t(ctx, M->y32, 3 * n + 1, &y32));
        k_to_f32<<<grid_for(18 * n, 256), 256, 0, st>>>(18 * n, (const double *)M->F.p, F32);
        k_to_f32<<<grid_for(6 * n, 256), 256, 0, st>>>(6 * n, (const double *)M->Dinv.p, D32);
    } else if (M->kind == PREC_JACOBI) {
        SGP_TRY(ensure_t(ctx, M->Dinv32, 6 * n + 1, &D32));
        k_to_f32<<<grid_for(6 * n, 256), 256, 0, st>>>(6 * n, (const double *)M->jdinv.p, D32);
    }
    LAUNCH_CHECK(ctx);
    M->have32 = true;
    return SGP_OK;
}

// ---------------------------------------------------------------- entry points

extern "C" int sgp_factor_tree(sgp_ctx ctx, sgp_graph g, sgp_tree T, double g_par, double g_perp, double g_med,
                               int32_t schedule, sgp_prec M)
{
    if (!ctx || !g || !T || !M) return set_err(ctx, SGP_EINVAL, "factor_tree: null handle");
    if (!(g_par > 0) || !(g_perp > 0) || !(g_med >= 0))
        return set_err(ctx, SGP_EINVAL, "factor_tree: friction coefficients must be positive");
    if (schedule != SGP_SCHED_LEVEL && schedule != SGP_SCHED_CONTRACT)
        return set_err(ctx, SGP_EINVAL, "factor_tree: unknown schedule %d", schedule);
    if (T->n != g->n) return set_err(ctx, SGP_EINVAL, "factor_tree: tree and graph differ in size");
    hipStream_t st = ctx->stream;
    if (ctx->ev[6]) (void)hipEventRecord(ctx->ev[6], st);
    const int64_t n = g->n;
    M->kind = PREC_TREE;
    M->n = n;
    M->schedule = schedule;
    M->have32 = false;
    if (n == 0) {
        M->steps = 0;
        M->h_step_ptr.assign(1, 0);
        return SGP_OK;
    }
    int32_t *stepv, *up0, *up1, *hbuf = (int32_t *)ctx->pinned;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP0], n + 1, &stepv));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP1], n + 1, &up0));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP2], n + 1, &up1));
    const int32_t *parent = (const int32_t *)T->parent.p;
    int32_t S = 0;
    if (schedule == SGP_SCHED_LEVEL) {
        k_sched_level<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)T->depth.p, parent, T->max_depth, stepv,
                                                      up0, up1);
        LAUNCH_CHECK(ctx);
        S = T->max_depth + 1;
    } else {
        int32_t *par, *nch, *xch, *cnt;
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], n + 1, &par));
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], n + 1, &nch));
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP5], n + 1, &xch));
        SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP6], 4, &cnt));
        SGP_TRY(fill_i32(ctx, nch, 0, n));
        SGP_TRY(fill_i32(ctx, xch, 0, n));
        SGP_TRY(fill_i32(ctx, cnt, 0, 1));
        k_contract_init<<<grid_for(n, 256), 256, 0, st>>>(n, parent, par, nch, xch, stepv);
        LAUNCH_CHECK(ctx);
        int64_t done = 0;
        while (done < n) {
            if (S > 100000) return set_err(ctx, SGP_EINVAL, "factor_tree: contraction did not finish");
            k_contract_select<<<grid_for(n, 256), 256, 0, st>>>(n, S, par, nch, xch, stepv, up0, up1);
            k_contract_apply<<<grid_for(n, 256), 256, 0, st>>>(n, S, stepv, up0, up1, par, nch, xch, cnt);
            LAUNCH_CHECK(ctx);
            S++;
            SGP_TRY(readback(ctx, hbuf, cnt, 4));
            if (hbuf[0] <= done) return set_err(ctx, SGP_EINVAL, "factor_tree: contraction made no progress");
            done = hbuf[0];
        }
    }
    M->steps = S;
    // elimination order: by (step, id)
    uint32_t *ka, *kb;
    int32_t *elim, *vb, *pos, *scnt, *sptr;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_A], 2 * n + 2, &ka));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_KEY_B], 2 * n + 2, &kb));
    SGP_TRY(ensure_t(ctx, M->elim, n + 1, &elim));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_VAL_B], 2 * n + 2, &vb));
    SGP_TRY(ensure_t(ctx, M->pos, n + 1, &pos));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP7], (size_t)S + 2, &scnt));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP8], (size_t)S + 2, &sptr));
    int sbits = 1;
    while ((1 << sbits) < S) sbits++;
    k_stepkeys<<<grid_for(n, 256), 256, 0, st>>>(n, stepv, ka, elim);
    LAUNCH_CHECK(ctx);
    SGP_TRY(radix_sort_pairs(ctx, ka, elim, kb, vb, n, sbits));
    k_invperm<<<grid_for(n, 256), 256, 0, st>>>(n, elim, pos);
    SGP_TRY(fill_i32(ctx, scnt, 0, S));
    k_step_count<<<grid_for(n, 256), 256, 0, st>>>(n, stepv, scnt);
    SGP_TRY(scan_exclusive(ctx, scnt, sptr, S));
    M->h_step_ptr.resize(S + 1);
    SGP_TRY(readback(ctx, M->h_step_ptr.data(), sptr, (S + 1) * sizeof(int32_t)));
    // up links and in-lists
    int32_t *upq, *icnt, *in_ptr, *in_src;
    SGP_TRY(ensure_t(ctx, M->up, 2 * n + 2, &upq));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_DEG], n + 2, &icnt));
    SGP_TRY(ensure_t(ctx, M->in_ptr, n + 2, &in_ptr));
    SGP_TRY(ensure_t(ctx, M->in_src, 2 * n + 2, &in_src));
    SGP_TRY(fill_i32(ctx, icnt, 0, n));
    k_uplinks<<<grid_for(n, 256), 256, 0, st>>>(n, elim, pos, up0, up1, upq, ka, in_src, icnt);
    LAUNCH_CHECK(ctx);
    int kbits = 1;
    while (((int64_t)1 << kbits) <= n) kbits++;
    SGP_TRY(radix_sort_pairs(ctx, ka, in_src, kb, vb, 2 * n, kbits));
    SGP_TRY(scan_exclusive(ctx, icnt, in_ptr, n));
    // numeric factorisation
    double *Pd, *E0, *E, *C, *F, *Dinv;
    int32_t *status;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP3], 9 * n + 9, &Pd));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP4], 9 * n + 9, &E0));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP5], 9 * n + 9, &E));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_SLOTS], 12 * n + 12, &C));
    SGP_TRY(ensure_t(ctx, M->F, 18 * n + 18, &F));
    SGP_TRY(ensure_t(ctx, M->Dinv, 6 * n + 6, &Dinv));
    double *y;
    SGP_TRY(ensure_t(ctx, M->y, 3 * n + 3, &y));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP9], 4, &status));
    SGP_TRY(fill_i32(ctx, status, 0, 1));
    SGP_TRY(fill_f64(ctx, F, 0.0, 18 * n));
    k_tree_blocks<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)T->tptr.p, (const int32_t *)T->tadje.p,
                                                  (const int32_t *)T->pedge.p, (const double4 *)g->wu.p, g_par,
                                                  g_perp, g_med, Pd, E0);
    k_permute9<<<grid_for(n, 256), 256, 0, st>>>(n, elim, E0, E);
    LAUNCH_CHECK(ctx);
    for (int k = 0; k < S; k++) {
        int32_t q0 = M->h_step_ptr[k], q1 = M->h_step_ptr[k + 1];
        if (q1 > q0)
            k_factor_step<<<grid_for(q1 - q0, 128), 128, 0, st>>>(q0, q1, elim, upq, in_ptr, in_src, Pd, E, C, F,
                                                                  Dinv, status);
    }
    LAUNCH_CHECK(ctx);
    SGP_TRY(readback(ctx, hbuf, status, 4));
    if (ctx->ev[7]) {
        (void)hipEventRecord(ctx->ev[7], st);
        (void)hipEventSynchronize(ctx->ev[7]);
        (void)hipEventElapsedTime(&ctx->phase_ms[3], ctx->ev[6], ctx->ev[7]);
    }
    if (hbuf[0]) return set_err(ctx, SGP_ENOTSPD, "factor_tree: a pivot block is not positive definite");
    return SGP_OK;
}

__global__ void k_jacobi_make(int64_t n, const int32_t *diagpos, const double *val, double *dinv, int32_t *status)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *B = val + 9 * (int64_t)diagpos[i];
    double D[9];
    for (int t = 0; t < 9; t++) D[t] = B[t];
    double inv[6];
    if (!spd_inverse3(D, inv)) {
        atomicOr(status, 1);
        for (int t = 0; t < 6; t++) inv[t] = 0.0;
    }
    for (int t = 0; t < 6; t++) dinv[6 * i + t] = inv[t];
}

extern "C" int sgp_make_jacobi(sgp_ctx ctx, sgp_bsr A, sgp_prec M)
{
    if (!ctx || !A || !M) return set_err(ctx, SGP_EINVAL, "make_jacobi: null handle");
    hipStream_t st = ctx->stream;
    M->kind = PREC_JACOBI;
    M->n = A->n;
    M->steps = 0;
    M->have32 = false;
    double *dinv;
    int32_t *status;
    SGP_TRY(ensure_t(ctx, M->jdinv, 6 * A->n + 6, &dinv));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_TMP9], 4, &status));
    SGP_TRY(fill_i32(ctx, status, 0, 1));
    if (A->n > 0)
        k_jacobi_make<<<grid_for(A->n, 256), 256, 0, st>>>(A->n, (const int32_t *)A->diagpos.p,
                                                         (const double *)A->val.p, dinv, status);
    LAUNCH_CHECK(ctx);
    int32_t *h = (int32_t *)ctx->pinned;
    SGP_TRY(readback(ctx, h, status, 4));
    if (h[0]) return set_err(ctx, SGP_ENOTSPD, "make_jacobi: a diagonal block is not positive definite");
    return SGP_OK;
}

extern "C" int sgp_prec_steps(sgp_prec M, int32_t *steps)
{
    if (!M || !steps) return SGP_EINVAL;
    *steps = M->steps;
    return SGP_OK;
}

extern "C" int sgp_prec_apply(sgp_ctx ctx, sgp_prec M, const double *r, double *z)
{
    if (!ctx || !M) return set_err(ctx, SGP_EINVAL, "prec_apply: null handle");
    if (M->n == 0) return SGP_OK;
    return prec_apply_f64(ctx, M, r, z, nullptr);
}
