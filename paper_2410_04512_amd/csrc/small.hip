// The whole PCG of one small system in one workgroup (Section 1.1's PCG with
// the tree preconditioner of Section 3.1, its factor by Alg. 2 and the sweeps
// of App. B.1).  A solve of a thousand cells takes ~130 iterations of a few
// microseconds of work each; as separate launches (product, two reductions,
// vector passes, the tail sweep) an iteration costs ~45 us of dispatch
// latency.  Here one workgroup of SMALL_THREADS threads runs every iteration:
// thread t owns the elimination positions n-1-t and n-1-t-SMALL_THREADS (so
// the last 64 positions, the few vertices of the last steps, belong to wave
// 0, which sweeps those steps alone with wave-level syncs), their rows
// (the cells elim[q]) of every CG vector, and the pivot and first coupling of
// those positions in registers; p (for the product's gathers), the sweeps'
// values, the push slots and the second coupling planes live in LDS; the
// matrix entries are read from L2 every iteration, from a copy in which
// entry s of the row of position z sits at s * SMALL_MAX + z (so a wave's
// loads of its rows' s-th entries are contiguous), built once per matrix and
// factor and kept with the factor.  The product and both
// sweeps do the operations of k_spmv_edge and k_tail in the same order, so
// the only rounding difference from the launch-per-kernel path is the order
// in which the dot products are summed.
//
// Conditions (small_solve_fits): one cluster, n <= SMALL_MAX cells, a tree
// factor whose elimination lies wholly in the tail (tail_step == 0), and its
// LDS tables within SMALL_LDS_BYTES.
#include "sgp_internal.h"

#include <algorithm>

constexpr int SMALL_THREADS = 512;
constexpr int SMALL_MAX = 2 * SMALL_THREADS;
constexpr int SMALL_LDS_BYTES = 160 * 1024;
constexpr int SMALL_CHUNK = 4;   // matrix entries per row loaded together

static size_t small_lds_bytes(int64_t n, int64_t ni, int64_t steps)
{
    // p / sweep values (3n), push slots (3 ni), second couplings (9n),
    // reduction buffers (2 x 4 x waves), step bounds (steps + 1)
    return 8 * (3 * (size_t)n + 3 * (size_t)ni + 9 * (size_t)n + 2 * 4 * (SMALL_THREADS / 64)) +
           4 * (size_t)(steps + 1);
}

bool small_solve_fits(sgp_ctx ctx, sgp_bsr A, sgp_prec M)
{
    // (not while a step is recorded: the copy of the entries below is built
    // on first use, so a recording and its capture would differ)
    if (!ctx->small_solve || !M || M->kind != PREC_TREE || M->aug || ctx->spmv_form != 1 ||
        ctx->plan_mode != PLAN_OFF)
        return false;
    const int64_t n = A->n;
    if (n < 1 || n > SMALL_MAX || M->n != n || M->steps < 1 || M->tail_step != 0 || M->tail_nt != n) return false;
    return small_lds_bytes(n, M->tail_ni, M->steps) <= (size_t)SMALL_LDS_BYTES;
}

struct SmallArgs {
    int32_t n, S, ni;
    const int32_t *ecnt;    // entries of the row of each position
    const int32_t *ecol;    // [deg][SMALL_MAX] columns
    const double *ew;       // [deg][EDGE_PLANES][SMALL_MAX] v = sqrt(w) u planes
    const double *dg;
    double gpar, gperp;
    const int32_t *sp, *elim, *iptr, *tslot, *upq;
    const double *F, *Dinv;
    int64_t fs;
    const double *f;   // force, internal order
    double *x;         // x0 in (use_x0), solution out; internal order
    PcgScalars *sc;
    double tol2;
    int32_t max_iter, fixed, use_x0;
};

// sums of NV values over the workgroup, in a fixed order (each wave by a
// butterfly, then the waves in order); every thread gets the totals.
// Two buffers, used in turn: a buffer is reused only after the barrier of the
// reduction between, so no barrier is needed after reading.
template <int NV>
SGP_DEV void small_sum(double *red, int &buf, double *v)
{
    constexpr int W = SMALL_THREADS / 64;
    double *b = red + buf * 4 * W;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < NV; a++) {
        double s = v[a];
        for (int o = 32; o > 0; o >>= 1) s = s + __shfl_xor(s, o, 64);
        if (lane == 0) b[a * W + wv] = s;
    }
    lds_barrier();
#pragma unroll
    for (int a = 0; a < NV; a++) {
        double s = b[a * W];
        for (int w = 1; w < W; w++) s = s + b[a * W + w];
        v[a] = s;
    }
    buf ^= 1;
}

// orders a wave's LDS accesses before and after it (lanes of one wave only)
SGP_DEV void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// the constants of one elimination position of a thread
struct SmallVtx {
    double d[6], f0[9];
    int32_t q, v, in0, in1, s0, s1, a0, a1, cnt, step;
    bool on;
};

__global__ __launch_bounds__(SMALL_THREADS) void k_small_pcg(SmallArgs A)
{
    extern __shared__ unsigned char lds_raw[];
    const int32_t n = A.n;
    double *pv = (double *)lds_raw;        // p by row (product), the sweeps' values by position
    double *slot = pv + 3 * (int64_t)n;    // push slots
    double *f1l = slot + 3 * (int64_t)A.ni;   // second coupling planes
    double *red = f1l + 9 * (int64_t)n;
    int32_t *ssp = (int32_t *)(red + 2 * 4 * (SMALL_THREADS / 64));
    const int tid = threadIdx.x;
    for (int32_t k = tid; k <= A.S; k += SMALL_THREADS) ssp[k] = A.sp[k];
    for (int64_t i = tid; i < 9 * (int64_t)n; i += SMALL_THREADS) f1l[i] = A.F[A.fs + i];
    SmallVtx V[2];
#pragma unroll
    for (int u = 0; u < 2; u++) {
        const int32_t q = n - 1 - (tid + SMALL_THREADS * u);
        SmallVtx &c = V[u];
        c.on = q >= 0;
        const int32_t qc = c.on ? q : 0;
        c.q = qc;
        c.v = A.elim[qc];
        for (int t = 0; t < 6; t++) c.d[t] = A.Dinv[6 * (int64_t)qc + t];
        for (int t = 0; t < 9; t++) c.f0[t] = A.F[9 * (int64_t)qc + t];
        c.in0 = A.iptr[qc];
        c.in1 = A.iptr[qc + 1];
        c.s0 = A.tslot[2 * qc];
        c.s1 = A.tslot[2 * qc + 1];
        c.a0 = A.upq[2 * qc];
        c.a1 = A.upq[2 * qc + 1];
        c.cnt = c.on ? A.ecnt[qc] : 0;
    }
    // (a position past n keeps zeros: its values are computed and never used)
    double f[2][3], x[2][3], r[2][3] = {}, p[2][3] = {}, q[2][3] = {}, z[2][3] = {};
    double acc[3] = {0.0, 0.0, 0.0};   // ||f||^2, ||r||^2, non-finite count
#pragma unroll
    for (int u = 0; u < 2; u++)
        for (int t = 0; t < 3; t++) {
            f[u][t] = A.f[3 * (int64_t)V[u].v + t];
            x[u][t] = A.use_x0 ? A.x[3 * (int64_t)V[u].v + t] : 0.0;
        }
    __syncthreads();
    // the elimination step of each of the thread's positions (-1: none)
#pragma unroll
    for (int u = 0; u < 2; u++) {
        const int32_t qq = V[u].q;
        V[u].step = -1;
        if (V[u].on)
            for (int32_t k = 0; k < A.S; k++)
                if (qq >= ssp[k] && qq < ssp[k + 1]) V[u].step = k;
    }
    // the first step whose positions all lie in the last 64 (wave 0's)
    int32_t kw = A.S;
    while (kw > 0 && n - ssp[kw - 1] <= 64) kw--;
    int buf = 0;

    // q = Gamma p for the thread's rows, p of all rows in pv (by row):
    // diagonal block first, then minus every entry's W_e p_j in entry order
    auto product = [&]() {
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const SmallVtx &c = V[u];
            const double *g = A.dg + ((int64_t)c.v >> 6) * 384 + (c.v & 63);
            double dr[6];
            for (int t = 0; t < 6; t++) dr[t] = g[64 * t];
            const double p0 = p[u][0], p1 = p[u][1], p2 = p[u][2];
            q[u][0] = dr[0] * p0 + dr[1] * p1 + dr[2] * p2;
            q[u][1] = dr[1] * p0 + dr[3] * p1 + dr[4] * p2;
            q[u][2] = dr[2] * p0 + dr[4] * p1 + dr[5] * p2;
            // the row's entries, SMALL_CHUNK at a time (the loads of a chunk
            // issued together, and only for the entries the row has).
            // Loading both rows' chunks in one round measured slower.
            const int64_t z = c.q;
            for (int32_t base = 0; base < c.cnt; base += SMALL_CHUNK) {
                double e[SMALL_CHUNK][EDGE_PLANES];
                int32_t j[SMALL_CHUNK];
#pragma unroll
                for (int s = 0; s < SMALL_CHUNK; s++) {
                    const int64_t sk = min(base + s, c.cnt - 1);
                    for (int t = 0; t < EDGE_PLANES; t++) e[s][t] = A.ew[(EDGE_PLANES * sk + t) * SMALL_MAX + z];
                    j[s] = A.ecol[sk * SMALL_MAX + z];
                }
#pragma unroll
                for (int s = 0; s < SMALL_CHUNK; s++) {
                    if (base + s >= c.cnt) break;
                    const int64_t jj = j[s];
                    const double x0 = pv[3 * jj], x1 = pv[3 * jj + 1], x2 = pv[3 * jj + 2];
                    double o0, o1, o2;
                    edge_wp(e[s][0], e[s][1], e[s][2], x0, x1, x2, A.gpar, A.gperp, o0, o1, o2);
                    q[u][0] -= o0;
                    q[u][1] -= o1;
                    q[u][2] -= o2;
                }
            }
        }
    };
    // z = P^{-1} r by the two sweeps over the elimination steps; pv holds
    // y, then x, by elimination position
    // one elimination step of the forward sweep for the thread's positions
    auto fwd_step = [&](int32_t k) {
#pragma unroll
        for (int u = 0; u < 2; u++) {
            if (V[u].step != k) continue;
            const int32_t qq = V[u].q;
            const SmallVtx &c = V[u];
            // the second coupling (zero without a second link) and the
            // in-slots, four at a time (clamped addresses, surplus masked),
            // read ahead of their use
            double g1[9];
            const double *gs = f1l + 9 * (int64_t)qq;
            for (int t = 0; t < 9; t++) g1[t] = gs[t];
            double c0 = r[u][0], c1 = r[u][1], c2 = r[u][2];
            for (int32_t s = c.in0; s < c.in1; s += 4) {
                double h[12];
#pragma unroll
                for (int m = 0; m < 4; m++) {
                    const int32_t sm = min(s + m, c.in1 - 1);
                    h[3 * m] = slot[3 * sm];
                    h[3 * m + 1] = slot[3 * sm + 1];
                    h[3 * m + 2] = slot[3 * sm + 2];
                }
#pragma unroll
                for (int m = 0; m < 4; m++) {
                    const bool on = s + m < c.in1;
                    c0 = on ? c0 - h[3 * m] : c0;
                    c1 = on ? c1 - h[3 * m + 1] : c1;
                    c2 = on ? c2 - h[3 * m + 2] : c2;
                }
            }
            double o0, o1, o2;
            sym_mv(c.d, c0, c1, c2, o0, o1, o2);
            pv[3 * qq] = o0;
            pv[3 * qq + 1] = o1;
            pv[3 * qq + 2] = o2;
            if (c.s0 >= 0) {
                const double *g = c.f0;
                slot[3 * c.s0] = g[0] * o0 + g[1] * o1 + g[2] * o2;
                slot[3 * c.s0 + 1] = g[3] * o0 + g[4] * o1 + g[5] * o2;
                slot[3 * c.s0 + 2] = g[6] * o0 + g[7] * o1 + g[8] * o2;
            }
            if (c.s1 >= 0) {
                const double *g = g1;
                slot[3 * c.s1] = g[0] * o0 + g[1] * o1 + g[2] * o2;
                slot[3 * c.s1 + 1] = g[3] * o0 + g[4] * o1 + g[5] * o2;
                slot[3 * c.s1 + 2] = g[6] * o0 + g[7] * o1 + g[8] * o2;
            }
        }
    };
    // one elimination step of the backward sweep
    auto bwd_step = [&](int32_t k) {
#pragma unroll
        for (int u = 0; u < 2; u++) {
            if (V[u].step != k) continue;
            const int32_t qq = V[u].q;
            const SmallVtx &c = V[u];
            // every LDS read of the vertex first: own y, x of both
            // up-links (a missing link reads the vertex's own y, masked)
            // and the second coupling
            const int32_t b0 = c.a0 >= 0 ? c.a0 : qq, b1 = c.a1 >= 0 ? c.a1 : qq;
            const double y0 = pv[3 * qq], y1 = pv[3 * qq + 1], y2 = pv[3 * qq + 2];
            const double p0 = pv[3 * b0], p1 = pv[3 * b0 + 1], p2 = pv[3 * b0 + 2];
            const double x0 = pv[3 * b1], x1 = pv[3 * b1 + 1], x2 = pv[3 * b1 + 2];
            double g1[9];
            const double *gs = f1l + 9 * (int64_t)qq;
            for (int t = 0; t < 9; t++) g1[t] = gs[t];
            double c0 = 0, c1 = 0, c2 = 0;
            if (c.a0 >= 0) {
                const double *g = c.f0;
                c0 = c0 + (g[0] * p0 + g[3] * p1 + g[6] * p2);
                c1 = c1 + (g[1] * p0 + g[4] * p1 + g[7] * p2);
                c2 = c2 + (g[2] * p0 + g[5] * p1 + g[8] * p2);
            }
            if (c.a1 >= 0) {
                const double *g = g1;
                c0 = c0 + (g[0] * x0 + g[3] * x1 + g[6] * x2);
                c1 = c1 + (g[1] * x0 + g[4] * x1 + g[7] * x2);
                c2 = c2 + (g[2] * x0 + g[5] * x1 + g[8] * x2);
            }
            double d0, d1, d2;
            sym_mv(c.d, c0, c1, c2, d0, d1, d2);
            const double n0 = y0 - d0, n1 = y1 - d1, n2 = y2 - d2;
            pv[3 * qq] = n0;
            pv[3 * qq + 1] = n1;
            pv[3 * qq + 2] = n2;
            z[u][0] = n0;
            z[u][1] = n1;
            z[u][2] = n2;
        }
    };
    // z = P^{-1} r by the two sweeps over the elimination steps; pv holds
    // y, then x, by elimination position.  Steps from kw on lie in the last
    // 64 positions: wave 0 runs them (forward, then backward) alone, with
    // wave-level syncs; the others take a barrier of the workgroup each.
    auto sweeps = [&]() {
        for (int32_t k = 0; k < kw; k++) {
            fwd_step(k);
            lds_barrier();
        }
        if (tid < 64) {
            for (int32_t k = kw; k < A.S; k++) {
                fwd_step(k);
                wave_lds_sync();
            }
            for (int32_t k = A.S - 1; k >= kw; k--) {
                bwd_step(k);
                wave_lds_sync();
            }
        }
        lds_barrier();
        for (int32_t k = kw - 1; k >= 0; k--) {
            bwd_step(k);
            lds_barrier();
        }
    };
    auto publish_p = [&]() {
#pragma unroll
        for (int u = 0; u < 2; u++)
            if (V[u].on)
                for (int t = 0; t < 3; t++) pv[3 * (int64_t)V[u].v + t] = p[u][t];
        lds_barrier();
    };

    // r = f - Gamma x0 (or f)
    if (A.use_x0) {
#pragma unroll
        for (int u = 0; u < 2; u++)
            for (int t = 0; t < 3; t++) p[u][t] = x[u][t];
        publish_p();
        product();
    }
#pragma unroll
    for (int u = 0; u < 2; u++) {
        if (!V[u].on) continue;
        for (int t = 0; t < 3; t++) {
            const double ft = f[u][t];
            const double rt = A.use_x0 ? ft - q[u][t] : ft;
            r[u][t] = rt;
            if (!isfinite(ft) || (A.use_x0 && !isfinite(x[u][t]))) acc[2] = 1.0;
            acc[0] = acc[0] + ft * ft;
            acc[1] = acc[1] + rt * rt;
        }
    }
    small_sum<3>(red, buf, acc);
    const double nF2 = acc[0];
    double rr = acc[1];
    int32_t status = SGP_OK, iter = 0, done = 0;
    double relres2 = nF2 > 0.0 ? rr / nF2 : 0.0;
    if (acc[2] != 0.0 || !isfinite(rr)) {
        status = SGP_ENONFINITE;
        done = 1;
    } else if (nF2 == 0.0) {
        done = 2;   // zero force: v = 0
#pragma unroll
        for (int u = 0; u < 2; u++)
            for (int t = 0; t < 3; t++) x[u][t] = 0.0;
    } else if (!A.fixed && relres2 <= A.tol2) {
        done = 1;
    }
    if (!done) {
        __syncthreads();   // the product's reads of pv are over
        sweeps();
        double rho[1] = {0.0};
#pragma unroll
        for (int u = 0; u < 2; u++)
            if (V[u].on)
                for (int t = 0; t < 3; t++) {
                    p[u][t] = z[u][t];
                    rho[0] = rho[0] + r[u][t] * z[u][t];
                }
        small_sum<1>(red, buf, rho);
        double rh = rho[0];
        for (;;) {
            publish_p();
            product();
            double pq[1] = {0.0};
#pragma unroll
            for (int u = 0; u < 2; u++)
                if (V[u].on)
                    for (int t = 0; t < 3; t++) pq[0] = pq[0] + p[u][t] * q[u][t];
            small_sum<1>(red, buf, pq);
            if (!(pq[0] > 0.0) || !isfinite(pq[0])) {
                status = SGP_EBREAKDOWN;
                break;
            }
            const double alpha = rh / pq[0];
            double rs[1] = {0.0};
#pragma unroll
            for (int u = 0; u < 2; u++)
                if (V[u].on)
                    for (int t = 0; t < 3; t++) {
                        r[u][t] = r[u][t] - alpha * q[u][t];
                        rs[0] = rs[0] + r[u][t] * r[u][t];
                    }
            small_sum<1>(red, buf, rs);
            rr = rs[0];
            iter++;
            relres2 = rr / nF2;
            if (!isfinite(rr)) {
                status = SGP_ENONFINITE;
                break;
            }
            bool stop = false;
            if (A.fixed) {
                stop = iter >= A.fixed;
            } else if (relres2 <= A.tol2) {
                stop = true;
            } else if (iter >= A.max_iter) {
                status = SGP_ENOCONV;
                stop = true;
            }
            if (stop) {   // the last x update only
#pragma unroll
                for (int u = 0; u < 2; u++)
                    for (int t = 0; t < 3; t++) x[u][t] = x[u][t] + alpha * p[u][t];
                break;
            }
            __syncthreads();   // the product's reads of pv are over
            sweeps();
            double rz[1] = {0.0};
#pragma unroll
            for (int u = 0; u < 2; u++)
                if (V[u].on)
                    for (int t = 0; t < 3; t++) rz[0] = rz[0] + r[u][t] * z[u][t];
            small_sum<1>(red, buf, rz);
            const double beta = rz[0] / rh;
            rh = rz[0];
#pragma unroll
            for (int u = 0; u < 2; u++)
                for (int t = 0; t < 3; t++) {
                    x[u][t] = x[u][t] + alpha * p[u][t];
                    p[u][t] = z[u][t] + beta * p[u][t];
                }
        }
        done = 1;
    }
#pragma unroll
    for (int u = 0; u < 2; u++)
        if (V[u].on)
            for (int t = 0; t < 3; t++) A.x[3 * (int64_t)V[u].v + t] = x[u][t];
    if (tid == 0) {
        PcgScalars *s = A.sc;
        s->nF2 = nF2;
        s->rr = rr;
        s->relres2 = relres2;
        s->iter = iter;
        s->status = status;
        s->done = done;
    }
}

// entries of the row of every position, and their maximum (one workgroup)
__global__ __launch_bounds__(SMALL_MAX) void k_small_deg(int32_t n, const int32_t *elim, const int32_t *rowptr,
                                                        int32_t *cnt, int32_t *maxd)
{
    __shared__ int32_t sh[SMALL_MAX / 64];
    const int32_t q = threadIdx.x;
    int32_t c = 0;
    if (q < n) {
        const int32_t v = elim[q];
        c = rowptr[v + 1] - rowptr[v] - 1;   // the block row less its diagonal block
    }
    cnt[q] = c;
    for (int o = 32; o > 0; o >>= 1) c = max(c, __shfl_xor(c, o, 64));
    if ((q & 63) == 0) sh[q >> 6] = c;
    __syncthreads();
    if (q == 0) {
        int32_t m = sh[0];
        for (int w = 1; w < SMALL_MAX / 64; w++) m = max(m, sh[w]);
        maxd[0] = m;
    }
}

// the copy: entry s of the row of position z at s * SMALL_MAX + z
__global__ void k_small_ell(int32_t n, int32_t deg, const int32_t *elim, const int32_t *rowptr, const int32_t *cnt,
                            const int32_t *ecol, const double *ew, int32_t *ecol_out, double *ew_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t z = (int32_t)(i % SMALL_MAX), s = (int32_t)(i / SMALL_MAX);
    if (s >= deg || z >= n || s >= cnt[z]) return;
    const int32_t v = elim[z];
    const int64_t k = (int64_t)rowptr[v] - v + s;
    ecol_out[(int64_t)s * SMALL_MAX + z] = ecol[k];
    const double *g = ew + (k >> 6) * (64 * EDGE_PLANES) + (k & 63);
    for (int t = 0; t < EDGE_PLANES; t++) ew_out[(int64_t)(EDGE_PLANES * s + t) * SMALL_MAX + z] = g[64 * t];
}

// the factor's copy of the matrix entries, built when the matrix or the
// factor changed since the last one
static int small_ell(sgp_ctx ctx, sgp_bsr A, sgp_prec M)
{
    if (M->small_ell.p && M->small_a_gen == A->gen && M->small_m_gen == M->gen) return SGP_OK;
    hipStream_t st = ctx->stream;
    const int32_t n = (int32_t)A->n;
    const int32_t *elim = (const int32_t *)M->elim_int.p, *rowptr = (const int32_t *)A->rowptr.p;
    int32_t *tmp;
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_PAIR], SMALL_MAX + 2, &tmp));
    k_small_deg<<<1, SMALL_MAX, 0, st>>>(n, elim, rowptr, tmp, tmp + SMALL_MAX);
    LAUNCH_CHECK(ctx);
    int32_t deg = 0;
    SGP_TRY(readback(ctx, &deg, tmp + SMALL_MAX, 4));
    // [cnt: SMALL_MAX][ecol: deg x SMALL_MAX] int32, then [deg][EDGE_PLANES][SMALL_MAX] doubles
    const size_t ints = (size_t)(1 + deg) * SMALL_MAX;
    const size_t bytes = 4 * ints + 8 * EDGE_PLANES * (size_t)deg * SMALL_MAX + 8;
    int32_t *e;
    SGP_TRY(ensure_t(ctx, M->small_ell, bytes / 4 + 2, &e));
    HIP_TRY(ctx, hipMemcpyAsync(e, tmp, 4 * SMALL_MAX, hipMemcpyDeviceToDevice, st));
    if (deg > 0) {
        const int64_t total = (int64_t)deg * SMALL_MAX;
        k_small_ell<<<grid_for(total, 256), 256, 0, st>>>(n, deg, elim, rowptr, e, (const int32_t *)A->ecol.p,
                                                         (const double *)A->ew.p, e + SMALL_MAX,
                                                         (double *)(e + ints));
        LAUNCH_CHECK(ctx);
    }
    M->small_deg = deg;
    M->small_a_gen = A->gen;
    M->small_m_gen = M->gen;
    return SGP_OK;
}

// One solve on F, x (internal order) into S[0]; x0 read when use_x0
int solve_small(sgp_ctx ctx, sgp_bsr A, sgp_prec M, const double *F, double *x, const sgp_solve_opts *o,
                PcgScalars *S)
{
    static bool attr = false;
    if (!attr) {
        HIP_TRY(ctx, hipFuncSetAttribute((const void *)k_small_pcg, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         SMALL_LDS_BYTES));
        attr = true;
    }
    const int64_t n = A->n;
    SGP_TRY(small_ell(ctx, A, M));
    const int32_t *e = (const int32_t *)M->small_ell.p;
    SmallArgs a;
    a.n = (int32_t)n;
    a.S = M->steps;
    a.ni = M->tail_ni;
    a.ecnt = e;
    a.ecol = e + SMALL_MAX;
    a.ew = (const double *)(e + (size_t)(1 + M->small_deg) * SMALL_MAX);
    a.dg = (const double *)A->dg.p;
    a.gpar = A->gpar;
    a.gperp = A->gperp;
    a.sp = (const int32_t *)M->step_ptr.p;
    a.elim = (const int32_t *)M->elim_int.p;
    a.iptr = (const int32_t *)M->tail_iptr.p;
    a.tslot = (const int32_t *)M->tail_tslot.p;
    a.upq = (const int32_t *)M->up.p;
    a.F = (const double *)M->F.p;
    a.Dinv = (const double *)M->Dinv.p;
    a.fs = 9 * n;
    a.f = F;
    a.x = x;
    a.sc = S;
    a.tol2 = o->rtol * o->rtol;
    a.max_iter = o->max_iter > 0 ? o->max_iter : 10000;
    a.fixed = std::max(0, o->fixed_iters);
    a.use_x0 = o->use_x0 ? 1 : 0;
    const size_t lds = small_lds_bytes(n, M->tail_ni, M->steps);
    k_small_pcg<<<1, SMALL_THREADS, lds, ctx->stream>>>(a);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}
