// Steps 2 and 5 of Section 2 for the time-stepping workload: contact forces
// and the forward Euler update.
//
// F_i = noise_i + sum over the contacts j of i, in ascending j, of
//       k_rep w_ij (r_i - r_j) / d_ij,
// where (r_i - r_j)/d_ij = -u_e for i < j and +u_e for i > j (u_e points from
// the smaller to the larger id).  One thread per cell gathers its row, so no
// atomics are needed and the sum order is fixed.
#include "sgp_internal.h"

__global__ void k_forces(int64_t n, const int32_t *rowptr, const int32_t *col, const int32_t *ent_edge,
                         const double4 *wu, double k_rep, const double *noise, double *F)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
        double4 q = wu[ent_edge[p]];
        double s = (i < col[p]) ? -1.0 : 1.0;
        double mag = k_rep * q.x;
        a0 = a0 + mag * (s * q.y);
        a1 = a1 + mag * (s * q.z);
        a2 = a2 + mag * (s * q.w);
    }
    F[3 * i] = a0 + noise[3 * i];
    F[3 * i + 1] = a1 + noise[3 * i + 1];
    F[3 * i + 2] = a2 + noise[3 * i + 2];
}

__global__ void k_euler(int64_t len, double dt, const double *v, double *pos)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) pos[t] = pos[t] + dt * v[t];
}

extern "C" int sgp_forces(sgp_ctx ctx, sgp_graph g, double k_rep, const double *noise, double *F)
{
    if (!ctx || !g || (g->n > 0 && (!noise || !F))) return set_err(ctx, SGP_EINVAL, "forces: bad arguments");
    if (g->n == 0) return SGP_OK;
    k_forces<<<grid_for(g->n, 256), 256, 0, ctx->stream>>>(g->n, (const int32_t *)g->rowptr.p,
                                                          (const int32_t *)g->col.p, (const int32_t *)g->ent_edge.p,
                                                          (const double4 *)g->wu.p, k_rep, noise, F);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

extern "C" int sgp_euler(sgp_ctx ctx, int64_t n, double dt, const double *v, double *pos)
{
    if (!ctx || n < 0 || (n > 0 && (!v || !pos))) return set_err(ctx, SGP_EINVAL, "euler: bad arguments");
    if (n == 0) return SGP_OK;
    k_euler<<<grid_for(3 * n, 256), 256, 0, ctx->stream>>>(3 * n, dt, v, pos);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}
