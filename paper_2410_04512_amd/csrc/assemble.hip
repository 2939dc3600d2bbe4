// Step 3 of Section 2: the friction matrix Gamma as a 3x3-block CSR matrix.
//
// Gamma is the block Laplacian of the collision graph (Section 2, definition
// of the block Laplacian): for a contact e = (i, j) with overlap w and unit
// vector u, W_e = w (g_par u u^T + g_perp (I - u u^T)) (eq.
// cell_cell_friction); Gamma_ij = Gamma_ji = -W_e; Gamma_ii = g_med I plus
// the W_e of i's contacts.  In the caller's numbering (the export), row i of
// the block matrix is row i of the neighbour list with the diagonal block
// inserted in column order, so block k of row i sits at rowptr[i] + i + k'.
// The diagonal sum runs over the neighbours in ascending column order, with
// the same operation order as the definition (no fused multiply-add), so the
// assembled values are reproducible bit for bit.
#include "sgp_internal.h"

SGP_DEV void friction_block_asm(double w, double ux, double uy, double uz, double gpar, double gperp, double *W)
{
    const double u[3] = {ux, uy, uz};
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double uu = u[a] * u[b];
            double id = (a == b) ? 1.0 : 0.0;
            W[3 * a + b] = w * (gpar * uu + gperp * (id - uu));
        }
}

SGP_DEV void put_sym(double *val, int64_t k, const double *B)
{
    double *g = val + (k >> 6) * 384 + (k & 63);
    g[0] = B[0];
    g[64] = B[1];
    g[128] = B[2];
    g[192] = B[4];
    g[256] = B[5];
    g[320] = B[8];
}

// internal row i holds caller row perm[i] plus its diagonal block
__global__ void k_int_degree(int64_t n, const int32_t *rowptr, const int32_t *perm, int32_t *d)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t u = perm[i];
    d[i] = rowptr[u + 1] - rowptr[u] + 1;
}

// Gamma in the internal order.  Row i (caller row perm[i]) holds the
// off-diagonal blocks -W_e in the caller row's neighbour order, then the
// diagonal block, summed over the same neighbours in the same (the
// definition's) order.  Any fixed block order within a row serves the
// product, which sums a row's blocks in storage order; this one needs no
// per-row sort.  ASM_LANES threads share a row, one block each, so a wave's
// stores land in runs of consecutive blocks; the row's first thread also
// forms the diagonal block.
constexpr int ASM_LANES = 16;

__global__ __launch_bounds__(256) void k_assemble(int64_t n, const int32_t *rowptr, const int32_t *col,
                                                  const int32_t *ent_edge, const double4 *wu, const int32_t *perm,
                                                  const int32_t *inv, double gpar, double gperp, double gmed,
                                                  const int32_t *brow, int32_t *bcol, double *val,
                                                  int32_t *diagpos, int32_t *ecol, double *ew, double *dg)
{
    // per 16-lane group: the 16 blocks W of one round, for the diagonal sum
    __shared__ double sW[256 / ASM_LANES][ASM_LANES][9];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / ASM_LANES;
    const int c0 = (int)(t % ASM_LANES);
    const int grp = threadIdx.x / ASM_LANES;
    const bool row_ok = i < n;
    int32_t b = 0, e = 0;
    int64_t k0 = 0;
    if (row_ok) {
        const int32_t u = perm[i];
        b = rowptr[u];
        e = rowptr[u + 1];
        k0 = brow[i];
    }
    const int deg = e - b;
    // rounds of 16 blocks; the same count for the whole wave (its largest row)
    int rounds = (deg + ASM_LANES - 1) / ASM_LANES;
    for (int o = 32; o > 0; o >>= 1) {
        const int r2 = __shfl_xor(rounds, o, 64);
        rounds = r2 > rounds ? r2 : rounds;
    }
    // lane x < 9 of the group keeps entry x of the diagonal block and adds the
    // blocks' entry x in the row's neighbour order, as the definition sums them
    double d = (c0 < 9 && c0 % 4 == 0) ? gmed : 0.0;
    for (int r = 0; r < rounds; r++) {
        const int c = r * ASM_LANES + c0;
        double W[9];
        for (int x = 0; x < 9; x++) W[x] = 0.0;
        if (row_ok && c < deg) {
            // both gathers before the first store (a load behind a store waits for it)
            const double4 q = wu[ent_edge[b + c]];
            const int32_t jc = inv[col[b + c]];
            double B[9];
            friction_block_asm(q.x, q.y, q.z, q.w, gpar, gperp, W);
            for (int x = 0; x < 9; x++) B[x] = -W[x];
            if (val) {
                put_sym(val, k0 + c, B);
                bcol[k0 + c] = jc;
            }
            if (ew) {
                // edge form: entry k0 + c - i keeps v = sqrt(w) u
                const int64_t ke = k0 + c - i;
                double *g = ew + (ke >> 6) * (64 * EDGE_PLANES) + (ke & 63);
                const double sw = sqrt(q.x);
                g[0] = sw * q.y;
                g[64] = sw * q.z;
                g[128] = sw * q.w;
                ecol[ke] = jc;
            }
        }
        for (int x = 0; x < 9; x++) sW[grp][c0][x] = W[x];
        // lanes exchange through LDS within their wave only
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
        if (c0 < 9) {
            const int kmax = deg - r * ASM_LANES < ASM_LANES ? deg - r * ASM_LANES : ASM_LANES;
            for (int k = 0; k < kmax; k++) d = d + sW[grp][k][c0];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    }
    if (!row_ok) return;
    // the six distinct entries of the symmetric diagonal block, one per lane
    const int slot = c0 == 0 ? 0 : c0 == 1 ? 1 : c0 == 2 ? 2 : c0 == 4 ? 3 : c0 == 5 ? 4 : c0 == 8 ? 5 : -1;
    const int64_t k = k0 + deg;
    if (slot >= 0) {
        if (val) val[(k >> 6) * 384 + 64 * slot + (k & 63)] = d;
        if (ew) dg[(i >> 6) * 384 + 64 * slot + (i & 63)] = d;
    }
    if (c0 == 0 && val) {
        bcol[k] = (int32_t)i;
        diagpos[i] = (int32_t)k;
    }
}

// Gamma in the caller's numbering, 9 entries per block (for export)
__global__ void k_assemble_canon(int64_t n, const int32_t *rowptr, const int32_t *col, const int32_t *ent_edge,
                                 const double4 *wu, double gpar, double gperp, double gmed, int32_t *brow,
                                 int32_t *bcol, double *val)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = rowptr[i], e = rowptr[i + 1];
    const int64_t base = (int64_t)b + i;
    double D[9];
    for (int t = 0; t < 9; t++) D[t] = (t % 4 == 0) ? gmed : 0.0;
    int64_t dpos = base + (e - b);
    bool placed = false;
    for (int32_t p = b; p < e; p++) {
        int32_t j = col[p];
        if (!placed && j > i) {
            dpos = base + (p - b);
            placed = true;
        }
        int64_t k = base + (p - b) + (placed ? 1 : 0);
        double4 q = wu[ent_edge[p]];
        double W[9];
        friction_block_asm(q.x, q.y, q.z, q.w, gpar, gperp, W);
        for (int t = 0; t < 9; t++) {
            if (val) val[9 * k + t] = -W[t];
            D[t] = D[t] + W[t];
        }
        if (bcol) bcol[k] = j;
    }
    if (val)
        for (int t = 0; t < 9; t++) val[9 * dpos + t] = D[t];
    if (bcol) bcol[dpos] = (int32_t)i;
    if (brow) {
        brow[i] = (int32_t)base;
        if (i == n - 1) brow[n] = (int32_t)(e + n);
    }
}

extern "C" int sgp_assemble_gamma(sgp_ctx ctx, sgp_graph g, double g_par, double g_perp, double g_med, sgp_bsr A)
{
    if (!ctx || !g || !A) return set_err(ctx, SGP_EINVAL, "assemble_gamma: null handle");
    if (!(g_par > 0) || !(g_perp > 0) || !(g_med >= 0))
        return set_err(ctx, SGP_EINVAL, "assemble_gamma: need g_par > 0, g_perp > 0, g_med >= 0");
    hipStream_t st = ctx->stream;
    phase_begin(ctx, 1);
    const int64_t n = g->n, nnzb = n + 2 * g->m;
    A->gen = next_gen();
    A->n = n;
    A->nnzb = nnzb;
    A->have32 = A->have_val32 = false;
    A->have_blocks = false;
    A->src_version = g->version;
    int32_t *brow, *deg, *ecol;
    double *ew, *dg;
    const int64_t ne = 2 * g->m;
    SGP_TRY(ensure_t(ctx, A->rowptr, n + 1, &brow));
    SGP_TRY(ensure_t(ctx, A->ecol, ne + 1, &ecol));
    SGP_TRY(ensure_t(ctx, A->ew, edge_group_size(ne) + 8, &ew));
    SGP_TRY(ensure_t(ctx, A->dg, sym_group_size(n) + 8, &dg));
    A->src = g;
    A->gpar = g_par;
    A->gperp = g_perp;
    A->gmed = g_med;
    if (n == 0) {
        A->nwaves = 0;
        return fill_i32(ctx, brow, 0, 1);
    }
    SGP_TRY(copy_order(ctx, A->perm, A->inv, g->perm, g->inv, n));
    // zero the padding of the last groups (read by no row, kept finite)
    SGP_TRY(fill_f64(ctx, dg + (sym_group_size(n) - 384), 0.0, 384));
    if (ne > 0) SGP_TRY(fill_f64(ctx, ew + (edge_group_size(ne) - 64 * EDGE_PLANES), 0.0, 64 * EDGE_PLANES));
    SGP_TRY(ensure_t(ctx, ctx->ws[WS_DEG], n + 1, &deg));
    k_int_degree<<<grid_for(n, 256), 256, 0, st>>>(n, (const int32_t *)g->rowptr.p, (const int32_t *)g->perm.p, deg);
    SGP_TRY(scan_exclusive(ctx, deg, brow, n));
    k_assemble<<<grid_for(ASM_LANES * n, 256), 256, 0, st>>>(n, (const int32_t *)g->rowptr.p, (const int32_t *)g->col.p,
                                                 (const int32_t *)g->ent_edge.p, (const double4 *)g->wu.p,
                                                 (const int32_t *)g->perm.p, (const int32_t *)g->inv.p, g_par,
                                                 g_perp, g_med, brow, nullptr, nullptr, nullptr, ecol, ew, dg);
    LAUNCH_CHECK(ctx);
    // the 3x3 blocks only for the block-CSR product (else on first use)
    if (ctx->spmv_form == 0) SGP_TRY(bsr_blocks(ctx, A));
    SGP_TRY(bsr_prepare(ctx, A));
    phase_end(ctx, 1);
    return SGP_OK;
}

// Gamma's 3x3 blocks in block CSR (val, bcol, diagpos), read only by the
// block-CSR product (spmv_form 0) and its FP32 copy: assembled with the edge
// form when that product is the knob's choice, else on first use, by the
// same kernel from the same graph (so bit for bit the same values; an error
// if the graph has been collided again since).
int bsr_blocks(sgp_ctx ctx, sgp_bsr A)
{
    if (A->have_blocks) return SGP_OK;
    const int64_t n = A->n, nnzb = A->nnzb;
    int32_t *bcol, *dpos;
    double *val;
    SGP_TRY(ensure_t(ctx, A->bcol, nnzb + 1, &bcol));
    SGP_TRY(ensure_t(ctx, A->val, sym_group_size(nnzb) + 8, &val));
    SGP_TRY(ensure_t(ctx, A->diagpos, n + 1, &dpos));
    if (n > 0) {
        sgp_graph g = A->src;
        if (!g || g->n != n || g->version != A->src_version)
            return set_err(ctx, SGP_ESTALE, "Gamma's blocks: the graph was collided again since the assembly");
        SGP_TRY(fill_f64(ctx, val + (sym_group_size(nnzb) - 384), 0.0, 384));
        k_assemble<<<grid_for(ASM_LANES * n, 256), 256, 0, ctx->stream>>>(
            n, (const int32_t *)g->rowptr.p, (const int32_t *)g->col.p, (const int32_t *)g->ent_edge.p,
            (const double4 *)g->wu.p, (const int32_t *)g->perm.p, (const int32_t *)g->inv.p, A->gpar, A->gperp,
            A->gmed, (const int32_t *)A->rowptr.p, bcol, val, dpos, nullptr, nullptr, nullptr);
        LAUNCH_CHECK(ctx);
    }
    A->have_blocks = true;
    return SGP_OK;
}

extern "C" int sgp_bsr_size(sgp_bsr A, int64_t *n, int64_t *nnzb)
{
    if (!A) return SGP_EINVAL;
    if (n) *n = A->n;
    if (nnzb) *nnzb = A->nnzb;
    return SGP_OK;
}

// The export is Gamma in the caller's numbering, rebuilt from the graph it
// was assembled from (same arithmetic, so the same values bit for bit).
extern "C" int sgp_bsr_export(sgp_ctx ctx, sgp_bsr A, int32_t *rowptr, int32_t *bcol, double *val)
{
    if (!ctx || !A) return set_err(ctx, SGP_EINVAL, "bsr_export: null handle");
    if (A->n == 0) {
        if (rowptr) SGP_TRY(fill_i32(ctx, rowptr, 0, 1));
        return SGP_OK;
    }
    sgp_graph g = A->src;
    if (!g || g->n != A->n) return set_err(ctx, SGP_EINVAL, "bsr_export: the source graph changed or was freed");
    k_assemble_canon<<<grid_for(A->n, 128), 128, 0, ctx->stream>>>(
        A->n, (const int32_t *)g->rowptr.p, (const int32_t *)g->col.p, (const int32_t *)g->ent_edge.p,
        (const double4 *)g->wu.p, A->gpar, A->gperp, A->gmed, rowptr, bcol, val);
    LAUNCH_CHECK(ctx);
    return SGP_OK;
}

__global__ void k_round32(int64_t len, const double *a, float *b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) b[i] = (float)a[i];
}

// FP32 copy of the values for the refinement's inner solve (rounded once,
// same layout)
int bsr_make32(sgp_ctx ctx, sgp_bsr A)
{
    // the blocks' FP32 copy for the block-CSR product only
    if (ctx->spmv_form == 0 && !A->have_val32) {
        SGP_TRY(bsr_blocks(ctx, A));
        float *v32;
        int64_t len = sym_group_size(A->nnzb);
        SGP_TRY(ensure_t(ctx, A->val32, len + 8, &v32));
        if (A->nnzb > 0) k_round32<<<grid_for(len, 256), 256, 0, ctx->stream>>>(len, (const double *)A->val.p, v32);
        LAUNCH_CHECK(ctx);
        A->have_val32 = true;
    }
    if (A->have32) return SGP_OK;
    // the edge form: (w, u) and the diagonal blocks, rounded once
    float *e32, *d32;
    const int64_t elen = edge_group_size(A->nnzb - A->n), dlen = sym_group_size(A->n);
    SGP_TRY(ensure_t(ctx, A->ew32, elen + 8, &e32));
    SGP_TRY(ensure_t(ctx, A->dg32, dlen + 8, &d32));
    if (elen > 0) k_round32<<<grid_for(elen, 256), 256, 0, ctx->stream>>>(elen, (const double *)A->ew.p, e32);
    if (A->n > 0) k_round32<<<grid_for(dlen, 256), 256, 0, ctx->stream>>>(dlen, (const double *)A->dg.p, d32);
    LAUNCH_CHECK(ctx);
    A->have32 = true;
    return SGP_OK;
}
