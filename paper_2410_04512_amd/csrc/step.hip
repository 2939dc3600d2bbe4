// One whole batched step -- collide -> assemble_gamma -> build_tree ->
// factor_tree -> pcg_solve_batched -- recorded once and replayed as a single
// hipGraph.
//
// A recorded step replays for the inputs it was recorded with (positions,
// radii, forces and, with a warm start, the initial velocity, compared
// through a 64-bit device-side hash before the graph is launched): the
// graph's launch sizes, buffer sizes and iteration count are those of the
// recorded data, so other data would not just give other results but could
// index past buffers sized for the recorded contacts.  Changed inputs give
// SGP_ESTALE without launching the graph; the step is then recorded again.
//
// The step's launch sequence depends on its data only through the values the
// host reads back (the bounding box, the edge count, the rounds of Boruvka and
// of the elimination schedule, the schedule's step sizes, the CG's
// convergence polls) and the small host tables it uploads.  Recording runs the
// step eagerly and keeps every such value (StepPlan).  Capturing runs the same
// host code once more on a capturing stream: each readback returns its
// recorded value at once and enqueues a device-side comparison of the live
// value with it, each upload copies its recorded block from a device copy of
// the plan, and nothing allocates (the recorded run sized every buffer).  The
// graph therefore repeats exactly the recorded launches, and a replay whose
// data would have led the host elsewhere (another edge count, tree shape,
// schedule or iteration count) raises the flag: the replay reports
// SGP_ESTALE and the step must be recorded again.
#include "sgp_internal.h"

#include <cstring>

// The step owns its context (workspaces, counters, pinned block) and its
// graph, matrix, tree and preconditioner handles: the graph holds pointers to
// their device buffers, which nothing outside the step can grow or free.
struct sgp_step_ {
    sgp_ctx c = nullptr;
    sgp_graph g = nullptr;
    sgp_bsr A = nullptr;
    sgp_tree T = nullptr;
    sgp_prec M = nullptr;
    StepPlan plan;
    hipGraphExec_t exec = nullptr;
    std::vector<sgp_solve_info> info;   // the recorded run's results (equal to a valid replay's)
    std::vector<int64_t> off;
    // the inputs a replay reads, and their hash when recorded
    const double *pos = nullptr, *radius = nullptr, *F = nullptr, *v = nullptr;
    int64_t n = 0;
    bool use_x0 = false;
    uint64_t hash = 0;
    DevBuf hbuf;
    ~sgp_step_()
    {
        if (c) (void)hipStreamSynchronize(c->stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        release(plan.arena);
        release(plan.flag);
        release(hbuf);
        sgp_prec_free(M);
        sgp_tree_free(T);
        sgp_bsr_free(A);
        sgp_graph_free(g);
        sgp_destroy(c);
    }
};

__global__ void k_zero_flag(int32_t *flag) { *flag = 0; }
__global__ void k_zero_hash(unsigned long long *h) { *h = 0ull; }

// Hash of the step's inputs: sum over the 8-byte words w_k of each array a of
// mix(w_k + (k + 1) * c_a) with a per-array constant c_a (integer sums modulo
// 2^64 commute, so the atomic order does not matter).
__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__global__ void k_hash_words(const uint64_t *w, int64_t len, uint64_t salt, unsigned long long *out)
{
    uint64_t h = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += (int64_t)gridDim.x * blockDim.x)
        h += mix64(w[k] + (uint64_t)(k + 1) * salt);
    for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, (unsigned long long)h);
}

static int input_hash(sgp_ctx ctx, sgp_step S, uint64_t *h)
{
    unsigned long long *d;
    SGP_TRY(ensure_t(ctx, S->hbuf, 2, &d));
    k_zero_hash<<<1, 1, 0, ctx->stream>>>(d);
    const double *arr[4] = {S->pos, S->radius, S->F, S->use_x0 ? S->v : nullptr};
    const int64_t len[4] = {3 * S->n, S->n, 3 * S->n, 3 * S->n};
    for (int a = 0; a < 4; a++)
        if (arr[a] && len[a] > 0)
            k_hash_words<<<256, 256, 0, ctx->stream>>>((const uint64_t *)arr[a], len[a],
                                                       0x9e3779b97f4a7c15ull * (uint64_t)(2 * a + 1), d);
    LAUNCH_CHECK(ctx);
    return readback(ctx, h, d, sizeof *h);
}

struct StepArgs {
    int64_t n_inst;
    const int64_t *off;
    const double *pos, *radius;
    int32_t max_deg;
    double gpar, gperp, gmed;
    int32_t prec, schedule;
    const double *F;
    double *v;
    sgp_solve_opts opts;
    sgp_graph g;
    sgp_bsr A;
    sgp_tree T;
    sgp_prec M;
};

// the caller's launch-shape knobs and contact model, copied to the step's context
static void copy_settings(sgp_ctx to, const sgp_ctx_ *from)
{
    to->check_every = from->check_every;
    to->tail_max = from->tail_max;
    to->use_graph = 0;
    to->spmv_waves = from->spmv_waves;
    to->spmv_form = from->spmv_form;
    to->light_height = from->light_height;
    to->light_cap = from->light_cap;
    to->fuse_step0 = from->fuse_step0;
    to->mid_lds = from->mid_lds;
    to->tail_side = from->tail_side;
    to->prefetch = from->prefetch;
    to->small_solve = from->small_solve;
    to->contact_model = from->contact_model;
}

static int run_step(sgp_ctx ctx, const StepArgs &a, sgp_solve_info *info)
{
    SGP_TRY(sgp_collide_batched(ctx, a.n_inst, a.off, a.pos, a.radius, a.max_deg, a.g));
    SGP_TRY(sgp_assemble_gamma(ctx, a.g, a.gpar, a.gperp, a.gmed, a.A));
    sgp_prec M = nullptr;
    if (a.prec == SGP_STEP_TREE) {
        SGP_TRY(sgp_build_tree(ctx, a.g, a.T));
        SGP_TRY(sgp_factor_tree(ctx, a.g, a.T, a.gpar, a.gperp, a.gmed, a.schedule, a.M));
        M = a.M;
    } else if (a.prec == SGP_STEP_JACOBI) {
        SGP_TRY(sgp_make_jacobi(ctx, a.A, a.M));
        M = a.M;
    }
    return sgp_pcg_solve_batched(ctx, a.A, M, a.n_inst, a.off, a.F, a.v, &a.opts, info);
}

extern "C" int sgp_step_create(sgp_ctx ctx, sgp_step *out)
{
    if (!ctx || !out) return SGP_EINVAL;
    *out = nullptr;
    sgp_step S = new (std::nothrow) sgp_step_();
    if (!S) return set_err(ctx, SGP_ENOMEM, "step_create: out of host memory");
    int rc = sgp_create(&S->c, ctx->stream);
    if (rc == SGP_OK) rc = sgp_graph_create(S->c, &S->g);
    if (rc == SGP_OK) rc = sgp_bsr_create(S->c, &S->A);
    if (rc == SGP_OK) rc = sgp_tree_create(S->c, &S->T);
    if (rc == SGP_OK) rc = sgp_prec_create(S->c, &S->M);
    if (rc != SGP_OK) {
        delete S;
        return set_err(ctx, rc, "step_create: could not create the step's context and handles");
    }
    *out = S;
    return SGP_OK;
}

extern "C" void sgp_step_free(sgp_step S) { delete S; }

// errors of the step's own context are reported on the caller's
static int pass_err(sgp_ctx ctx, sgp_step S, int rc)
{
    if (rc != SGP_OK) set_err(ctx, rc, "%s", S->c->err.c_str());
    return rc;
}

static int record(sgp_ctx caller, sgp_step S, int64_t n_inst, const int64_t *offsets, const double *pos,
                  const double *radius, int32_t max_deg, double g_par, double g_perp, double g_med, int32_t prec,
                  int32_t schedule, const double *F, double *v, const sgp_solve_opts *opts)
{
    sgp_ctx ctx = S->c;
    ctx->stream = caller->stream;
    copy_settings(ctx, caller);
    if (S->exec) {
        (void)hipGraphExecDestroy(S->exec);
        S->exec = nullptr;
    }
    S->plan.bytes.clear();
    S->plan.off.clear();
    S->plan.len.clear();
    S->plan.kind.clear();
    S->plan.pos = 0;
    S->off.assign(offsets, offsets + n_inst + 1);
    S->pos = pos;
    S->radius = radius;
    S->F = F;
    S->v = v;
    S->n = offsets[n_inst];
    S->use_x0 = opts->use_x0 != 0;
    SGP_TRY(input_hash(ctx, S, &S->hash));
    StepArgs a = {n_inst, S->off.data(), pos, radius, max_deg, g_par, g_perp, g_med, prec, schedule, F, v, *opts,
                  S->g, S->A, S->T, S->M};
    // 1. the eager run, keeping every value the host reads and uploads
    ctx->plan = &S->plan;
    ctx->plan_mode = PLAN_RECORD;
    S->info.assign(n_inst, sgp_solve_info{});
    int rc = run_step(ctx, a, S->info.data());
    ctx->plan_mode = PLAN_OFF;
    if (rc == SGP_OK) {
        // 2. the plan on the device (compared against during replays)
        uint8_t *arena = nullptr;
        int32_t *flag = nullptr;
        rc = ensure_t(ctx, S->plan.arena, S->plan.bytes.size() + 8, &arena);
        if (rc == SGP_OK) rc = ensure_t(ctx, S->plan.flag, 4, &flag);
        if (rc == SGP_OK && !S->plan.bytes.empty()) {
            hipError_t e = hipMemcpyAsync(arena, S->plan.bytes.data(), S->plan.bytes.size(), hipMemcpyHostToDevice,
                                          ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) rc = set_err(ctx, SGP_EHIP, "step_record: plan upload: %s", hipGetErrorString(e));
        }
    }
    // 3. the same host code once more, captured
    if (rc == SGP_OK) {
        if (!ctx->cap_stream) {
            hipError_t e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) rc = set_err(ctx, SGP_EHIP, "step_record: stream: %s", hipGetErrorString(e));
        }
    }
    if (rc == SGP_OK) {
        hipStream_t saved = ctx->stream;
        ctx->stream = ctx->cap_stream;
        hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            ctx->stream = saved;
            rc = set_err(ctx, SGP_EHIP, "step_record: begin capture: %s", hipGetErrorString(e));
        } else {
            k_zero_flag<<<1, 1, 0, ctx->stream>>>((int32_t *)S->plan.flag.p);
            ctx->plan_mode = PLAN_CAPTURE;
            S->plan.pos = 0;
            std::vector<sgp_solve_info> scratch(n_inst);
            rc = run_step(ctx, a, scratch.data());
            ctx->plan_mode = PLAN_OFF;
            if (rc == SGP_OK && S->plan.pos != S->plan.len.size())
                rc = set_err(ctx, SGP_EINVAL, "step_record: the captured run read %zu of %zu recorded values",
                             S->plan.pos, S->plan.len.size());
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &graph);
            ctx->stream = saved;
            if (rc == SGP_OK && e2 != hipSuccess)
                rc = set_err(ctx, SGP_EHIP, "step_record: end capture: %s", hipGetErrorString(e2));
            if (rc == SGP_OK) {
                e = hipGraphInstantiate(&S->exec, graph, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    S->exec = nullptr;
                    rc = set_err(ctx, SGP_EHIP, "step_record: instantiate: %s", hipGetErrorString(e));
                }
            }
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
        }
    }
    ctx->plan = nullptr;
    return rc;
}

extern "C" int sgp_step_record_batched(sgp_ctx ctx, sgp_step S, int64_t n_inst, const int64_t *offsets,
                                       const double *pos, const double *radius, int32_t max_deg, double g_par,
                                       double g_perp, double g_med, int32_t prec, int32_t schedule, const double *F,
                                       double *v, const sgp_solve_opts *opts, sgp_solve_info *info)
{
    if (!ctx || !S || !offsets || n_inst <= 0 || !opts || !info)
        return set_err(ctx, SGP_EINVAL, "step_record: bad arguments");
    if (prec != SGP_STEP_NONE && prec != SGP_STEP_JACOBI && prec != SGP_STEP_TREE)
        return set_err(ctx, SGP_EINVAL, "step_record: unknown preconditioner %d", prec);
    const int rc = pass_err(ctx, S, record(ctx, S, n_inst, offsets, pos, radius, max_deg, g_par, g_perp, g_med, prec,
                                           schedule, F, v, opts));
    if (rc == SGP_OK) memcpy(info, S->info.data(), n_inst * sizeof(sgp_solve_info));
    return rc;
}

extern "C" int sgp_step_replay(sgp_ctx ctx, sgp_step S, sgp_solve_info *info)
{
    if (!ctx || !S || !info) return set_err(ctx, SGP_EINVAL, "step_replay: bad arguments");
    if (!S->exec) return set_err(ctx, SGP_EINVAL, "step_replay: nothing recorded");
    S->c->stream = ctx->stream;
    uint64_t h = 0;
    SGP_TRY(pass_err(ctx, S, input_hash(S->c, S, &h)));
    if (h != S->hash)
        return set_err(ctx, SGP_ESTALE, "step_replay: the inputs differ from the recorded ones; record again");
    HIP_TRY(ctx, hipGraphLaunch(S->exec, ctx->stream));
    int32_t stale = 0;
    SGP_TRY(readback(ctx, &stale, S->plan.flag.p, sizeof stale));
    memcpy(info, S->info.data(), S->info.size() * sizeof(sgp_solve_info));
    if (stale)
        return set_err(ctx, SGP_ESTALE, "step_replay: the data no longer has the recorded structure; record again");
    return SGP_OK;
}

extern "C" int sgp_step_size(sgp_step S, int64_t *values, int64_t *bytes)
{
    if (!S) return SGP_EINVAL;
    if (values) *values = (int64_t)S->plan.len.size();
    if (bytes) *bytes = (int64_t)S->plan.bytes.size();
    return SGP_OK;
}
