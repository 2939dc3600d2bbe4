// Context and handle lifetime of the C ABI (include/sgp.h).
#include "sgp_internal.h"

#include <new>

extern "C" int sgp_create(sgp_ctx *out, void *hip_stream)
{
    if (!out) return SGP_EINVAL;
    *out = nullptr;
    sgp_ctx c = new (std::nothrow) sgp_ctx_();
    if (!c) return SGP_ENOMEM;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMalloc((void **)&c->tickets, 64 * sizeof(unsigned));
    if (e == hipSuccess) e = hipMemsetAsync(c->tickets, 0, 64 * sizeof(unsigned), c->stream);
    if (e == hipSuccess) e = hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault);
    for (int k = 0; k < 12 && e == hipSuccess; k++) e = hipEventCreate(&c->ev[k]);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        sgp_destroy(c);
        return SGP_EHIP;
    }
    const int s = noalloc_scratch_init(c);
    if (s != SGP_OK) {
        sgp_destroy(c);
        return s;
    }
    c->n_tickets = 64;
    *out = c;
    return SGP_OK;
}

extern "C" void sgp_destroy(sgp_ctx c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipEvent_t e : c->kev) (void)hipEventDestroy(e);
    for (auto &b : c->ws) release(b);
    if (c->tickets) (void)hipFree(c->tickets);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->poll_ev) (void)hipEventDestroy(c->poll_ev);
    for (int k = 0; k < 12; k++)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    delete c;
}

extern "C" const char *sgp_last_error(sgp_ctx c) { return c ? c->err.c_str() : "null context"; }

extern "C" int sgp_set_stream(sgp_ctx c, void *hip_stream)
{
    if (!c) return SGP_EINVAL;
    c->stream = (hipStream_t)hip_stream;
    return SGP_OK;
}

extern "C" int sgp_phase_times(sgp_ctx c, double *ms5)
{
    if (!c || !ms5) return SGP_EINVAL;
    for (int k = 0; k < 5; k++) {
        if (c->phase_pending[k]) {
            float ms = 0.f;
            if (hipEventSynchronize(c->ev[2 * k + 1]) == hipSuccess &&
                hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]) == hipSuccess)
                c->phase_ms[k] = ms;
            c->phase_pending[k] = false;
        }
        ms5[k] = c->phase_ms[k];
    }
    return SGP_OK;
}

#define HANDLE_FUNCS(T, name)                                      \
    extern "C" int sgp_##name##_create(sgp_ctx c, T *out)          \
    {                                                              \
        if (!c || !out) return set_err(c, SGP_EINVAL, #name "_create: null"); \
        *out = new (std::nothrow) T##_();                          \
        return *out ? SGP_OK : set_err(c, SGP_ENOMEM, #name "_create: out of memory"); \
    }

HANDLE_FUNCS(sgp_graph, graph)
HANDLE_FUNCS(sgp_bsr, bsr)
HANDLE_FUNCS(sgp_tree, tree)
HANDLE_FUNCS(sgp_prec, prec)

extern "C" void sgp_graph_free(sgp_graph g)
{
    if (!g) return;
    (void)hipDeviceSynchronize();
    release(g->rowptr); release(g->col); release(g->ent_edge); release(g->ei);
    release(g->ej); release(g->wu); release(g->inst_off); release(g->inst_of); release(g->w);
    release(g->perm); release(g->inv);
    delete g;
}

extern "C" void sgp_bsr_free(sgp_bsr A)
{
    if (!A) return;
    (void)hipDeviceSynchronize();
    release(A->rowptr); release(A->bcol); release(A->val); release(A->val32); release(A->diagpos);
    release(A->wrow); release(A->perm); release(A->inv);
    release(A->ecol); release(A->ew); release(A->dg); release(A->ew32); release(A->dg32); release(A->ewrow);
    delete A;
}

extern "C" void sgp_tree_free(sgp_tree T)
{
    if (!T) return;
    (void)hipDeviceSynchronize();
    release(T->tree_edge); release(T->parent); release(T->pedge); release(T->depth); release(T->comp);
    release(T->tptr); release(T->tadj); release(T->tadje);
    delete T;
}

extern "C" void sgp_prec_free(sgp_prec M)
{
    if (!M) return;
    (void)hipDeviceSynchronize();
    release(M->elim); release(M->pos); release(M->up); release(M->in_ptr); release(M->in_src);
    release(M->F); release(M->Dinv); release(M->y); release(M->F32); release(M->Dinv32); release(M->y32);
    release(M->tout); release(M->cs); release(M->cs32); release(M->step_ptr);
    release(M->elim_int); release(M->perm); release(M->inv); release(M->tail_iptr); release(M->tail_tslot);
    release(M->tail_b); release(M->light_ptr); release(M->mid_ptr); release(M->wu0); release(M->wu032);
    release(M->jdinv);
    release(M->aug_piece); release(M->aug_list); release(M->aug_tptr); release(M->aug_tadj); release(M->aug_twu);
    release(M->aug_ptr); release(M->aug_adj); release(M->aug_wu); release(M->small_ell); release(M->mid_tab);
    delete M;
}

// ---------------------------------------------------------------- kernel timing

int ktimer_begin(sgp_ctx c, int32_t iter)
{
    if (!c->ktiming || c->plan_mode != PLAN_OFF) return SGP_OK;
    if ((int)c->kev_iter.size() <= c->kev_used / 2) c->kev_iter.resize(c->kev_used / 2 + 64);
    c->kev_iter[c->kev_used / 2] = iter;
    if (c->kev_used + 2 > (int)c->kev.size()) {
        for (int k = 0; k < 64; k++) {
            hipEvent_t e;
            HIP_TRY(c, hipEventCreate(&e));
            c->kev.push_back(e);
        }
    }
    // the product launched next takes the pair as its own start and stop
    // (hipExtLaunchKernel): the events time the kernel itself and add no
    // packets of their own to the stream
    c->kt_start = c->kev[c->kev_used];
    c->kt_stop = c->kev[c->kev_used + 1];
    c->kt_used = false;
    return SGP_OK;
}

int ktimer_end(sgp_ctx c)
{
    if (!c->ktiming) return SGP_OK;
    if (c->kt_used) c->kev_used += 2;   // else nothing was launched (an empty product)
    c->kt_start = c->kt_stop = nullptr;
    c->kt_used = false;
    return SGP_OK;
}

int ktimer_flush(sgp_ctx c, int32_t iters_done)
{
    if (!c->ktiming || c->kev_used == 0) return SGP_OK;
    HIP_TRY(c, hipEventSynchronize(c->kev[c->kev_used - 1]));
    for (int k = 0; k < c->kev_used; k += 2) {
        if (c->kev_iter[k / 2] >= iters_done) continue;   // issued past convergence: a no-op launch
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->kev[k], c->kev[k + 1]));
        c->ktime_ms += ms;
        c->klaunches++;
    }
    c->kev_used = 0;
    return SGP_OK;
}

extern "C" int sgp_kernel_timing(sgp_ctx c, int32_t enable)
{
    if (!c) return SGP_EINVAL;
    c->ktiming = enable ? 1 : 0;
    c->ktime_ms = 0.0;
    c->klaunches = 0;
    c->kev_used = 0;
    return SGP_OK;
}

extern "C" int sgp_kernel_stats(sgp_ctx c, double *total_ms, int64_t *launches)
{
    if (!c) return SGP_EINVAL;
    SGP_TRY(ktimer_flush(c, INT32_MAX));
    if (total_ms) *total_ms = c->ktime_ms;
    if (launches) *launches = c->klaunches;
    return SGP_OK;
}
