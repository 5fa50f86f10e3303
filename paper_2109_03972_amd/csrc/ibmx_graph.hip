// Batching form of the forcing loop: the whole call (geometry, binning, the
// n_iter passes, f_tot, particle sums, residuals) captured once into a HIP
// graph and replayed with one launch per call, and the tile-shape autotuner.
#include <float.h>
#include <string.h>

#include "ibmx_internal.hpp"

void ibmx_plan_drop_graph(ibmx_plan p)
{
    if (p && p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
    }
}

namespace {

ibmx_status capture_forcing(ibmx_plan p, const void *const key[10])
{
    if (!p->cap_stream)
        IBMX_HIP_CHECK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    const hipStream_t user = p->stream;
    const int prof = p->prof;
    p->stream = p->cap_stream;
    p->prof = 0;
    hipGraph_t graph = nullptr;
    ibmx_status st = IBMX_EDEVICE;
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        st = ibmx_forcing(p, (void *)key[0], (void *)key[1], (const double *)key[2],
                          (const double *)key[3], (const double *)key[4], (const uint8_t *)key[5],
                          (double *)key[6], (double *)key[7], (double *)key[8], (void *)key[9]);
        const hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
        if (st == IBMX_OK && (e != hipSuccess || !graph))
            st = IBMX_EDEVICE;
    }
    p->stream = user;
    p->prof = prof;
    if (st != IBMX_OK) {
        if (graph)
            (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return st;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
        return IBMX_EDEVICE;
    ibmx_plan_drop_graph(p);
    p->gexec = exec;
    memcpy(p->gkey, key, sizeof(p->gkey));
    return IBMX_OK;
}

}  // namespace

extern "C" ibmx_status ibmx_forcing_graph(ibmx_plan p, void *u, void *f_tot, const double *xp,
                                          const double *up, const double *wp,
                                          const uint8_t *marker_active, double *S_out,
                                          double *T_out, double *resid_out, void *U_debug)
{
    if (!p)
        return IBMX_EINVAL;
    const void *key[10] = {u, f_tot, xp, up, wp, marker_active, S_out, T_out, resid_out, U_debug};
    if (!p->gexec || memcmp(key, p->gkey, sizeof(key)) != 0) {
        const ibmx_status st = capture_forcing(p, key);
        if (st != IBMX_OK)
            return st;
    }
    ProfScope ps(p, IBMX_K_GRAPH);
    IBMX_HIP_CHECK(hipGraphLaunch(p->gexec, p->stream));
    return IBMX_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
namespace {

// tile shapes tried, the one that wins on dense beds in both precisions
// first (a later one must beat the best so far by 2%);
// ibmx_plan_alloc_tiles rejects the ones whose LDS footprint does not fit
// the precision
const int kTileCandidates[][3] = {
    {32, 8, 8},  {16, 16, 8}, {16, 16, 16}, {32, 16, 8}, {32, 16, 4}, {32, 32, 4},
    {16, 16, 4}, {16, 8, 8},  {8, 16, 8},   {16, 8, 16}, {8, 8, 8},   {32, 8, 16},
};

struct TuneScratch {
    void *u = nullptr, *f = nullptr;
    double *S = nullptr, *T = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneScratch()
    {
        void *ptrs[] = {u, f, S, T};
        for (void *q : ptrs)
            if (q)
                (void)hipFree(q);
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
    }
};

// Read and clear the plan's deferred error (the stream is synchronised).
int take_error(ibmx_plan p)
{
    int err = 0;
    if (hipStreamSynchronize(p->stream) != hipSuccess ||
        hipMemcpy(&err, p->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return (int)IBMX_EDEVICE;
    if (err != 0)
        (void)hipMemset(p->d_err, 0, sizeof(int));
    return err;
}

}  // namespace

extern "C" ibmx_status ibmx_tune(ibmx_plan p, void *u, void *f_tot, const double *xp,
                                 const double *up, const double *wp, const uint8_t *marker_active)
{
    if (!p || !u || !f_tot)
        return IBMX_EINVAL;
    if (p->nm > 0 && (!p->body || !p->dV))
        return IBMX_ESTATE;
    const size_t Ts = p->prec == IBMX_F64 ? sizeof(double) : sizeof(float);
    const size_t gbytes = Ts * 3 * (size_t)p->g.nodes;
    const size_t pbytes = sizeof(double) * 3 * (size_t)(p->np > 0 ? p->np : 1);
    TuneScratch sc;
    IBMX_HIP_CHECK(hipMalloc(&sc.u, gbytes));
    IBMX_HIP_CHECK(hipMalloc(&sc.f, gbytes));
    IBMX_HIP_CHECK(hipMalloc((void **)&sc.S, pbytes));
    IBMX_HIP_CHECK(hipMalloc((void **)&sc.T, pbytes));
    IBMX_HIP_CHECK(hipEventCreate(&sc.e0));
    IBMX_HIP_CHECK(hipEventCreate(&sc.e1));
    hipStream_t s = p->stream;
    IBMX_HIP_CHECK(hipMemcpyAsync(sc.u, u, gbytes, hipMemcpyDeviceToDevice, s));
    IBMX_HIP_CHECK(hipMemcpyAsync(sc.f, f_tot, gbytes, hipMemcpyDeviceToDevice, s));
    const int pending = take_error(p);   // an earlier call's error, handed back at the end
    if (pending == (int)IBMX_EDEVICE)
        return IBMX_EDEVICE;
    const int prof = p->prof;
    p->prof = 0;
    const int orig[3] = {p->tc.B[0], p->tc.B[1], p->tc.B[2]};
    const int orig_block = p->block, orig_persist = p->persist;
    int best[3] = {orig[0], orig[1], orig[2]};
    int best_block = orig_block, best_persist = orig_persist;
    float best_ms = FLT_MAX;
    ibmx_status st = IBMX_OK;
    int last_err = 0;
    // time the current launch form: the best of three calls after a warm-up
    // (false when the call raised a deferred error)
    auto trial = [&](float *t_out) -> bool {
        float t_min = FLT_MAX;
        bool ok = true;
        for (int rep = 0; rep < 4 && ok; ++rep) {
            (void)hipEventRecord(sc.e0, s);
            st = ibmx_forcing(p, u, f_tot, xp, up, wp, marker_active, sc.S, sc.T, nullptr,
                              nullptr);
            (void)hipEventRecord(sc.e1, s);
            if (st != IBMX_OK)
                return false;
            if (hipMemcpyAsync(u, sc.u, gbytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                hipMemcpyAsync(f_tot, sc.f, gbytes, hipMemcpyDeviceToDevice, s) != hipSuccess) {
                st = IBMX_EDEVICE;
                return false;
            }
            const int err = take_error(p);
            if (err == (int)IBMX_EDEVICE) {
                st = IBMX_EDEVICE;
                return false;
            }
            ok = err == 0;
            if (!ok)
                last_err = err;
            float ms = 0.f;
            if (ok && rep > 0 && hipEventElapsedTime(&ms, sc.e0, sc.e1) == hipSuccess)
                t_min = ms < t_min ? ms : t_min;
        }
        *t_out = t_min;
        return ok;
    };
    // tile shapes at 256 threads per workgroup, one workgroup per tile; a
    // later candidate must win by 2% (timing noise keeps the earlier shapes)
    p->block = 256;
    p->persist = 0;
    for (const auto &cand : kTileCandidates) {
        if (ibmx_plan_alloc_tiles(p, cand[0], cand[1], cand[2]) != IBMX_OK)
            continue;
        float t = FLT_MAX;
        const bool ok = trial(&t);
        if (st != IBMX_OK)
            break;
        if (ok && t < 0.98f * best_ms) {
            best_ms = t;
            for (int a = 0; a < 3; ++a)
                best[a] = cand[a];
            best_block = 256;
            best_persist = 0;
        }
    }
    // the launch form for the chosen shape: workgroup size and persistence
    if (st == IBMX_OK && best_ms < FLT_MAX &&
        ibmx_plan_alloc_tiles(p, best[0], best[1], best[2]) == IBMX_OK) {
        const int forms[][2] = {{256, 1}, {128, 0}, {128, 1}, {64, 0}, {64, 1}};
        for (const auto &fm : forms) {
            p->block = fm[0];
            p->persist = fm[1];
            float t = FLT_MAX;
            const bool ok = trial(&t);
            if (st != IBMX_OK)
                break;
            if (ok && t < 0.98f * best_ms) {
                best_ms = t;
                best_block = fm[0];
                best_persist = fm[1];
            }
        }
    }
    p->prof = prof;
    // leave u and f_tot as they came in, whatever happened above
    (void)hipMemcpyAsync(u, sc.u, gbytes, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(f_tot, sc.f, gbytes, hipMemcpyDeviceToDevice, s);
    if (st == IBMX_OK && best_ms == FLT_MAX && last_err != 0)
        st = (ibmx_status)last_err;   // no candidate ran cleanly
    if (best_ms == FLT_MAX) {
        best_block = orig_block;
        best_persist = orig_persist;
    }
    ibmx_status st2 = ibmx_plan_alloc_tiles(p, best[0], best[1], best[2]);
    if (st2 != IBMX_OK)
        st2 = ibmx_plan_alloc_tiles(p, orig[0], orig[1], orig[2]);
    (void)ibmx_plan_set_launch(p, best_block, best_persist);
    if (pending != 0)
        (void)hipMemcpy(p->d_err, &pending, sizeof(int), hipMemcpyHostToDevice);
    if (hipStreamSynchronize(s) != hipSuccess)
        return IBMX_EDEVICE;
    return st != IBMX_OK ? st : st2;
}
