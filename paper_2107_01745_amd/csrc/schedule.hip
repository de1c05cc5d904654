// Sweep schedules of a handle: the knobs of the work lists, a timing-driven
// autotuner over them, and the dual-gradient sweep recorded as a HIP graph.
//
// Knobs (all results are independent of the first two; the third reorders
// the per-node sums above s*):
//   group_min   smallest lane group that walks one chain below s*;
//   chain_order costliest wavefront items first, or instance order;
//   trunk_cap   cap on the wavefronts that share one node above s*;
//   trunk_fused the launch form of the stages above s* (per stage, one
//               backward launch, lane groups, or the first stages fused);
//   panel_min   on a shared handle, the fewest unfinished copies that are
//               still swept as panels on the matrix cores (fewer: the
//               lane-group sweeps, which skip finished copies one by one).
// The autotuner times homogeneous sweeps (Algorithm 4) on zero duals, which
// stream exactly the data of a dual-gradient sweep, for each candidate of
// one knob at a time (coordinate descent), and keeps the fastest schedule.
// On a shared handle it tunes the lane-group route first, then times one
// panel sweep of all copies against it and sets panel_min where the two
// costs meet (the lane-group cost taken as proportional to the copies swept).
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

struct sweep_graph {
    tree_factors *f;
    long long epoch;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace stotree {

namespace {

constexpr int kPanelMinMax = 1 << 24;

bool valid_knobs(const int32_t *k)
{
    const bool g = k[0] == 8 || k[0] == 16 || k[0] == 32 || k[0] == 64;
    const bool o = k[1] == 0 || k[1] == 1;
    const bool t = k[2] == 1 || k[2] == 2 || k[2] == 4 || k[2] == 8 || k[2] == 16;
    const bool m = k[3] >= 0 && k[3] <= 4;
    const bool p = k[4] >= 0 && k[4] <= kPanelMinMax;
    return g && o && t && m && p;
}

// Lane-group width of every instance under group_min g (equal vectors give
// identical chain work lists).
std::vector<int> groups_of(const tree_factors *f, int g)
{
    std::vector<int> v;
    for (const InstDesc &I : f->inst) v.push_back(I.sstar < I.N ? chain_group(I.ldM, g) : 0);
    return v;
}

}  // namespace

int set_schedule(tree_factors *f, const int32_t *knobs)
{
    if (!valid_knobs(knobs)) {
        set_error("sweep_schedule: knobs must be group in {8,16,32,64}, order in {0,1}, cap in {1,2,4,8,16}, "
                  "trunk mode in {0,...,4}, panel minimum in [0, 2^24]");
        return STOTREE_ERR_ARG;
    }
    // the old work lists may still be read by queued sweeps
    STOTREE_HIP(hipDeviceSynchronize());
    f->group_min = knobs[0];
    f->chain_order = knobs[1];
    f->trunk_cap = knobs[2];
    f->trunk_fused = knobs[3];
    f->panel_min = knobs[4];
    ++f->schedule_epoch;
    return build_schedule(f);
}

int autotune(tree_factors *f, int nrhs, int reps, int32_t *knobs_out, double *ms_out, hipStream_t st)
{
    int rc = ensure_sweep_ws(f, nrhs);
    if (rc) return rc;
    double *y = nullptr, *x = nullptr, *u = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Cleanup {
        double *&y, *&x, *&u;
        hipEvent_t &e0, &e1;
        ~Cleanup()
        {
            for (double *p : {y, x, u})
                if (p) (void)hipFree(p);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } cleanup{y, x, u, e0, e1};
    STOTREE_HIP(hipMalloc(&y, sizeof(double) * (size_t)nrhs * f->mxu_tot));
    STOTREE_HIP(hipMalloc(&x, sizeof(double) * (size_t)nrhs * f->x_tot));
    STOTREE_HIP(hipMalloc(&u, sizeof(double) * (size_t)nrhs * f->u_tot));
    STOTREE_HIP(hipMemsetAsync(y, 0, sizeof(double) * (size_t)nrhs * f->mxu_tot, st));
    STOTREE_HIP(hipEventCreate(&e0));
    STOTREE_HIP(hipEventCreate(&e1));
    const bool timing_was = timing_on();
    timing_enable(0);
    auto measure = [&](const int32_t *k, double *ms) -> int {
        int r = set_schedule(f, k);
        if (r) return r;
        if ((r = enqueue_dual_grad(f, nullptr, y, 1, nrhs, x, u, st))) return r;
        STOTREE_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < reps; ++i)
            if ((r = enqueue_dual_grad(f, nullptr, y, 1, nrhs, x, u, st))) return r;
        STOTREE_HIP(hipEventRecord(e1, st));
        STOTREE_HIP(hipEventSynchronize(e1));
        float t = 0.0f;
        STOTREE_HIP(hipEventElapsedTime(&t, e0, e1));
        *ms = t / reps;
        return STOTREE_OK;
    };
    int32_t best[kKnobs] = {f->group_min, f->chain_order, f->trunk_cap, f->trunk_fused, f->panel_min};
    const bool shared = shared_panels(f);
    if (shared) best[4] = kPanelMinMax;    // lane-group route while its knobs are tuned
    double best_ms = 0.0;
    rc = measure(best, &best_ms);
    const std::vector<std::vector<int>> values = {{8, 16, 32, 64}, {1, 0}, {16, 8, 4, 2}, {0, 2, 1, 3, 4}};
    for (int knob = 0; knob < kKnobs - 1 && !rc; ++knob) {
        const int32_t start = best[knob];
        for (int v : values[knob]) {
            if (rc) break;
            if (v == start) continue;
            if (knob == 0 && groups_of(f, v) == groups_of(f, best[0])) continue;
            int32_t cand[kKnobs] = {best[0], best[1], best[2], best[3], best[4]};
            cand[knob] = v;
            double ms = 0.0;
            rc = measure(cand, &ms);
            if (!rc && ms < best_ms) {
                best_ms = ms;
                best[knob] = v;
            }
        }
    }
    if (shared && !rc) {
        int32_t cand[kKnobs] = {best[0], best[1], best[2], best[3], 0};
        double ms = 0.0;
        rc = measure(cand, &ms);
        if (!rc) {
            // panels cost ms while any copy is unfinished; the lane groups
            // best_ms * active / ninst
            const double meet = ms < best_ms ? std::ceil(f->ninst * ms / best_ms) : f->ninst + 1.0;
            best[4] = (int32_t)(meet < 1.0 ? 1.0 : meet);
            if (ms < best_ms) best_ms = ms;
        }
    }
    timing_enable(timing_was ? 1 : 0);
    if (rc) return rc;
    if ((rc = set_schedule(f, best))) return rc;
    if (knobs_out) for (int k = 0; k < kKnobs; ++k) knobs_out[k] = best[k];
    if (ms_out) *ms_out = best_ms;
    return STOTREE_OK;
}

int graph_create(tree_factors *f, const double *x0, const double *y, int homogeneous, int nrhs, double *x,
                 double *u, sweep_graph **out)
{
    // workspace first: nothing may be allocated while the stream records
    int rc = ensure_sweep_ws(f, nrhs >= 2 ? 2 : 1);
    if (rc) return rc;
    hipStream_t cs = nullptr;
    STOTREE_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const bool timing_was = timing_on();
    timing_enable(0);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = enqueue_dual_grad(f, x0, y, homogeneous, nrhs, x, u, cs);
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (!rc && e2 != hipSuccess) e = e2;
    }
    timing_enable(timing_was ? 1 : 0);
    (void)hipStreamDestroy(cs);
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (!rc) {
            set_error(std::string("sweep_graph_create: capture failed: ") + hipGetErrorString(e));
            rc = STOTREE_ERR_DEVICE;
        }
        return rc;
    }
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_error(std::string("sweep_graph_create: instantiate failed: ") + hipGetErrorString(e));
        return STOTREE_ERR_DEVICE;
    }
    *out = new sweep_graph{f, f->schedule_epoch, g, ge};
    return STOTREE_OK;
}

int graph_launch(sweep_graph *g, hipStream_t st)
{
    if (g->epoch != g->f->schedule_epoch) {
        set_error("sweep_graph_launch: the handle's schedule changed after the graph was recorded");
        return STOTREE_ERR_ARG;
    }
    STOTREE_HIP(hipGraphLaunch(g->exec, st));
    return STOTREE_OK;
}

void graph_free(sweep_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // namespace stotree
