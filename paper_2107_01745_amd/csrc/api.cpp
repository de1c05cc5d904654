// C ABI of the stotree library (declared in include/stotree.h).
#include <chrono>
#include <cstring>
#include <string>

#include "internal.h"

namespace stotree {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

}  // namespace stotree

using namespace stotree;

extern "C" {

const char *stotree_last_error(void) { return g_last_error.c_str(); }

int tree_factor(const tree_desc *tree, const problem_data *data, int precondition, void *hip_stream,
                tree_factors **out)
{
    set_error("");
    return factor_forest(1, tree, data, precondition, (hipStream_t)hip_stream, out);
}

int tree_factor_batch(int count, const tree_desc *trees, const problem_data *data, int precondition,
                      void *hip_stream, tree_factors **out)
{
    set_error("");
    return factor_forest(count, trees, data, precondition, (hipStream_t)hip_stream, out);
}

int tree_factor_shared(const tree_desc *tree, const problem_data *data, int precondition, int count,
                       const double *c, void *hip_stream, tree_factors **out)
{
    set_error("");
    if (count < 1) {
        if (out) *out = nullptr;
        set_error("tree_factor_shared: count < 1");
        return STOTREE_ERR_ARG;
    }
    int rc = factor_forest(1, tree, data, precondition, (hipStream_t)hip_stream, out, c != nullptr);
    if (rc) return rc;
    if ((rc = replicate_instances(*out, count, c, (hipStream_t)hip_stream))) {
        free_tree(*out);
        *out = nullptr;
    }
    return rc;
}

void tree_factors_free(tree_factors *f) { free_tree(f); }

int tree_dims(const tree_factors *f, int64_t *out)
{
    if (!f || !out) { set_error("tree_dims: NULL argument"); return STOTREE_ERR_ARG; }
    out[0] = f->ninst; out[1] = f->precondition; out[2] = f->m_tot; out[3] = f->n_tot;
    out[4] = f->x_tot; out[5] = f->u_tot; out[6] = f->nx_tot; out[7] = f->V_tot;
    out[8] = (int64_t)(f->bytes + f->sws.bytes); out[9] = f->max_width;
    return STOTREE_OK;
}

int tree_instance_dims(const tree_factors *f, int b, int64_t *out)
{
    if (!f || !out || b < 0 || b >= f->ninst) {
        set_error("tree_instance_dims: NULL argument or instance out of range");
        return STOTREE_ERR_ARG;
    }
    const InstDesc &I = f->inst[b];
    out[0] = I.nx; out[1] = I.nu; out[2] = I.N; out[3] = I.V; out[4] = I.Vnl; out[5] = I.m;
    out[6] = (int64_t)I.Vnl * I.nu + (int64_t)(I.V - 1) * I.nx; out[7] = I.sstar;
    out[8] = I.y; out[9] = I.x; out[10] = I.u; out[11] = I.x0;
    return STOTREE_OK;
}

int dual_grad(const tree_factors *fc, const double *x0, const double *y, int homogeneous, int nrhs,
              double *x, double *u, void *hip_stream)
{
    if (!fc || !y || !x || !u || nrhs < 1 || (!homogeneous && !x0)) {
        set_error("dual_grad: NULL pointer or nrhs < 1");
        return STOTREE_ERR_ARG;
    }
    tree_factors *f = const_cast<tree_factors *>(fc);
    if (f->cmap) return dual_grad_mapped(f, x0, y, homogeneous, nrhs, x, u, (hipStream_t)hip_stream);
    return enqueue_dual_grad(f, x0, y, homogeneous, nrhs, x, u, (hipStream_t)hip_stream);
}

int dual_grad_noalloc(const tree_factors *fc, const double *x0, const double *y, int homogeneous, int nrhs,
                      double *x, double *u, void *hip_stream)
{
    if (!fc || !y || !x || !u || nrhs < 1 || (!homogeneous && !x0)) {
        set_error("dual_grad_noalloc: NULL pointer or nrhs < 1");
        return STOTREE_ERR_ARG;
    }
    return dual_grad_noalloc_impl(fc, x0, y, homogeneous, nrhs, x, u, (hipStream_t)hip_stream);
}

int sweep_schedule(tree_factors *f, const int32_t *knobs)
{
    if (!f || !knobs) { set_error("sweep_schedule: NULL argument"); return STOTREE_ERR_ARG; }
    return set_schedule(f, knobs);
}

int sweep_schedule_get(const tree_factors *f, int32_t *knobs)
{
    if (!f || !knobs) { set_error("sweep_schedule_get: NULL argument"); return STOTREE_ERR_ARG; }
    knobs[0] = f->group_min; knobs[1] = f->chain_order; knobs[2] = f->trunk_cap; knobs[3] = f->trunk_fused;
    knobs[4] = f->panel_min;
    return STOTREE_OK;
}

int sweep_autotune(tree_factors *f, int nrhs, int reps, int32_t *knobs_out, double *ms_out, void *hip_stream)
{
    if (!f || nrhs < 1 || nrhs > 2 || reps < 1) { set_error("sweep_autotune: bad argument"); return STOTREE_ERR_ARG; }
    return autotune(f, nrhs, reps, knobs_out, ms_out, (hipStream_t)hip_stream);
}

int sweep_graph_create(const tree_factors *f, const double *x0, const double *y, int homogeneous, int nrhs,
                       double *x, double *u, sweep_graph **out)
{
    if (!out) { set_error("sweep_graph_create: out is NULL"); return STOTREE_ERR_ARG; }
    *out = nullptr;
    if (!f || !y || !x || !u || nrhs < 1 || nrhs > 2 || (!homogeneous && !x0)) {
        set_error("sweep_graph_create: NULL pointer or nrhs not in {1, 2}");
        return STOTREE_ERR_ARG;
    }
    if (f->cmap) {
        set_error("sweep_graph_create: handles with a constraint map are not supported");
        return STOTREE_ERR_ARG;
    }
    return graph_create(const_cast<tree_factors *>(f), x0, y, homogeneous, nrhs, x, u, out);
}

int sweep_graph_launch(sweep_graph *g, void *hip_stream)
{
    if (!g) { set_error("sweep_graph_launch: NULL graph"); return STOTREE_ERR_ARG; }
    return graph_launch(g, (hipStream_t)hip_stream);
}

void sweep_graph_free(sweep_graph *g) { graph_free(g); }

int dual_lipschitz(const tree_factors *f, int iters, double *L_out, void *hip_stream)
{
    if (!f || !L_out || iters < 1) { set_error("dual_lipschitz: bad argument"); return STOTREE_ERR_ARG; }
    return lipschitz(f, iters, L_out, (hipStream_t)hip_stream);
}

static int run_solver(const tree_factors *f, const double *x0, const solver_opts *opts, double *y,
                      double *x, double *u, solver_info *info, void *hip_stream, int method)
{
    if (!f || !x0 || !y || !x || !u) { set_error("solve: NULL pointer"); return STOTREE_ERR_ARG; }
    const auto t0 = std::chrono::steady_clock::now();
    solver_info local{};
    const int rc = solve(f, x0, opts, y, x, u, &local, (hipStream_t)hip_stream, method);
    local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = local;
    return rc;
}

int minfbe_solve(const tree_factors *f, const double *x0, const solver_opts *opts, double *y_inout,
                 double *x, double *u, solver_info *info, void *hip_stream)
{
    return run_solver(f, x0, opts, y_inout, x, u, info, hip_stream, 0);
}

int nama_solve(const tree_factors *f, const double *x0, const solver_opts *opts, double *y_inout,
               double *x, double *u, solver_info *info, void *hip_stream)
{
    return run_solver(f, x0, opts, y_inout, x, u, info, hip_stream, 1);
}

int gpad_solve(const tree_factors *f, const double *x0, const solver_opts *opts, double *y_inout, double *x,
               double *u, solver_info *info, void *hip_stream)
{
    return run_solver(f, x0, opts, y_inout, x, u, info, hip_stream, 2);
}

int solve_info_batch(const tree_factors *f, solver_info *infos)
{
    if (!f || !infos) { set_error("solve_info_batch: NULL argument"); return STOTREE_ERR_ARG; }
    for (int b = 0; b < f->ninst; ++b) infos[b] = f->last_info[b];
    return STOTREE_OK;
}

int64_t warm_mlp_params(int din, int dh, int dout)
{
    if (din < 1 || dh < 1 || dout < 1) return -1;
    return mlp_param_count(din, dh, dout);
}

int64_t warm_mlp_work_len(int rows, int din, int dh, int dout)
{
    if (rows < 1 || din < 1 || dh < 1 || dout < 1) return -1;
    return mlp_work_len(rows, din, dh, dout);
}

int warm_mlp_forward(int rows, int din, int dh, int dout, const float *params, const float *X, float *H, float *Y,
                     void *hip_stream)
{
    if (rows < 1 || din < 1 || dh < 1 || dout < 1 || !params || !X || !H || !Y) {
        set_error("warm_mlp_forward: bad argument");
        return STOTREE_ERR_ARG;
    }
    return mlp_forward_impl(rows, din, dh, dout, params, X, H, Y, (hipStream_t)hip_stream);
}

int warm_mlp_backward(int rows, int din, int dh, int dout, const float *params, const float *X, const float *H,
                      const float *dY, float *grad, float *work, void *hip_stream)
{
    if (rows < 1 || din < 1 || dh < 1 || dout < 1 || !params || !X || !H || !dY || !grad || !work) {
        set_error("warm_mlp_backward: bad argument");
        return STOTREE_ERR_ARG;
    }
    return mlp_backward_impl(rows, din, dh, dout, params, X, H, dY, grad, work, (hipStream_t)hip_stream);
}

int warm_mse_grad(int64_t n, const float *Y, const float *T, const float *mask, float inv_count, float *dY,
                  double *loss2, double *part, void *hip_stream)
{
    if (n < 1 || !Y || !T || !mask || !dY || !loss2 || !part) {
        set_error("warm_mse_grad: bad argument");
        return STOTREE_ERR_ARG;
    }
    return mse_grad_impl(n, Y, T, mask, inv_count, dY, loss2, part, (hipStream_t)hip_stream);
}

int warm_gather(int64_t rows, int cols, const float *src, int64_t src_rows, const int64_t *idx, float *dst,
                int *bad, void *hip_stream)
{
    if (rows < 1 || cols < 1 || src_rows < 1 || !src || !idx || !dst || !bad) {
        set_error("warm_gather: bad argument");
        return STOTREE_ERR_ARG;
    }
    return gather_rows_impl(rows, cols, src, src_rows, reinterpret_cast<const long long *>(idx), dst, bad,
                            (hipStream_t)hip_stream);
}

int warm_adam(int64_t n, float *params, const float *grad, float *m, float *v, float lr, float beta1, float beta2,
              float eps, int step, void *hip_stream)
{
    if (n < 1 || !params || !grad || !m || !v || step < 1) {
        set_error("warm_adam: bad argument");
        return STOTREE_ERR_ARG;
    }
    return adam_impl(n, params, grad, m, v, lr, beta1, beta2, eps, step, (hipStream_t)hip_stream);
}

int warm_features(const tree_factors *f, const double *x0, float c_scale, float *X, void *hip_stream)
{
    if (!f || !x0 || !X || !(c_scale > 0.0f) || f->cmap) { set_error("warm_features: bad argument (or a constraint map)"); return STOTREE_ERR_ARG; }
    return warm_features_impl(f, x0, c_scale, X, (hipStream_t)hip_stream);
}

int warm_scatter(const tree_factors *f, const float *Y, float y_scale, double *y, void *hip_stream)
{
    if (!f || !Y || !y || f->cmap) { set_error("warm_scatter: bad argument (or a constraint map)"); return STOTREE_ERR_ARG; }
    return warm_scatter_impl(f, Y, y_scale, y, (hipStream_t)hip_stream);
}

int warm_targets(const tree_factors *f, const double *y, float y_scale, float *T, float *mask, void *hip_stream)
{
    if (!f || !y || !T || !mask || !(y_scale > 0.0f) || f->cmap) { set_error("warm_targets: bad argument (or a constraint map)"); return STOTREE_ERR_ARG; }
    return warm_targets_impl(f, y, y_scale, T, mask, (hipStream_t)hip_stream);
}

int dual_select(const tree_factors *f, double *y, const int32_t *keep, void *hip_stream)
{
    if (!f || !y || !keep) { set_error("dual_select: bad argument"); return STOTREE_ERR_ARG; }
    for (int b = 0; b < f->ninst; ++b)
        if (!keep[b])
            STOTREE_HIP(hipMemsetAsync(y + f->inst[b].y, 0, sizeof(double) * f->inst[b].m, (hipStream_t)hip_stream));
    return STOTREE_OK;
}

int dual_merge(const tree_factors *f, double *y, const double *y_other, const int32_t *keep, void *hip_stream)
{
    if (!f || !y || !y_other || !keep) { set_error("dual_merge: bad argument"); return STOTREE_ERR_ARG; }
    for (int b = 0; b < f->ninst; ++b)
        if (!keep[b])
            STOTREE_HIP(hipMemcpyAsync(y + f->inst[b].y, y_other + f->inst[b].y, sizeof(double) * f->inst[b].m,
                                       hipMemcpyDeviceToDevice, (hipStream_t)hip_stream));
    return STOTREE_OK;
}

int stotree_timing(int enable) { return timing_enable(enable); }

int stotree_timing_read(double *ms, int64_t *count)
{
    if (!ms || !count) { set_error("stotree_timing_read: NULL argument"); return STOTREE_ERR_ARG; }
    long long c[4];
    const int rc = timing_read(ms, c);
    for (int p = 0; p < 4; ++p) count[p] = c[p];
    return rc;
}

}  // extern "C"
