// Internal declarations of the stotree HIP library (not part of the ABI).
//
// A handle holds a forest: one or more independent scenario trees
// ("instances"), possibly of different sizes, horizons and nx/nu.  Every
// per-instance quantity lives in shared pools at an offset recorded in the
// instance's descriptor, and every kernel works on a flat list of
// (instance, item) pairs, so one launch covers all instances.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "stotree.h"

namespace stotree {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kWavesPerBlock = 4;    // independent wavefronts per block in chain kernels
constexpr int kMaxWidth = 256;       // nx + nu supported by the sweep kernels
constexpr int kRhsPanel = 64;        // right-hand sides of one matrix-core (panel) sweep

inline int pad2(int n) { return (n + 1) & ~1; }

// Per-instance sizes and offsets (elements) into the handle's pools.
struct InstDesc {
    int nx, nu, N, V, Vnl, sstar, nchains, ldM, ldx, ldu;
    int sp, cp;                      // offsets into the stage_ptr / child_ptr pools
    long long Mb, Mf, Kb, Kf, Rn;    // factor pools
    long long chat, sig, c, sc;      // node-vector pools (chat, c: V*nx; sig: Vnl*nu; sc: V)
    long long y;                     // first dual row in the concatenated dual vector
    long long x, u;                  // offsets in the concatenated x [sum V nx], u [sum Vnl nu]
    long long x0;                    // offset in the concatenated x0 [sum nx]
    long long m;                     // dual rows of the instance
    long long box;                   // first row of the instance's boxes in lo / hi
    long long node0;                 // first node of the instance in node-indexed work arrays
    // dual (constraint) layout: nc rows per non-leaf node, ncN per leaf; with
    // cmap the rows are z = [F G] (x, u) / FN x (matrices at Fo in the cmap
    // pool: F [nc][nx], G [nc][nu], FN [ncN][nx]); otherwise nc = nx + nu,
    // ncN = nx and the rows are (x, u) themselves
    int nc, ncN, cmap;
    long long Fo;
};

struct Item {
    int inst, idx;                   // instance and node / chain index within it
};

// Everything a sweep launch needs; passed by value to the kernels.
struct SweepArgs {
    const InstDesc *inst;
    const Item *items;
    int nitems;
    const int *sp, *cp;              // stage_ptr / child_ptr pools (local node ids)
    const int *anc;                  // ancestors, node-indexed at the instance's sc offset
    const double *Mb, *Mf, *Kb, *Kf, *Rn;
    const double *chat, *sig, *cvec, *sc;   // sc null: no preconditioning
    const double *x0; long long x0_rs;      // per right-hand side strides
    const double *y; long long y_rs;
    double *qhat, *kbuf; long long qhat_rs, kbuf_rs;
    double *xo, *uo; long long xo_rs, uo_rs;
    int dual_out;                    // 1: write H x into the dual layout at xo; 0: x at xo, u at uo
    int affine;
    int t;                           // stage of a per-stage launch
    long long chat_rs, c_rs;         // panel sweeps: chat / c stride between right-hand sides
    const int *done; int done_stride;       // per-instance skip flags (may be null)
    int panel_done;                  // 1: done holds the flags of one shared panel's kRhsPanel copies
};

// One launch of the chain kernels: the chains of every instance that uses
// lane groups of G lanes (G * 2 * CH >= nx + nu), kWave / G chains per item.
struct ChainPlan {
    int G, CH;
    int ldq;                         // largest padded nx + nu of its instances
    int count;                       // items = wavefronts
    Item *items;                     // device: (instance, first chain)
};

// One launch of the per-stage kernels: all (instance, node) pairs of one stage.
// With lane groups above s* (trunk mode 2) the stage is split into the nodes
// of instances with nx + nu > 64 (workgroups of wide_nw wavefronts per node)
// and lane-group items of kWave/G consecutive nodes of one instance.
struct LevelPlan {
    int t;
    int count;
    int nw;                          // wavefronts per node
    Item *items;                     // device
    int wide_count = 0, wide_nw = 1;
    Item *wide_items = nullptr;
    std::vector<ChainPlan> narrow;
};

// Solver workspace kept in the handle (allocated at the first solve).
struct SolverWS {
    int mem = 0;
    bool has_g = false;
    int nblocks = 0;
    double *buf = nullptr;
    size_t bytes = 0;
    double *y[2], *r[2], *hx, *hr2, *d, *S, *Qv, *g[2];
    double *yck = nullptr;           // iterate at the last infeasibility test (then the change since)
    double *Rw = nullptr, *hw = nullptr;  // backtracking test 1: R(w) and H x(w) of the last update
    double *xu = nullptr;            // constraint-map handles: [2][mxu] inputs and [2][mxu] outputs of the sweeps
    bool has_div = false, has_bt = false;
    double *partials;                // [kNVMax][nblocks]
    void *ctl;                       // device array of per-instance control blocks
    int *blk;                        // device: per block {instance, local block, blocks of the instance}
    int *ndone;                      // device counter of finished instances
    std::vector<int> blk_first;      // host: first block of each instance
};

}  // namespace stotree

struct tree_factors {
    int ninst = 0, precondition = 0;
    std::vector<stotree::InstDesc> inst;    // host copy
    stotree::InstDesc *d_inst = nullptr;
    std::vector<int> sp_pool;               // host copy of the stage pointers
    int *d_sp = nullptr, *d_cp = nullptr, *d_anc = nullptr;  // anc: node-indexed (sc offsets)
    double *Mb = nullptr, *Mf = nullptr, *Kb = nullptr, *Kf = nullptr, *Rn = nullptr;
    double *chat = nullptr, *sig = nullptr, *cvec = nullptr, *sc = nullptr;
    double *lo = nullptr, *hi = nullptr;    // unscaled box rows in the dual layout
    double *pw = nullptr, *hub = nullptr;   // soft rows: pi * weight (+inf: hard) and Huber threshold, or null
    double *Fm = nullptr;                   // constraint-map matrices (instances with cmap)
    // descriptors the sweeps use: the (x, u) layout of the duals they read and
    // of the H x they write (the same array as d_inst without a constraint map)
    stotree::InstDesc *d_inst_xu = nullptr;
    long long mxu_tot = 0;                  // length of the (x, u) layout (= m_tot without a map)
    bool cmap = false;                      // some instance has a constraint map
    double *map_ws = nullptr;               // dual_grad's (x, u)-layout inputs (constraint-map handles)
    long long map_ws_len = 0;
    double *Pcal = nullptr;                 // value-function Hessians [V][nx][nx] (kept only on request)
    long long m_tot = 0, n_tot = 0, x_tot = 0, u_tot = 0, nx_tot = 0, V_tot = 0;
    int max_width = 0;                      // max nx+nu over instances
    // schedule of a sweep
    std::vector<stotree::ChainPlan> chains;  // stages s*..N, one plan per lane-group width
    std::vector<stotree::LevelPlan> levels;  // stages 0..max(s*)-1
    stotree::Item *panel_chain_items = nullptr;  // (instance, chain) pairs of the panel sweeps
    int npanel_chain_items = 0;
    // shared > 1: the instances are copies of instance 0 (same tree, factors
    // and boxes; own x0 and vectors), and panel sweeps run across instances
    int shared = 1;
    std::vector<stotree::LevelPlan> panel_levels;  // shared handles: instance 0's trunk nodes
    // tuning knobs (sweep_schedule / sweep_autotune)
    int trunk_cap = 16;                     // cap on wavefronts per node above s*
    int chain_order = 1;                    // 1: longest chains first, 0: instance order
    int group_min = 8;                      // smallest lane group used for chains
    int trunk_fused = 0;                    // stages above s*: 0 per-stage launches, 1 one backward
                                            // launch, 2 per-stage launches with lane groups, 3 / 4
                                            // the first stages (at most kFuseNodes[mode] nodes each)
                                            // in one launch per direction, the rest per stage
    int panel_min = 16;                     // shared handles: fewest unfinished copies swept as panels
    stotree::LevelPlan trunk_entry{};       // nodes of stage s*-1 of every instance
    int *trunk_cnt = nullptr;               // per node (node0-indexed): children finished / parent
                                            // done; [V_tot]: error word of the fused launches
    stotree::LevelPlan fused_bwd{}, fused_fwd{};  // trunk modes 3, 4: the first stages' nodes
    std::vector<stotree::LevelPlan> rest_levels;  // trunk modes 3, 4: the other stages above s*
    long long schedule_epoch = 0;           // bumped whenever the work lists are rebuilt
    // sweep workspace (grows with nrhs)
    double *qhat = nullptr, *kbuf = nullptr;
    int ws_nrhs = 0;
    stotree::SolverWS sws;
    std::vector<solver_info> last_info;     // per instance, from the last solve
    size_t bytes = 0;
};

namespace stotree {

void set_error(const std::string &msg);

// factor.hip
int factor_forest(int count, const tree_desc *t, const problem_data *d, int precondition,
                  hipStream_t st, tree_factors **out, bool keep_pcal = false);
// count copies of instance 0; c_host [count][V][nx] (or null): per-copy
// disturbances, whose affine terms are derived from the kept P_i.
int replicate_instances(tree_factors *f, int count, const double *c_host, hipStream_t st);
void free_tree(tree_factors *f);
int build_schedule(tree_factors *f);
int chain_group(int ldM, int group_min);  // lanes per chain for padded width ldM

// sweep.hip
SweepArgs sweep_args(const tree_factors *f, int affine);
int ensure_sweep_ws(tree_factors *f, int nrhs);
// One full sweep (Algorithm 3 if a.affine, else Algorithm 4), nrhs in {1,2}.
// sweep_mfma.hip: the same for a panel of kRhsPanel right-hand sides on the
// matrix cores; panel_tpw == 0 if an instance is too wide for it.
int panel_tpw(const tree_factors *f);
hipError_t launch_panel_sweep(const tree_factors *f, const SweepArgs &a, hipStream_t st);
// Any sweep of nrhs in {1,2} right-hand sides over every instance: on a
// shared handle with at least panel_min of its copies unfinished (active;
// negative: all), panels of kRhsPanel copies; otherwise launch_sweep_tree.
bool shared_panels(const tree_factors *f);
bool panel_route(const tree_factors *f, int active);
hipError_t launch_sweep_any(const tree_factors *f, const SweepArgs &a, int nrhs, hipStream_t st, int active = -1);
hipError_t launch_sweep_tree(const tree_factors *f, const SweepArgs &a, int nrhs, hipStream_t st);
int timing_enable(int on);
bool timing_on();
int timing_read(double *ms, long long *count);
// dual_grad's work: right-hand sides two at a time, one sweep each pair.
// ws: null, the handle's workspace; else caller device memory of
// dual_grad_ws_rhs(f, nrhs) * (x_tot + u_tot) doubles.
int dual_grad_ws_rhs(const tree_factors *f, int nrhs);
int enqueue_dual_grad(tree_factors *f, const double *x0, const double *y, int homogeneous, int nrhs, double *x,
                      double *u, hipStream_t st, double *ws = nullptr);
// dual_grad with the q-hat / k workspace in the library's static device
// scratch (no allocation).
int dual_grad_noalloc_impl(const tree_factors *f, const double *x0, const double *y, int homogeneous, int nrhs,
                           double *x, double *u, hipStream_t st);

// schedule.hip
constexpr int kKnobs = 5;            // group_min, chain_order, trunk_cap, trunk_fused, panel_min
constexpr int kFusedKids = 1 << 30;  // Item.idx flag of the fused trunk lists: the children are listed too
// trunk modes 3 and 4: most nodes a stage may have to run in the fused launch
inline int fuse_limit(int mode) { return mode == 3 ? 64 : mode == 4 ? 256 : 0; }
int set_schedule(tree_factors *f, const int32_t *knobs);
int autotune(tree_factors *f, int nrhs, int reps, int32_t *knobs_out, double *ms_out, hipStream_t st);
int graph_create(tree_factors *f, const double *x0, const double *y, int homogeneous, int nrhs, double *x,
                 double *u, sweep_graph **out);
int graph_launch(sweep_graph *g, hipStream_t st);
void graph_free(sweep_graph *g);

// warm.hip
long long mlp_param_count(int din, int dh, int dout);
long long mlp_work_len(int rows, int din, int dh, int dout);
int mlp_forward_impl(int rows, int din, int dh, int dout, const float *P, const float *X, float *H, float *Y,
                     hipStream_t st);
int mlp_backward_impl(int rows, int din, int dh, int dout, const float *P, const float *X, const float *H,
                      const float *dY, float *G, float *work, hipStream_t st);
int mse_grad_impl(long long n, const float *Y, const float *T, const float *mask, float inv_count, float *dY,
                  double *loss2, double *part, hipStream_t st);
int gather_rows_impl(long long rows, int cols, const float *src, long long src_rows, const long long *idx,
                     float *dst, int *bad, hipStream_t st);
int adam_impl(long long n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
              int step, hipStream_t st);
int warm_features_impl(const tree_factors *f, const double *x0, float c_scale, float *X, hipStream_t st);
int warm_scatter_impl(const tree_factors *f, const float *Y, float y_scale, double *y, hipStream_t st);
int warm_targets_impl(const tree_factors *f, const double *y, float y_scale, float *T, float *mask, hipStream_t st);

// cmap.hip: the constraint map of Sec. II-B around the sweeps (no-ops
// without a map).  to_xu: out[k] = H' y[k] in the (x, u) layout (mxu_tot
// per right-hand side); from_xu: out[k] = H xu[k] in the dual layout.
hipError_t map_to_xu(const tree_factors *f, const double *y, long long y_rs, double *out, int nrhs, hipStream_t st);
hipError_t map_from_xu(const tree_factors *f, const double *xu, double *out, long long o_rs, int nrhs,
                       hipStream_t st);
int dual_grad_mapped(tree_factors *f, const double *x0, const double *y, int homogeneous, int nrhs, double *x,
                     double *u, hipStream_t st);

// solver.hip
int solve(const tree_factors *f, const double *x0, const solver_opts *opts, double *y,
          double *x, double *u, solver_info *info, hipStream_t st, int method);
int lipschitz(const tree_factors *f, int iters, double *L, hipStream_t st);

}  // namespace stotree

#define STOTREE_HIP(call)                                                        \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            stotree::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return e_ == hipErrorOutOfMemory ? STOTREE_ERR_OOM : STOTREE_ERR_DEVICE; \
        }                                                                        \
    } while (0)
