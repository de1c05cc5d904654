// Internal declarations of the stotree HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "stotree.h"

namespace stotree {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kWavesPerBlock = 4;    // independent waves per block in sweeps
constexpr int kMaxWidth = 256;       // nx + nu supported by the sweep kernels

inline int pad2(int n) { return (n + 1) & ~1; }

// Everything a sweep launch needs; passed by value to the kernels.
struct SweepArgs {
    int nx, nu, N, V, Vnl, sstar, nchains;
    int ldM, ldx, ldu;                 // padded row lengths (even)
    const int *stage_ptr, *child_ptr;  // device copies
    const double *Mb, *Mf, *Kb, *Kf, *Rn;
    const double *chat, *sig, *cvec, *sc;  // sc may be null (no preconditioning)
    const double *x0;  long long x0_rs;    // per right-hand side
    const double *y;   long long y_rs;
    double *qhat, *kbuf;                   // work: [nrhs][V][nx], [nrhs][Vnl][nu]
    long long qhat_rs, kbuf_rs;
    double *xo; long long xo_s;            // x of non-leaf i at xo + i*xo_s
    double *xl; long long xl_s;            // x of leaf j at xl + (j-Vnl)*xl_s
    double *uo; long long uo_s;            // u of non-leaf i at uo + i*uo_s
    long long xo_rs, uo_rs;                // right-hand-side strides of outputs
    int affine;
    const int *done;                       // if set and nonzero, the sweep is skipped
};

// Solver workspace kept in the handle (allocated at the first solve).
struct SolverWS {
    int mem = 0;
    int nblocks = 0;
    double *buf = nullptr;   // one allocation for all vectors
    size_t bytes = 0;
    double *y[2], *r[2], *hx, *hr2, *d, *S, *Qv, *g[2];
    double *partials;        // [nblocks][kPartialWidth]
    double *ctl;             // device control block (scalars)
};

}  // namespace stotree

struct tree_factors {
    int nx, nu, N, V, Vnl;
    long long m, n;
    int sstar, nchains, precondition;
    int ldM, ldx, ldu;
    std::vector<int> stage_ptr;  // host copy
    int *d_stage_ptr = nullptr, *d_child_ptr = nullptr;
    double *Mb = nullptr, *Mf = nullptr, *Kb = nullptr, *Kf = nullptr, *Rn = nullptr;
    double *chat = nullptr, *sig = nullptr, *cvec = nullptr, *sc = nullptr;
    double *lo = nullptr, *hi = nullptr;  // unscaled box rows in the dual layout
    // sweep workspace (grows with nrhs)
    double *qhat = nullptr, *kbuf = nullptr;
    int ws_nrhs = 0;
    stotree::SolverWS sws;
    size_t bytes = 0;
};

namespace stotree {

void set_error(const std::string &msg);

// factor.hip
int factor_tree(const tree_desc *t, const problem_data *d, int precondition,
                hipStream_t st, tree_factors **out);
void free_tree(tree_factors *f);

// sweep.hip
SweepArgs sweep_args(const tree_factors *f, int affine);
int ensure_sweep_ws(tree_factors *f, int nrhs);
// One full sweep (Algorithm 3 if a.affine, else Algorithm 4) for nrhs in {1,2}.
hipError_t launch_sweep_tree(const tree_factors *f, const SweepArgs &a, int nrhs, hipStream_t st);
int timing_enable(int on);
int timing_read(double *ms, long long *count);

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
