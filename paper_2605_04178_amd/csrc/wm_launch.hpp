// wm_launch.hpp -- internal interface between the C ABI layer (wm_api.cpp)
// and the kernels (wm_kernels.hip).  Not installed; the public interface is
// include/wavemodel.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wavemodel.h"
#include "wm_model.hpp"

namespace wm {

constexpr int kGradMaxBlocks = 8192;   // partial-row cap of the persistent gradient grids
constexpr int kRedoMaxBlocks = 256;    // float64 re-evaluation grid cap
constexpr int kMaxSets = 16;           // parameter sets per batched calibration
constexpr float kTileWindow = 3e-5f;   // float32 window re-evaluated in float64

// A kernel launch shape: threads per block, descriptors per thread (forward
// sweep), persistent grid as a multiple of the resident blocks, and the work
// item size of the multi-set sweep.
struct LaunchCfg {
    int32_t block, vec, grid_mult, chunk;
};

// op codes as in the public header
constexpr int kOpPredict = 0, kOpVjp = 2, kOpLossGrad = 3, kOpSelectTile = 4,
              kOpCalibrate = 5, kOpCalibrateBatched = 6, kOpPredictApps = 7, kOpAppsLossGrad = 8;
constexpr int64_t kMinChunk = 256;

LaunchCfg default_cfg(int op);
bool cfg_valid(int op, const LaunchCfg& c);
// tuned configuration for (current device, op, floor(log2 n)) or the default
LaunchCfg launch_cfg(int op, int64_t n);
// record a configuration (and append it to the cache file, if one is set)
void store_cfg(int op, int64_t n, const LaunchCfg& c, double us, bool persist);

struct DescPtrs {
    const float *F, *B, *r1, *r2, *r3, *K, *u, *W;
    const int32_t *vgpr, *lds, *gpack, *grid;
};

// Segment rows (parallel to the descriptor rows) and the application CSR
// offsets over them.
struct SegPtrs {
    const int32_t* off;
    const float* n_exec;
    const int32_t *n_kern, *cls;
    const float *h2d, *d2h;
};

// Segment parameters: class scales of the kernel time, reciprocal transfer
// bandwidths, fixed cost per transfer episode.
template <typename R>
struct SegConst {
    R kappa[4];
    R inv_bw_h2d, inv_bw_d2h, tau;
};
struct SegSet {
    SegConst<float> f;
    SegConst<double> d;
    double inv_bw2_h2d, inv_bw2_d2h;  // 1 / B^2, for the bandwidth gradients
};
constexpr int kSegParams = 7;                 // kappa[4], bw_h2d, bw_d2h, tau_memcpy
constexpr int kAppRow = kAcc + 8;             // loss, count, grad theta[24], then the segment sums:
                                              // extra launches, kappa[4], h2d, d2h, transfers
constexpr int kAppsOut = kAcc + kSegParams;   // loss, count, grad theta[24], grad seg params[7]
constexpr int kAppsMaxBlocks = 4096;          // partial-row cap of the application sweep
constexpr int kAppsLongBlocks = 64;           // blocks of the pass over applications longer than a piece
constexpr int kFitMultMaxBlocks = 4096;       // multiplier sweep: one row per block
constexpr int kPlanMaxRun = 32;               // longest fused run

struct ShapePtrs {
    const int32_t *M, *N, *K, *dtype;
};

struct AdamOpts {
    int32_t steps, order;   // order: bit 0 slots 0-3 non-increasing, bit 1 slots 4-7 non-decreasing
    double lr, lr_final, beta1, beta2, eps;
    uint32_t free_mask, pad2_;
    double lo_log[kTheta], hi_log[kTheta];   // box on log(theta) of the fitted slots (+-inf: none)
    // per step s < steps, {learning rate, 1 - beta1^(s+1), 1 - beta2^(s+1)}
    // (device, formed on the host), or null to form them on the device
    const double* sched;
};

// The Adam schedule of one step: the learning rate (decayed geometrically
// from lr to lr_final over the steps when lr_final > 0) and the two bias
// corrections.  One definition for the host table and the device fallback.
WM_HD void adam_schedule(const AdamOpts& o, int32_t step_index, double* lr, double* c1,
                                double* c2)
{
    const double t = (double)(step_index + 1);
    double l = o.lr;
    if (o.lr_final > 0.0 && o.steps > 1)
        l = o.lr * pow(o.lr_final / o.lr, (double)step_index / (double)(o.steps - 1));
    *lr = l;
    *c1 = 1.0 - pow(o.beta1, t);
    *c2 = 1.0 - pow(o.beta2, t);
}

// device-resident calibration state of one parameter set
struct CalibState {
    double theta[kTheta];
    double theta_ok[kTheta];  // theta of the last step whose loss was finite
    double phi[kTheta];
    double m[kTheta];
    double v[kTheta];
    int32_t diverged;  // set once the loss, a gradient or theta left the finite range
    int32_t t;         // index of the next step
};

// Gradient sweep geometry for n descriptors: nb phase-1 blocks, nb2 phase-2
// blocks (partial rows nb + nb2), nwords 64-bit redo-flag words.
struct GradLayout {
    int nb, nb2;
    int64_t nwords;
};
GradLayout grad_layout(int64_t n);
// records e as the library's last HIP error and returns WM_EHIP
int32_t record_hip_error(hipError_t e);
// argument check of the gradient calls (wm_predict_vjp, wm_loss_grad): a
// valid descriptor set and parameter set, an output, weights unless n = 0
bool grad_args_ok(const wm_desc_t* desc, const float* w, const wm_params_t* params, const double* out);
// phase-1 blocks actually launched (<= grad_layout(n).nb): the blocks
// resident at once on the current device times cfg.grid_mult, so partial
// rows = that + nb2
int grad_grid(int mode, bool from_device_set, int64_t n, const LaunchCfg& cfg);
// blocks of `block` threads of `kernel` resident at once on the current device
int resident_blocks(const void* kernel, int block);
// blocks for the multi-set sweep over n_items work items
int batched_grid(int n_items, int grid_mult);
// blocks per set of the multi-set float64 pass (at most cap): all sets'
// blocks resident at once, no more than the largest set's flag words need
int batched_redo_grid(int n_sets, int64_t max_set_words, int cap);

hipError_t launch_predict(const DescPtrs& d, int64_t n, const Set& S, float* T, int32_t* occ,
                          bool vec_ok, const LaunchCfg& cfg, hipStream_t stream);
hipError_t launch_roofline(const DescPtrs& d, int64_t n, const Set& S, float* T,
                           hipStream_t stream);
// mode 0: weights are dL/dT, out = dL/dtheta[24]; mode 1: weights are measured
// times, out = [loss, count, grad[24]].  S_dev != nullptr reads the set from
// device memory (graph replay with a changing theta).  out == nullptr skips
// the final reduction.
hipError_t launch_grad(int mode, const DescPtrs& d, int64_t n, const float* w, const Set& S,
                       const Set* S_dev, double* partials, uint64_t* flags, const GradLayout& L,
                       const LaunchCfg& cfg, double* out, hipStream_t stream);
// The exact variant of launch_grad: every descriptor evaluated and
// differentiated in float64 (persistent grid of resident blocks x grid_mult).
hipError_t launch_grad_exact(int mode, const DescPtrs& d, int64_t n, const float* w, const Set& S,
                             double* partials, uint64_t* flags, const GradLayout& L, int grid_mult,
                             double* out, hipStream_t stream);
// Fixed-order reduction of `rows` partial rows of 26 doubles: mode 0 writes
// the 24 gradient sums, mode 1 [loss, count, grad[24]] divided by the count.
hipError_t launch_reduce(int mode, const double* partials, int rows, double* out, hipStream_t stream);
hipError_t launch_adam(const double* partials, int rows, CalibState* st, const AdamOpts& o, Set* S,
                       double* loss_hist, hipStream_t stream);
// Multi-set step: the work is n_items items of `chunk` descriptors (the
// last item of a set may be short); set k owns items item_off[k] ..
// item_off[k + 1] - 1 (device int32 [n_sets + 1]).
hipError_t launch_grad_batched(const DescPtrs* sets, const float* const* meas, const Set* S_all,
                               const int32_t* item_off, int n_items, int64_t chunk, int n_sets,
                               const int64_t* set_n, const int64_t* flag_off, uint64_t* flags,
                               double* partials, int nb, int nb2, hipStream_t stream);
hipError_t launch_adam_batched(const double* partials, int rows, int n_sets, CalibState* st,
                               const AdamOpts* opts, Set* S_all, int steps, double* loss_hist,
                               hipStream_t stream);
// Application totals (and, if T_seg != nullptr, segment times) in float32.
hipError_t launch_predict_apps(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg, int64_t n_apps,
                               const Set& S, const SegSet& Q, float* T_app, float* T_seg,
                               const LaunchCfg& cfg, hipStream_t stream);
// Application mean relative error and its gradient [kAppsOut] (float64), in
// one sweep over the rows.  Workspace: rows ((kAppsMaxBlocks + kAppsLongBlocks
// + kRedoMaxBlocks) x kAppRow doubles), aflags and lflags ((n_apps + 63) / 64
// words each), rflags ((n_seg + 63) / 64 words, cleared here), wrow (n_seg
// floats, written for flagged rows).
hipError_t launch_apps_loss_grad(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg, int64_t n_apps,
                                 const float* measured, const Set& S, const SegSet& Q, double* rows,
                                 uint64_t* aflags, uint64_t* lflags, uint64_t* rflags, float* wrow,
                                 const LaunchCfg& cfg, double* out, hipStream_t stream);
// Per-group weighted-median multipliers; rows: kFitMultMaxBlocks x 4
// doubles of workspace (one row per block); stats [4] float64 device.
hipError_t launch_fit_multipliers(const float* T, const float* meas, const int32_t* off,
                                  int64_t n_groups, int64_t n, const uint8_t* train, double* mult,
                                  float* T_scaled, double* rows, double* stats, hipStream_t s);
// Fusion-planning workspace over n descriptor rows.
struct PlanBufs {
    double* cost;       // n x R run costs (row of the run's last kernel, length - 1)
    int64_t* redo;      // n chains queued for the float64 redo
    uint8_t* cut;       // n chosen run lengths (rows beyond the ones kept in registers)
    uint8_t* cov;       // n: runs costed from each row (bits 0-5), bit 7 = one of them
                        // is uncertain
    uint32_t* n_redo;   // the queue's length
};
// Fusion plans of chains over n descriptor rows.
hipError_t launch_plan_fusion(const DescPtrs& d, const float* edge, const int32_t* off,
                              int64_t n_chains, int64_t n, int32_t R, const Set& S,
                              const double* peaks, const PlanBufs& wb, double* total,
                              double* unfused, uint8_t* start, hipStream_t s);
// Vector-Jacobian product of the application totals: out [31] = sum_a
// w_app[a] dT_a/d(theta[24], seg params[7]); workspace as the loss gradient.
hipError_t launch_apps_vjp(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg, int64_t n_apps,
                           const float* w_app, const Set& S, const SegSet& Q, double* rows, uint64_t* lflags,
                           uint64_t* rflags, float* wrow, const LaunchCfg& cfg, double* out, hipStream_t stream);
// every candidate's float32 cost, as the selection's first pass computes it
hipError_t launch_tile_costs(const ShapePtrs& sh, const int32_t* off, const uint32_t* code, int64_t n,
                             int64_t n_cand, const Set& S, float* cost, hipStream_t stream);
hipError_t launch_select_tile(const ShapePtrs& sh, const int32_t* off, const uint32_t* code,
                              int64_t n, int64_t n_cand, const Set& S, int32_t* best,
                              double* best_cost, uint8_t* near_tie, const LaunchCfg& cfg,
                              hipStream_t stream);

}  // namespace wm
