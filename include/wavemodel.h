/*
 * wavemodel.h -- C ABI of libwavemodel.so: batched evaluation, adjoint,
 * calibration and tile selection for the CDNA wavefront-centric
 * execution-time model (Section IV-B of "Microbenchmark-Driven Analytical
 * Performance Modeling Across Modern GPU Architectures").
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Memory.  Every array argument is DEVICE memory (HIP, gfx950) owned by
 *    the caller unless the comment says "host".  Structs passed by pointer
 *    (wm_desc_t, wm_params_t, wm_shapes_t, wm_calib_opts_t) live in host
 *    memory and are read during the call only.  The library allocates no
 *    memory: scratch comes from a caller workspace `ws` of `ws_bytes` bytes,
 *    sized by wm_workspace_bytes(), 256-byte aligned.
 *  - Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls enqueue work and return without synchronising, except
 *    wm_calibrate, wm_calibrate_batched and the wm_autotune_* calls, which synchronise
 *    `stream` once before returning (they write host results).
 *  - Errors.  Return value 0 (WM_OK) or a negative status.  Arguments are
 *    validated on the host before any HIP call, so a bad call never launches
 *    a kernel.  n == 0 returns WM_OK without a launch (array pointers may
 *    then be NULL), except that wm_predict_vjp and wm_loss_grad still write
 *    their zero-valued outputs and the calibration calls still take their
 *    steps over the empty set (loss 0, gradient 0, so theta keeps its value
 *    up to the rounding of exp(log theta)).  Problems of single
 *    descriptors are not errors: an invalid descriptor yields T = NaN and
 *    occ = -1; a resource-infeasible one (zero resident workgroups) yields
 *    T = +inf and occ = 0.
 *  - Determinism.  Same inputs on the same device give bitwise-identical
 *    outputs (no floating-point atomics; fixed-order FP64 reductions).
 *  - Thread safety.  Calls may come from several host threads; calls whose
 *    workspaces overlap race.
 *
 * Array layouts
 * -------------
 *  Descriptors are structure-of-arrays, n entries each: 8 float32 arrays
 *  (F flops, B bytes, r1/r2/r3 L1/L2/LLC hit rates, K steps per workgroup,
 *  u compute utilisation, W working-set bytes with 0 = unknown) and 4 int32
 *  arrays (vgpr VGPRs per thread, lds LDS bytes per workgroup, gpack, grid
 *  workgroups).  gpack bits: [0,11) workgroup threads g (1..1024), [11,14)
 *  dtype (0 fp64, 1 fp32, 2 bf16/fp16, 3 fp8, 4 int8), [14,17) concurrent
 *  kernels - 1, [17,20) devices - 1, [20] fused, [21,25) host syncs;
 *  bits 25..31 must be zero.  The vector path needs every array 16-byte
 *  aligned; misaligned arrays take a scalar path with the same results.
 */
#ifndef WAVEMODEL_H
#define WAVEMODEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define WM_OK 0
#define WM_EINVAL (-1)      /* null pointer, n < 0, invalid parameter set or option */
#define WM_EWORKSPACE (-2)  /* workspace missing, too small or misaligned */
#define WM_EHIP (-3)        /* a HIP call failed; see wm_last_hip_error() */
#define WM_EDIVERGED (-4)   /* calibration loss became non-finite */
#define WM_ETOOLARGE (-5)   /* input larger than a fixed-size scratch allows */

#define WM_N_THETA 24

/*
 * Parameter vector theta (SI units, latencies in cycles), Section IV-B and
 * Tables "arch-params" / "parameters":
 *   0-3   BW_L1, BW_L2, BW_LLC, BW_HBM      sustained bandwidth per level, B/s (> 0)
 *   4-7   Lat_L1, Lat_L2, Lat_LLC, Lat_HBM  load latency per level, cycles (>= 0), Eq. (10)
 *   8-12  P_fp64, P_fp32, P_bf16, P_fp8, P_int8  sustained peak per dtype, flop/s (> 0), Eq. (11)
 *   13    T_launch   launch + coherence + cross-XCD constant, s (>= 0), Eq. (13)
 *   14    tau_wg     per-workgroup dispatch overhead, s (>= 0), Eq. (14)
 *   15    tau_bar    per round x step synchronisation, s (>= 0)
 *   16    tau_interf per extra concurrent kernel, s (>= 0)
 *   17    tau_gpu    per extra device, s (>= 0)
 *   18    tau_fusion fused-kernel overhead, s (>= 0)
 *   19    tau_sync   per host synchronisation, s (>= 0), Section IV-E
 *   20-21 alpha, beta  h_LLC(W) exponents (> 0), Table "hlcc-piecewise"
 *   22    w0         working-set blend scale, bytes (<= 0 disables), Eq. (16)
 *   23    B_peak     HBM bandwidth ceiling for small working sets, B/s (> 0), Eq. (16)
 * With n_levels == 3 (no last-level cache) slots 2, 6, 20, 21 are unused.
 *
 * Structural integers are not calibrated.  wave in {32, 64}; vgpr_gran and
 * lds_gran powers of two; w_lo_mib < c_llc_mib, both exactly representable
 * as float32; combine 0 = HK_MAX (T_ov + max of compute, bandwidth and
 * latency stage times, Eq. (1)), 1 = PAPER_ETA (Eq. (9) and Eq. (12)).
 * mwp / cwp cap the wavefronts counted for overlap (0 = unset).
 */
typedef struct {
    int32_t n_levels, n_cu, n_simd, wave, vgpr_simd, vgpr_gran, waves_simd,
            lds_cu, lds_gran, bytes_inflight_wave, mwp, cwp, combine, reserved;
    double f_clk, w_lo_mib, c_llc_mib;
    double theta[WM_N_THETA];
} wm_params_t;

typedef struct {
    const float *F, *B, *r1, *r2, *r3, *K, *u, *W;
    const int32_t *vgpr, *lds, *gpack, *grid;
    int64_t n;
} wm_desc_t;

/* GEMM-like shapes for tile selection: M, N, K >= 1, dtype 0..3
 * (fp64, fp32, bf16/fp16, fp8), n shapes. */
typedef struct {
    const int32_t *M, *N, *K, *dtype;
    int64_t n;
} wm_shapes_t;

/* Calibration options.  Optional constraints keep a fit physical: after
 * every Adam update the fitted log-parameters are projected, first onto the
 * level ordering of `order` (the closest ordered values in log space), then
 * into the box [lo_j, hi_j] of each fitted slot.  Boxes of an ordered group
 * must be ordered the same way (then the two steps together are the
 * projection onto both constraints).  A zero-filled constraint part means
 * none; the first update projects a p0 that lies outside. */
typedef struct {
    int32_t steps;        /* Adam steps (>= 1) */
    int32_t order;        /* bit 0: BW_L1 >= BW_L2 >= BW_LLC >= BW_HBM (slots 0-3),
                             bit 1: Lat_L1 <= Lat_L2 <= Lat_LLC <= Lat_HBM (slots 4-7);
                             a set bit needs its group's four slots free; CDNA calls only */
    double lr;            /* initial learning rate on log(theta) (> 0) */
    double lr_final;      /* geometric decay to this rate at the last step; 0 = constant */
    double beta1, beta2;  /* Adam moment decay rates, in [0, 1) */
    double eps;           /* Adam epsilon (> 0) */
    uint32_t free_mask;   /* bit j set: slot j is fitted; the others stay fixed */
    uint32_t reserved2;
    double lo[WM_N_THETA];  /* lower bound of fitted slot j (> 0), 0 = none; finite */
    double hi[WM_N_THETA];  /* upper bound of fitted slot j (>= lo[j]), 0 = none; finite */
} wm_calib_opts_t;

/*
 * Workload segments (Sections IV-E, IV-F and V-B).  An application is a run
 * of consecutive segment rows; segment row i pairs descriptor row i of a
 * wm_desc_t with:
 *   n_exec [n] float32  executions of the segment (finite, >= 0)
 *   n_kern [n] int32    kernels launched per execution (>= 1); each beyond
 *                       the first adds T_launch (theta slot 13)
 *   cls    [n] int32    class 0 memory, 1 compute, 2 balanced, 3 stencil:
 *                       selects the scale kappa_cls of the kernel time
 *   h2d, d2h [n] float32  host-to-device / device-to-host bytes per
 *                       execution (finite, >= 0; 0 = no transfer)
 *   app_off [n_apps + 1] int32  application a owns rows
 *                       [app_off[a], app_off[a + 1]); non-decreasing,
 *                       app_off[0] = 0, app_off[n_apps] = n.  Offsets are
 *                       read on the device and clamped into [0, n]: offsets
 *                       that break these rules give unspecified results but
 *                       never an out-of-range access.
 * A row with a field outside these ranges makes its application's time NaN.
 */
typedef struct {
    const int32_t *app_off;
    const float *n_exec;
    const int32_t *n_kern, *cls;
    const float *h2d, *d2h;
    int64_t n_apps;
} wm_segs_t;

/* Segment parameters (host struct): kappa[4] per-class scales of the kernel
 * time (finite, >= 0; Section IV-F's separately calibrated class scales),
 * bw_h2d / bw_d2h effective transfer bandwidths in B/s (> 0) and tau_memcpy
 * the fixed cost per transfer episode in s (>= 0), Eq. (15).  Table
 * "parameters" defaults: 45e9, 45e9, 2e-6. */
typedef struct {
    double kappa[4];
    double bw_h2d, bw_d2h;
    double tau_memcpy;
} wm_segparams_t;

#define WM_N_SEGPARAMS 7

/* ---- host-only helpers (no HIP call) ---- */

/* Text for a status code; never NULL. */
const char *wm_strerror(int32_t status);

/* HIP error code of the last WM_EHIP on the calling thread (0 if none). */
int32_t wm_last_hip_error(void);

/* WM_OK if the parameter set is usable by the kernels (units and ranges as
 * listed above, every derived float32 constant finite), else WM_EINVAL. */
int32_t wm_validate_params(const wm_params_t *params);

/* Workspace bytes for an operation (0 if none is needed; 0 for bad
 * arguments):
 *  WM_OP_PREDICT, WM_OP_ROOFLINE, WM_OP_SELECT_TILE: 0.
 *  WM_OP_VJP, WM_OP_LOSS_GRAD: per-block FP64 partial sums for n descriptors.
 *  WM_OP_CALIBRATE: device parameter set, Adam state, a `steps`-entry loss
 *      history, the per-step Adam schedule (learning rate and the two bias
 *      corrections, formed on the host) and the partial sums for n
 *      descriptors.
 *  WM_OP_CALIBRATE_BATCHED: the same for n_sets sets holding n descriptors
 *      in total, plus the per-set pointer tables and item offsets.
 *  WM_OP_PREDICT_APPS: 0.
 *  WM_OP_APPS_LOSS_GRAD: 0 here; its size depends on the application count
 *      too: use wm_apps_workspace_bytes().
 *  WM_OP_FIT_MULTIPLIERS: a fixed block of per-wave partial sums (any n).
 *  Fusion planning: use wm_plan_workspace_bytes(). */
#define WM_OP_PREDICT 0
#define WM_OP_ROOFLINE 1
#define WM_OP_VJP 2
#define WM_OP_LOSS_GRAD 3
#define WM_OP_SELECT_TILE 4
#define WM_OP_CALIBRATE 5
#define WM_OP_CALIBRATE_BATCHED 6
#define WM_OP_PREDICT_APPS 7
#define WM_OP_APPS_LOSS_GRAD 8
#define WM_OP_FIT_MULTIPLIERS 9
size_t wm_workspace_bytes(int32_t op, int64_t n, int32_t n_sets, int32_t steps);

/* Workspace bytes of wm_apps_loss_grad for n segment rows in n_apps
 * applications: per-row adjoint weights, per-application flags and partial
 * sums (0 for negative arguments). */
size_t wm_apps_workspace_bytes(int64_t n, int64_t n_apps);

/* ---- device calls ---- */

/*
 * Predicted execution time of every descriptor (Section IV-B): occupancy
 * from VGPR, wave-slot and LDS limits; workgroup rounds n_r =
 * ceil(G / (N_CU o)) (Eq. (14)); hit-weighted bandwidth and latency over the
 * cache levels (Eq. (10)), with h_LLC(W) (Table "hlcc-piecewise") and the
 * Eq. (16) HBM blend when W > 0; compute time F / (u P_dtype) (Eq. (11));
 * stage times combined per params->combine plus the overhead terms of
 * Eq. (13), Eq. (14) and Section IV-E.
 *   T   [n] float32 seconds (required).
 *   occ [n] int32 resident workgroups per CU, or NULL to skip.
 * Computed in float32; error against the FP64 definition is below 1e-5
 * relative; occupancy is exact.
 */
int32_t wm_predict(const wm_desc_t *desc, const wm_params_t *params, float *T, int32_t *occ,
                   void *stream);

/* Naive roofline max(F / P_dtype, B / BW_HBM) (Section V-A), float32 [n];
 * NaN for invalid descriptors. */
int32_t wm_roofline(const wm_desc_t *desc, const wm_params_t *params, float *T, void *stream);

/*
 * Vector-Jacobian product: dL_dtheta[j] = sum_i dL_dT[i] * dT_i/dtheta_j over
 * descriptors with finite T (analytic derivative of the model; subgradient at
 * the max/min switches: first maximal stage, saturated overlap branch when
 * (N_eff - 1) T_c >= T_m).  dL_dT [n] float32; dL_dtheta [24] float64
 * device.  Partials are float32; descriptors within 1e-5 of a switch are
 * re-evaluated in float64; sums are float64 in a fixed order.
 * Workspace: wm_workspace_bytes(WM_OP_VJP, n, 1, 0).
 */
int32_t wm_predict_vjp(const wm_desc_t *desc, const wm_params_t *params, const float *dL_dT,
                       double *dL_dtheta, void *ws, size_t ws_bytes, void *stream);

/*
 * Mean relative error and its gradient: over descriptors with finite T and
 * finite measured m > 0, loss = mean |T - m| / m and
 * grad_j = mean sign(T - m) / m * dT/dtheta_j (sign(0) = 0).  Where
 * |T/m - 1| < 1e-5 in float32 the descriptor is re-evaluated in float64 to
 * take the sign.  out [26] float64 device: loss, count, grad[24].
 * Workspace: wm_workspace_bytes(WM_OP_LOSS_GRAD, n, 1, 0).
 */
int32_t wm_loss_grad(const wm_desc_t *desc, const float *measured, const wm_params_t *params,
                     double *out, void *ws, size_t ws_bytes, void *stream);

/*
 * The exact variants of wm_predict_vjp and wm_loss_grad: the same sums, but
 * every descriptor is evaluated and differentiated in float64 (no float32
 * stage, no near-switch redo).  The default calls form each descriptor's
 * Jacobian row in float32 (relative rounding ~1e-7 per term); near a
 * calibration optimum the signed terms of the loss gradient cancel to
 * ~1e-6 of their absolute sum, so that rounding alone can reach ~1e-4 of a
 * small slot's gradient.  These calls keep every slot to float64 rounding
 * at about 1.4x the sweep time.  Same arguments, workspace
 * (wm_workspace_bytes(WM_OP_VJP / WM_OP_LOSS_GRAD, n, 1, 0)) and status
 * codes as the default calls.
 */
int32_t wm_predict_vjp_exact(const wm_desc_t *desc, const wm_params_t *params, const float *dL_dT,
                             double *dL_dtheta, void *ws, size_t ws_bytes, void *stream);
int32_t wm_loss_grad_exact(const wm_desc_t *desc, const float *measured, const wm_params_t *params,
                           double *out, void *ws, size_t ws_bytes, void *stream);

/*
 * wm_loss_grad without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and status codes as wm_loss_grad; the workspace is a fixed device array of
 * wm_noalloc_scratch_bytes() bytes (about 9.7 MiB) inside the library, one
 * copy per GPU, held until the process ends.  n above WM_NOALLOC_MAX_N
 * returns WM_ETOOLARGE.  The array's device address is looked up on the
 * first call on each device (a HIP symbol lookup, no allocation; call once
 * before a graph capture starts).  All calls on one GPU share its array:
 * calls that overlap in time on one GPU (two streams, or two host threads)
 * race and give wrong results; calls in one stream are ordered and safe.
 */
#define WM_NOALLOC_MAX_N (1 << 26)
size_t wm_noalloc_scratch_bytes(void);
int32_t wm_loss_grad_noalloc(const wm_desc_t *desc, const float *measured, const wm_params_t *params,
                             double *out, void *stream);

/*
 * Adaptive tile selection (Section IV-B: evaluate candidate tiles with the
 * model and return the fastest).  Each shape i has candidates
 * cand_code[cand_off[i] .. cand_off[i+1]) (cand_off [n+1] int32,
 * non-decreasing, cand_off[0] = 0; n_cand = cand_off[n], passed for
 * validation).  Code = mt | nt << 2 | kd << 4 | (waves - 1) << 6 with
 * mt, nt in {32, 64, 128, 256}, kd in {16, 32, 64}, waves 1..8; other bits
 * zero.  The tile becomes a descriptor (grid ceil(M/mt) ceil(N/nt), K loop
 * ceil(K/kd) steps, padded flops, panel bytes, L2 reuse 1 - unique/loaded,
 * VGPRs for accumulators and panels, double-buffered LDS) whose predicted
 * time is its cost; a grid of more than 2^31 - 1 workgroups is infeasible.  Outputs per shape: best [n] int32 local index of the
 * cheapest candidate (ties to the lowest index; -1 if none is feasible),
 * best_cost [n] float64 its float64 cost (+inf if none), near_tie [n]
 * uint8 = 1 when the runner-up is within 1e-6 relative.  A float32 sweep
 * picks the candidates within 3e-5 of the minimum; those are re-evaluated in
 * float64, which decides.  One persistent launch.
 */
int32_t wm_select_tile(const wm_shapes_t *shapes, const int32_t *cand_off,
                       const uint32_t *cand_code, int64_t n_cand, const wm_params_t *params,
                       int32_t *best, double *best_cost, uint8_t *near_tie, void *stream);

/*
 * The float32 cost of every candidate, as the first pass of wm_select_tile
 * computes it (same tile derivation and model evaluation; Section IV-B,
 * adaptive tile selection): cost [n_cand] float32, +inf for an invalid code
 * or an infeasible tile.  Shapes and CSR lists as for wm_select_tile; a
 * candidate outside every shape's (clamped) list is not written.  For
 * ranking tiles, and for bounding the float32 error that the selection's
 * float64 window must cover.
 */
int32_t wm_tile_costs(const wm_shapes_t *shapes, const int32_t *cand_off, const uint32_t *cand_code,
                      int64_t n_cand, const wm_params_t *params, float *cost, void *stream);

/*
 * Calibration (Section IV-D): fit the free slots of theta to measured times
 * by Adam on log(theta) over the mean relative error (wm_loss_grad), all on
 * the device; the step loop is captured once as a HIP graph and replayed.
 * measured [n] float32 device.  p_out (host) receives p0 with the fitted
 * theta; loss_hist (host, [opts->steps], may be NULL) the loss before each
 * update.  Returns WM_EDIVERGED if the loss became non-finite; p_out then
 * holds the last theta with a finite loss.  Synchronises `stream`.
 * Workspace: wm_workspace_bytes(WM_OP_CALIBRATE, n, 1, opts->steps).
 */
int32_t wm_calibrate(const wm_desc_t *desc, const float *measured, const wm_params_t *p0,
                     const wm_calib_opts_t *opts, wm_params_t *p_out, double *loss_hist,
                     void *ws, size_t ws_bytes, void *stream);

/*
 * Calibration state, for checkpointing a calibration and resuming it: the
 * Adam iterate on log(theta) (Section IV-D's calibration) in plain doubles,
 * to be saved and restored by the caller as it is.
 */
typedef struct {
    double theta[WM_N_THETA];     /* current parameters */
    double theta_ok[WM_N_THETA];  /* parameters after the last step with a finite loss */
    double phi[WM_N_THETA];       /* log(theta) of the fitted slots, 0 for the others */
    double m[WM_N_THETA];         /* Adam first moments */
    double v[WM_N_THETA];         /* Adam second moments */
    int32_t step;                 /* steps taken (index of the next step) */
    int32_t diverged;             /* 1 once the loss became non-finite */
} wm_calib_state_t;

/*
 * wm_calibrate in pieces: run `run_steps` steps of the schedule that
 * opts->steps defines (the learning rate decays over opts->steps steps),
 * starting from state_in (host; NULL = a fresh start from p0's theta, with
 * zero moments) and write the state after the last step to state_out (host,
 * may be NULL).  Requires state_in->step + run_steps <= opts->steps; with a
 * state, p0 supplies the structure and the state the parameters (a
 * diverged state is rejected with WM_EINVAL).  A calibration split into calls with the state carried over (or saved and
 * restored) gives the same parameters and loss history, bit for bit, as one
 * call.  loss_hist (host, [run_steps], may be NULL): the losses of these
 * steps.  p_out, status and synchronisation as for wm_calibrate.
 * Workspace: wm_workspace_bytes(WM_OP_CALIBRATE, n, 1, opts->steps).
 */
int32_t wm_calibrate_resume(const wm_desc_t *desc, const float *measured, const wm_params_t *p0,
                            const wm_calib_opts_t *opts, const wm_calib_state_t *state_in,
                            int32_t run_steps, wm_calib_state_t *state_out, wm_params_t *p_out,
                            double *loss_hist, void *ws, size_t ws_bytes, void *stream);

/*
 * Several calibration problems (one parameter set and one descriptor set
 * each; different sizes and hierarchies, as in porting the model to several
 * architectures by parameters alone, Section IV-B) advanced together: each
 * step is one persistent sweep over all sets' descriptors in items of
 * `chunk` (each block takes a contiguous range of items), one float64 pass
 * with a block row per set, and one per-set reduce-and-Adam launch.  sets, measured, p0, opts, p_out: host
 * arrays of n_sets entries (measured[s] device pointers); every set uses
 * opts[s] but all must have the same step count; loss_hist host
 * [n_sets][steps] or NULL.  Workspace: wm_workspace_bytes(
 * WM_OP_CALIBRATE_BATCHED, sum of n, n_sets, steps).  At most 16 sets.
 * Synchronises `stream`.
 */
int32_t wm_calibrate_batched(int32_t n_sets, const wm_desc_t *sets, const float *const *measured,
                             const wm_params_t *p0, const wm_calib_opts_t *opts,
                             wm_params_t *p_out, double *loss_hist, void *ws, size_t ws_bytes,
                             void *stream);

/*
 * Application times: T_app[a] = sum over the application's rows of
 *   n_exec (kappa_cls T_kernel + (n_kern - 1) T_launch
 *           + [h2d > 0] (h2d / bw_h2d + tau_memcpy)
 *           + [d2h > 0] (d2h / bw_d2h + tau_memcpy)),
 * T_kernel the wm_predict time of the row's descriptor (segment times
 * multiply by n_exec, Section IV-E; extra launches of multi-kernel segments,
 * Section IV-F; transfers by Eq. (15); no overlap of copies and kernels).
 * NaN if any row is invalid, else +inf if any kernel is infeasible; 0 for an
 * application without rows.  T_app [n_apps] float32 (required); T_seg [n]
 * float32 segment times or NULL.  Segment times are float32; application
 * sums are float64 in row order, then rounded to float32.  One launch.
 */
int32_t wm_predict_apps(const wm_desc_t *desc, const wm_segs_t *segs, const wm_params_t *params,
                        const wm_segparams_t *segp, float *T_app, float *T_seg, void *stream);

/*
 * Application-level mean relative error and its gradient (Section V-B: an
 * application's prediction is the sum of its segments, compared with its
 * measured time): over applications with finite T_app and finite measured
 * m > 0, loss = mean |T_app - m| / m, with the gradient with respect to theta
 * and the segment parameters (sign(0) = 0; subgradients of the kernel model
 * as in wm_predict_vjp).  Applications with |T_app/m - 1| <= 1e-5 are summed
 * again in float64 to take the sign.  measured [n_apps] float32.  out [33]
 * float64 device: loss, count, dL/dtheta[24], dL/d(kappa[4], bw_h2d, bw_d2h,
 * tau_memcpy).  Workspace: wm_apps_workspace_bytes(n, n_apps).  An
 * application sweep, a float64 pass over the flagged applications, the
 * gradient sweep of wm_predict_vjp over the rows, and a final reduction.
 */
int32_t wm_apps_loss_grad(const wm_desc_t *desc, const wm_segs_t *segs, const float *measured,
                          const wm_params_t *params, const wm_segparams_t *segp, double *out,
                          void *ws, size_t ws_bytes, void *stream);

/*
 * Vector-Jacobian product of the application times: given dL/dT_app
 * [n_apps] float32, out [31] float64 device = sum over applications with
 * finite T_app of dL/dT_app * dT_app/d(theta[24], kappa[4], bw_h2d, bw_d2h,
 * tau_memcpy) (subgradients of the kernel model as in wm_predict_vjp).
 * Workspace: wm_apps_workspace_bytes(n, n_apps).
 */
int32_t wm_predict_apps_vjp(const wm_desc_t *desc, const wm_segs_t *segs, const float *dL_dTapp,
                            const wm_params_t *params, const wm_segparams_t *segp, double *out,
                            void *ws, size_t ws_bytes, void *stream);

/*
 * Per-group calibration multipliers (Section IV-D: optional per-case
 * multipliers, fitted with train / holdout separation; Section V-B: m_case).
 * Group g owns rows [group_off[g], group_off[g+1]) of n rows (CSR,
 * non-decreasing, group_off[n_groups] = n; offsets are clamped into [0, n]).
 * Over the group's valid training rows (T and measured finite and > 0,
 * train != 0) the multiplier minimises sum |mult * T - m| / m: a weighted
 * median of m/T with weights T/m -- the smallest ratio (ties: lowest row)
 * whose cumulative weight reaches half the total.  Groups without a valid
 * training row get 1.  Outputs (device): mult [n_groups] float64, T_scaled
 * [n] float32 = mult * T, stats [4] float64 = training error sum, training
 * rows, held-out error sum, held-out rows.  Ratios and weights are float64;
 * a group of up to 64 rows is sorted by (ratio, row) across one wave's lanes
 * (two groups of up to 32 rows share a wave) and its cumulative weights are
 * a float64 prefix sum in tree order; larger groups compare every candidate
 * with every row (float32 ratio order, float64 where those tie, float64 sums
 * in row order).  Either way a multiplier can differ from the sequential
 * sorted-order one only where two candidates' objectives tie to rounding.
 * Cost O(log^2 s) lane steps per group of s <= 64 rows, O(s^2 / 64) beyond.
 * Workspace: wm_workspace_bytes(WM_OP_FIT_MULTIPLIERS, n, 1, 0).
 */
int32_t wm_fit_multipliers(const float *T, const float *measured, const int32_t *group_off,
                           int64_t n_groups, int64_t n, const uint8_t *train, double *mult,
                           float *T_scaled, double *stats, void *ws, size_t ws_bytes, void *stream);

/*
 * Kernel-fusion planning (Section IV-B: a fused kernel is modelled with the
 * combined flops and bytes plus tau_fusion).  Chain c owns descriptor rows
 * [chain_off[c], chain_off[c+1]) in execution order (CSR, non-decreasing;
 * offsets are clamped into [0, n]; with offsets that are not non-decreasing,
 * a chain overlapping another can get NaN totals and leave its start flags
 * unwritten); edge [n] float32: bytes row i hands to row i + 1 (read only
 * inside a chain).  A plan cuts each chain into runs of 1 .. R (<= 32)
 * consecutive kernels, each run modelled as one kernel whose descriptor
 * combines the rows: flops, steps and host syncs add; bytes add minus twice
 * the edges inside the run (intermediates stay on chip); working set adds
 * minus the edges; hit rates are byte-weighted; u keeps the summed compute
 * time at the dtype of the largest-flop row (capped at 1); VGPRs, LDS,
 * workgroup size, grid and concurrency take the maximum; the fused flag adds
 * tau_fusion.  The sums forming a combined descriptor are float64; each
 * run's cost is the model evaluated in float32 on that descriptor (+inf for
 * runs with an invalid row or edge); the optimal plan comes from the prefix
 * dynamic programme over those costs in float64 (shortest run first on
 * ties).  A chain is redone with float64 costs when one of its decisions is
 * within 1e-5 relative of the runner-up, or when one of its runs has a cost
 * float32 cannot carry (not finite for valid rows, negative, or a working set
 * within 1e-6 relative of the LLC capacity, where the hit rate jumps): plans
 * then match a float64 evaluation except at its own ties, and totals match
 * it to the model's float32 error (float64 rounding for redone chains).
 * Outputs (device): total [n_chains] and unfused [n_chains] float64 (the
 * optimal and the all-singles sums), start [n] uint8 = 1 where a run of the
 * optimal plan begins.  Workspace: wm_plan_workspace_bytes(n, R); after the
 * call, the uint32 that starts its last 256 bytes is the number of chains
 * redone in float64.
 */
size_t wm_plan_workspace_bytes(int64_t n, int32_t R);
int32_t wm_plan_fusion(const wm_desc_t *desc, const float *edge, const int32_t *chain_off,
                       int64_t n_chains, int32_t R, const wm_params_t *params, double *total,
                       double *unfused, uint8_t *start, void *ws, size_t ws_bytes, void *stream);

/*
 * ---- Blackwell stage-centric family (Section IV-A) ----
 * A second per-descriptor model on the same batched machinery.  Parameter
 * vector (24 slots; rates per SM in B/s or flop/s, latencies in cycles at
 * f_clk, times in s):
 *   0 BW_TMEM_read   1 BW_TMEM_write   2 L_mma           (Eq. (2))
 *   3-7 R_TC per dtype: fp64, tf32, fp16/bf16, fp8, fp4  (Eq. (3))
 *   8 S_2SM (2-SM speedup)             (Eq. (6))
 *   9 L_TMA   10 B_TMA                 (Eq. (4))
 *   11 L_mbar   12 L_commit            (sync per K-step)
 *   13 BW_link  14 eta_DE  15 R_decomp  16 L_decomp_setup   (Eq. (5))
 *   17 eps = 1 - alpha, the exposed I/O fraction            (Eq. (7))
 *   18 B_gmem  19 L_store_setup  (C-tile writeback)
 *   20 L_alloc + L_dealloc (TMEM management, amortised over K-steps)
 *   21 O_misc (per step)  22 T_launch  23 BW_dsmem (2-SM B-tile exchange)
 * All slots > 0 except 2, 9, 11, 12, 16, 19, 20, 21, 22 (>= 0) and
 * 17 (>= 0).  Structure: n_sm (1..65536), max_cta (CTAs per SM cap,
 * 1..64), tmem_bytes per SM (1 .. 2^30 - 1), f_clk.
 * Descriptors (structure of arrays, 32 B each): bM, bN, bK tile sizes
 * (>= 1), G CTAs (>= 1), flags ([0,3) dtype 0..4, [3] 2-SM pair, [4] TMEM
 * strategy B (A tile through TMEM), [5,9) P_A - 1, [9,13) P_B - 1 multicast
 * participants, [13,16) barriers per K-step, [16] compressed operands; other
 * bits zero) as int32; Kt K-steps per tile (>= 1), CR compression ratio
 * (>= 1), ob output element bytes (> 0) as float32.  Invalid rows give NaN
 * and cta = -1; an accumulator larger than TMEM gives +inf and cta = 0.
 * The model, term by term: see the paper's Eq. (2)-(8); per K-step
 * T_step = max(T_compute, eps (T_tma + T_decomp + T_dsm) + T_sync) + T_sync +
 * O_misc; kernel T = T_launch + n_r (Kt T_step + T_store), n_r =
 * ceil(G / (n_sm cta)).
 */
typedef struct {
    int32_t n_sm, max_cta;
    int64_t tmem_bytes;
    double f_clk;
    double theta[WM_N_THETA];
} wm_bw_params_t;

typedef struct {
    const int32_t *bM, *bN, *bK, *G, *flags;
    const float *Kt, *CR, *ob;
    int64_t n;
} wm_bw_desc_t;

#define WM_BW_OP_GRAD 0       /* wm_bw_predict_vjp, wm_bw_loss_grad */
#define WM_BW_OP_CALIBRATE 1  /* wm_bw_calibrate */

int32_t wm_bw_validate_params(const wm_bw_params_t *params);
/* Workspace bytes of a Blackwell call for n descriptors (steps: calibration
 * steps, ignored for WM_BW_OP_GRAD); 0 for bad arguments. */
size_t wm_bw_workspace_bytes(int32_t op, int64_t n, int32_t steps);
/* Predicted time T [n] float32 s (required) and CTAs per SM cta [n] int32
 * (or NULL); float32, error against the FP64 definition below 1e-5. */
int32_t wm_bw_predict(const wm_bw_desc_t *desc, const wm_bw_params_t *params, float *T, int32_t *cta,
                      void *stream);
/* As wm_predict_vjp / wm_loss_grad for the Blackwell model (subgradient at
 * the compute / I-O switch: compute on ties; descriptors within 1e-5 of the
 * switch or of T = m are re-evaluated in float64). */
int32_t wm_bw_predict_vjp(const wm_bw_desc_t *desc, const wm_bw_params_t *params, const float *dL_dT,
                          double *dL_dtheta, void *ws, size_t ws_bytes, void *stream);
int32_t wm_bw_loss_grad(const wm_bw_desc_t *desc, const float *measured, const wm_bw_params_t *params,
                        double *out, void *ws, size_t ws_bytes, void *stream);
/* As wm_calibrate (Adam on log theta in captured HIP graphs). */
int32_t wm_bw_calibrate(const wm_bw_desc_t *desc, const float *measured, const wm_bw_params_t *p0,
                        const wm_calib_opts_t *opts, wm_bw_params_t *p_out, double *loss_hist,
                        void *ws, size_t ws_bytes, void *stream);

/* ---- launch configurations and autotuning ----
 *
 * Every call above launches its kernels with a configuration looked up by
 * (GPU architecture, compute-unit count, op, floor(log2 n)); without an entry
 * it uses the default.  Fields: block = threads per block (64, 128, 256,
 * 512); per_thread = descriptors per thread of the forward sweep (1, 2, 4,
 * 8; other ops ignore it); grid_mult = persistent grid as a multiple of the
 * blocks resident at once (1..8; gradient, tile and batched sweeps); chunk =
 * descriptors per work item of the batched sweep (power of two, 256..65536;
 * that op requires block 256).  Results do not depend on the configuration
 * except through the order of FP64 additions in gradient sums (differences
 * of order 1e-15 relative).  Entries live in process memory; if the
 * environment variable WAVEMODEL_TUNE_CACHE names a file, tuning results are
 * appended to it as JSON lines and read back at the first lookup.
 */
typedef struct {
    int32_t block, per_thread, grid_mult, chunk;
} wm_launch_t;

/* Configuration the next call of `op` on n items would use (host; queries the
 * current device).  WM_EINVAL for an unknown op or a NULL cfg. */
int32_t wm_get_launch(int32_t op, int64_t n, wm_launch_t *cfg);

/* Install a configuration for (current device, op, floor(log2 n)).
 * WM_EINVAL if it is not valid for the op (checked before any HIP call). */
int32_t wm_set_launch(int32_t op, int64_t n, const wm_launch_t *cfg);

/* Autotuners: time every candidate configuration on the caller's inputs
 * (one warm-up, median of 10 runs by HIP events on `stream`), install the
 * fastest for this size bucket, and return it with its median time in
 * microseconds (best / best_us, host, may be NULL).  They write the op's
 * outputs as a side effect and synchronise `stream`.  Arguments as for the
 * corresponding call; wm_autotune_grad takes op = WM_OP_VJP or
 * WM_OP_LOSS_GRAD and `w` = dL/dT or the measured times.  The batched tuner
 * times one calibration step per candidate in the workspace without
 * touching the caller's parameter sets. */
int32_t wm_autotune_predict(const wm_desc_t *desc, const wm_params_t *params, float *T,
                            int32_t *occ, void *stream, wm_launch_t *best, double *best_us);
int32_t wm_autotune_grad(int32_t op, const wm_desc_t *desc, const float *w,
                         const wm_params_t *params, double *out, void *ws, size_t ws_bytes,
                         void *stream, wm_launch_t *best, double *best_us);
int32_t wm_autotune_select_tile(const wm_shapes_t *shapes, const int32_t *cand_off,
                                const uint32_t *cand_code, int64_t n_cand,
                                const wm_params_t *params, int32_t *best_idx, double *best_cost,
                                uint8_t *near_tie, void *stream, wm_launch_t *best,
                                double *best_us);
/* op = WM_OP_PREDICT_APPS (writes T_app [n_apps]; measured, out, ws
 * unused) or WM_OP_APPS_LOSS_GRAD (writes out [33]; needs measured and a
 * wm_apps_workspace_bytes() workspace; T_app unused).  Tunes the application
 * sweep; the row gradient sweep keeps the WM_OP_VJP configuration. */
int32_t wm_autotune_apps(int32_t op, const wm_desc_t *desc, const wm_segs_t *segs,
                         const float *measured, const wm_params_t *params,
                         const wm_segparams_t *segp, float *T_app, double *out, void *ws,
                         size_t ws_bytes, void *stream, wm_launch_t *best, double *best_us);
int32_t wm_autotune_batched(int32_t n_sets, const wm_desc_t *sets, const float *const *measured,
                            const wm_params_t *p0, const wm_calib_opts_t *opts, void *ws,
                            size_t ws_bytes, void *stream, wm_launch_t *best, double *best_us);

#ifdef __cplusplus
}
#endif

#endif /* WAVEMODEL_H */
