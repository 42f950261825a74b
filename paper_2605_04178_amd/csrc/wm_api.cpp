// wm_api.cpp -- the C ABI of libwavemodel.so (include/wavemodel.h): host-side
// validation, parameter-set images, workspace carving, launches and the
// HIP-graph capture of the calibration loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/wavemodel.h"
#include "bw_launch.hpp"
#include "wm_launch.hpp"

using namespace wm;

namespace {

thread_local int32_t g_last_hip = 0;

int32_t hip_fail(hipError_t e)
{
    g_last_hip = (int32_t)e;
    return WM_EHIP;
}

#define WM_HIP(call)                                  \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_);    \
    } while (0)

bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2(int64_t x)
{
    int r = 0;
    while ((1ll << r) < x) ++r;
    return r;
}
bool fin(double x) { return std::isfinite(x); }
bool f32_exact(double x) { return (double)(float)x == x; }
bool f32_ok(double x) { return std::isfinite((float)x); }
bool f32_pos(double x) { return (float)x > 0.0f && std::isfinite((float)x); }

bool params_ok(const wm_params_t* p)
{
    if (!p) return false;
    if (p->n_levels != 3 && p->n_levels != 4) return false;
    if (p->n_cu < 1 || p->n_cu > 65536) return false;
    if (p->n_simd < 1 || p->n_simd > 16) return false;
    if (p->wave != 32 && p->wave != 64) return false;
    if (p->vgpr_simd < 1 || p->vgpr_simd > 65536) return false;
    if (!pow2(p->vgpr_gran) || p->vgpr_gran > 65536) return false;
    if (p->waves_simd < 1 || p->waves_simd > 64) return false;
    if (p->lds_cu < 0 || p->lds_cu > (1 << 24)) return false;
    if (!pow2(p->lds_gran) || p->lds_gran > (1 << 20)) return false;
    if (p->bytes_inflight_wave < 1 || p->bytes_inflight_wave > (1 << 30)) return false;
    if (p->mwp < 0 || p->cwp < 0) return false;
    if (p->combine != 0 && p->combine != 1) return false;
    if (!(fin(p->f_clk) && p->f_clk > 0.0 && f32_pos(1.0 / p->f_clk))) return false;
    if (!(fin(p->w_lo_mib) && fin(p->c_llc_mib) && p->w_lo_mib >= 0.0 &&
          p->w_lo_mib < p->c_llc_mib && f32_exact(p->w_lo_mib) && f32_exact(p->c_llc_mib)))
        return false;
    const double* th = p->theta;
    for (int j = 0; j < WM_N_THETA; ++j)
        if (!fin(th[j])) return false;
    const bool L4 = p->n_levels == 4;
    for (int l = 0; l < 4; ++l) {
        if (l == 2 && !L4) continue;
        if (!(th[l] > 0.0 && f32_pos(th[l]))) return false;
        if (!(th[4 + l] >= 0.0 && f32_ok(th[4 + l] / p->f_clk))) return false;
    }
    for (int t = 0; t < 5; ++t)
        if (!(th[8 + t] > 0.0 && f32_pos(1.0 / th[8 + t]))) return false;
    for (int j = 13; j < 20; ++j)
        if (!(th[j] >= 0.0 && f32_ok(th[j]))) return false;
    if (L4 && !(th[20] > 0.0 && th[21] > 0.0 && f32_ok(th[20]) && f32_ok(th[21]))) return false;
    if (th[22] > 0.0 && !f32_pos(1.0 / th[22])) return false;
    if (!(th[23] > 0.0 && f32_ok(th[23]) && f32_ok(th[23] - th[3]))) return false;
    return true;
}

Struct make_struct(const wm_params_t* p)
{
    Struct s;
    std::memset(&s, 0, sizeof(s));
    s.n_levels = p->n_levels;
    s.n_cu = p->n_cu;
    s.n_simd = p->n_simd;
    s.wave_shift = ilog2(p->wave);
    s.vgpr_simd = p->vgpr_simd;
    s.vgpr_gran_mask = p->vgpr_gran - 1;
    s.waves_simd = p->waves_simd;
    s.lds_cu = p->lds_cu;
    s.lds_gran_mask = p->lds_gran - 1;
    s.mwp = p->mwp;
    s.cwp = p->cwp;
    s.combine = p->combine;
    s.bytes_inflight_wave = p->bytes_inflight_wave;
    s.f_clk = p->f_clk;
    s.w_lo_mib = p->w_lo_mib;
    s.c_llc_mib = p->c_llc_mib;
    return s;
}

Set make_set(const wm_params_t* p)
{
    Set S;
    std::memset(&S, 0, sizeof(S));
    S.st = make_struct(p);
    make_const<float>(p->theta, S.st, S.cf);
    make_const<double>(p->theta, S.st, S.cd);
    return S;
}

bool desc_ok(const wm_desc_t* d)
{
    if (!d || d->n < 0) return false;
    if (d->n == 0) return true;
    const void* ptrs[12] = {d->F, d->B, d->r1, d->r2, d->r3, d->K, d->u, d->W,
                            d->vgpr, d->lds, d->gpack, d->grid};
    for (const void* q : ptrs)
        if (!q) return false;
    return true;
}

DescPtrs ptrs_of(const wm_desc_t* d)
{
    DescPtrs p;
    p.F = d->F; p.B = d->B; p.r1 = d->r1; p.r2 = d->r2; p.r3 = d->r3; p.K = d->K; p.u = d->u;
    p.W = d->W; p.vgpr = d->vgpr; p.lds = d->lds; p.gpack = d->gpack; p.grid = d->grid;
    return p;
}

bool aligned16(const wm_desc_t* d)
{
    const void* ptrs[12] = {d->F, d->B, d->r1, d->r2, d->r3, d->K, d->u, d->W,
                            d->vgpr, d->lds, d->gpack, d->grid};
    for (const void* q : ptrs)
        if (((uintptr_t)q & 15u) != 0) return false;
    return true;
}

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

bool opts_ok(const wm_calib_opts_t* o)
{
    if (!o) return false;
    if (o->steps < 1) return false;
    if (!(fin(o->lr) && o->lr > 0.0)) return false;
    if (!(fin(o->lr_final) && o->lr_final >= 0.0)) return false;
    if (!(o->beta1 >= 0.0 && o->beta1 < 1.0 && o->beta2 >= 0.0 && o->beta2 < 1.0)) return false;
    if (!(fin(o->eps) && o->eps > 0.0)) return false;
    if ((o->free_mask >> WM_N_THETA) != 0u) return false;
    // boxes: finite, non-negative, lo <= hi where both are set
    for (int j = 0; j < WM_N_THETA; ++j) {
        if (!(fin(o->lo[j]) && o->lo[j] >= 0.0 && fin(o->hi[j]) && o->hi[j] >= 0.0)) return false;
        if (o->lo[j] > 0.0 && o->hi[j] > 0.0 && o->lo[j] > o->hi[j]) return false;
    }
    if ((o->order & ~3) != 0) return false;
    // an ordered group: its four slots fitted, its boxes ordered the same way
    const double inf = HUGE_VAL;
    for (int g = 0; g < 2; ++g) {
        if (!((o->order >> g) & 1)) continue;
        const int b = 4 * g;
        if (((o->free_mask >> b) & 15u) != 15u) return false;
        for (int j = b; j < b + 3; ++j) {
            const double lo0 = o->lo[j] > 0.0 ? o->lo[j] : -inf, lo1 = o->lo[j + 1] > 0.0 ? o->lo[j + 1] : -inf;
            const double hi0 = o->hi[j] > 0.0 ? o->hi[j] : inf, hi1 = o->hi[j + 1] > 0.0 ? o->hi[j + 1] : inf;
            // group 0 (bandwidths) non-increasing, group 1 (latencies) non-decreasing
            if (g == 0 ? (lo0 < lo1 || hi0 < hi1) : (lo0 > lo1 || hi0 > hi1)) return false;
        }
    }
    return true;
}

static_assert(sizeof(wm_calib_opts_t) == 56 + 2 * 8 * WM_N_THETA, "wm_calib_opts_t layout");

// The per-step Adam schedule of a run, formed on the host (one table for
// every step index, so a resumed run reads the same values).
std::vector<double> adam_table(const AdamOpts& o)
{
    std::vector<double> t((size_t)3 * (size_t)(o.steps > 0 ? o.steps : 0));
    for (int32_t k = 0; k < o.steps; ++k) adam_schedule(o, k, &t[3 * k], &t[3 * k + 1], &t[3 * k + 2]);
    return t;
}

AdamOpts adam_of(const wm_calib_opts_t* o)
{
    AdamOpts a;
    std::memset(&a, 0, sizeof(a));
    a.steps = o->steps;
    a.lr = o->lr;
    a.lr_final = o->lr_final;
    a.beta1 = o->beta1;
    a.beta2 = o->beta2;
    a.eps = o->eps;
    a.free_mask = o->free_mask;
    a.order = o->order;
    for (int j = 0; j < kTheta; ++j) {
        a.lo_log[j] = o->lo[j] > 0.0 ? std::log(o->lo[j]) : -HUGE_VAL;
        a.hi_log[j] = o->hi[j] > 0.0 ? std::log(o->hi[j]) : HUGE_VAL;
    }
    return a;
}

// the slots a parameter set may move: positive everywhere they are fitted
bool free_slots_ok(const wm_params_t* p, uint32_t mask)
{
    for (int j = 0; j < WM_N_THETA; ++j)
        if (((mask >> j) & 1u) && !(p->theta[j] > 0.0)) return false;
    return true;
}

CalibState init_state(const wm_params_t* p, uint32_t mask)
{
    CalibState s;
    std::memset(&s, 0, sizeof(s));
    for (int j = 0; j < WM_N_THETA; ++j) {
        s.theta[j] = p->theta[j];
        s.theta_ok[j] = p->theta[j];
        s.phi[j] = ((mask >> j) & 1u) ? std::log(p->theta[j]) : 0.0;
    }
    return s;
}

bool segp_ok(const wm_segparams_t* q)
{
    if (!q) return false;
    for (int c = 0; c < 4; ++c)
        if (!(fin(q->kappa[c]) && q->kappa[c] >= 0.0 && f32_ok(q->kappa[c]))) return false;
    if (!(fin(q->bw_h2d) && q->bw_h2d > 0.0 && f32_pos(1.0 / q->bw_h2d))) return false;
    if (!(fin(q->bw_d2h) && q->bw_d2h > 0.0 && f32_pos(1.0 / q->bw_d2h))) return false;
    if (!(fin(q->tau_memcpy) && q->tau_memcpy >= 0.0 && f32_ok(q->tau_memcpy))) return false;
    return true;
}

// segment rows parallel to n descriptor rows
bool segs_ok(const wm_segs_t* s, int64_t n)
{
    if (!s || s->n_apps < 0 || n > 0x7fffffffll) return false;
    if (s->n_apps == 0) return n == 0;
    if (!s->app_off) return false;
    if (n > 0 && (!s->n_exec || !s->n_kern || !s->cls || !s->h2d || !s->d2h)) return false;
    return true;
}

SegSet make_segset(const wm_segparams_t* q)
{
    SegSet Q;
    std::memset(&Q, 0, sizeof(Q));
    for (int c = 0; c < 4; ++c) {
        Q.f.kappa[c] = (float)q->kappa[c];
        Q.d.kappa[c] = q->kappa[c];
    }
    Q.d.inv_bw_h2d = 1.0 / q->bw_h2d;
    Q.d.inv_bw_d2h = 1.0 / q->bw_d2h;
    Q.d.tau = q->tau_memcpy;
    Q.f.inv_bw_h2d = (float)Q.d.inv_bw_h2d;
    Q.f.inv_bw_d2h = (float)Q.d.inv_bw_d2h;
    Q.f.tau = (float)q->tau_memcpy;
    Q.inv_bw2_h2d = Q.d.inv_bw_h2d * Q.d.inv_bw_h2d;
    Q.inv_bw2_d2h = Q.d.inv_bw_d2h * Q.d.inv_bw_d2h;
    return Q;
}

SegPtrs segptrs_of(const wm_segs_t* s)
{
    SegPtrs p;
    p.off = s->app_off;
    p.n_exec = s->n_exec;
    p.n_kern = s->n_kern;
    p.cls = s->cls;
    p.h2d = s->h2d;
    p.d2h = s->d2h;
    return p;
}

// fusion-planning workspace: candidate costs, the redo queue, run lengths,
// per-row coverage bytes, the queue's length (last)
struct PlanWs {
    size_t cost, redo, cut, cov, n_redo, total;
};

PlanWs plan_ws(int64_t n, int32_t R)
{
    PlanWs W;
    size_t off = 0;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    W.cost = off;
    off += up256(sizeof(double) * nn * (size_t)R);
    W.redo = off;
    off += up256(sizeof(int64_t) * nn);
    W.cut = off;
    off += up256(nn);
    W.cov = off;
    off += up256(nn);
    W.n_redo = off;
    off += 256;
    W.total = off;
    return W;
}

constexpr size_t kFitMultWs = sizeof(double) * 4 * (size_t)kFitMultMaxBlocks;

// ---- Blackwell family helpers ----
bool bw_params_ok(const wm_bw_params_t* p)
{
    if (!p) return false;
    if (p->n_sm < 1 || p->n_sm > 65536 || p->max_cta < 1 || p->max_cta > 64) return false;
    if (p->tmem_bytes < 1 || p->tmem_bytes >= (1ll << 30)) return false;
    if (!(fin(p->f_clk) && p->f_clk > 0.0 && f32_pos(1.0 / p->f_clk))) return false;
    const double* th = p->theta;
    for (int j = 0; j < WM_N_THETA; ++j)
        if (!fin(th[j])) return false;
    const int pos[] = {0, 1, 3, 4, 5, 6, 7, 8, 10, 13, 14, 15, 18, 23};
    for (int j : pos)
        if (!(th[j] > 0.0 && f32_pos(th[j]) && f32_pos(1.0 / th[j]))) return false;
    const int nonneg[] = {2, 9, 11, 12, 16, 17, 19, 20, 21, 22};
    for (int j : nonneg)
        if (!(th[j] >= 0.0 && f32_ok(th[j]) && f32_ok(th[j] / p->f_clk))) return false;
    return true;
}

BwSet make_bw_set(const wm_bw_params_t* p)
{
    BwSet S;
    std::memset(&S, 0, sizeof(S));
    S.st.n_sm = p->n_sm;
    S.st.max_cta = p->max_cta;
    S.st.tmem_bytes = p->tmem_bytes;
    S.st.f_clk = p->f_clk;
    make_bw_const<float>(p->theta, S.st, S.cf);
    make_bw_const<double>(p->theta, S.st, S.cd);
    return S;
}

bool bw_desc_ok(const wm_bw_desc_t* d)
{
    if (!d || d->n < 0) return false;
    if (d->n == 0) return true;
    return d->bM && d->bN && d->bK && d->G && d->flags && d->Kt && d->CR && d->ob;
}

BwDescPtrs bw_ptrs_of(const wm_bw_desc_t* d)
{
    BwDescPtrs p;
    p.bM = d->bM; p.bN = d->bN; p.bK = d->bK; p.G = d->G; p.flags = d->flags;
    p.Kt = d->Kt; p.CR = d->CR; p.ob = d->ob;
    return p;
}

// calibration workspace layout
// gradient-sweep workspace: partial rows, then redo-flag words
struct GradWs {
    GradLayout g;
    size_t partials, flags, total;
};

GradWs grad_ws(int64_t n)
{
    GradWs W;
    W.g = grad_layout(n);
    W.partials = 0;
    W.flags = up256(sizeof(double) * kAcc * (size_t)(W.g.nb + W.g.nb2));
    W.total = W.flags + up256(sizeof(uint64_t) * (size_t)(W.g.nwords > 0 ? W.g.nwords : 1));
    return W;
}

// application loss-gradient workspace: row weights, application rows,
// application flag words, then the gradient sweep's partials and flags
struct AppsWs {
    size_t rows, aflags, lflags, rflags, wrow, total;
};

AppsWs apps_ws(int64_t n, int64_t n_apps)
{
    AppsWs W;
    size_t off = 0;
    W.rows = off;
    off += up256(sizeof(double) * kAppRow * (size_t)(kAppsMaxBlocks + kAppsLongBlocks + kRedoMaxBlocks));
    const size_t awords = (size_t)((n_apps + 63) / 64 > 0 ? (n_apps + 63) / 64 : 1);
    W.aflags = off;
    off += up256(sizeof(uint64_t) * awords);
    W.lflags = off;
    off += up256(sizeof(uint64_t) * awords);
    W.rflags = off;
    off += up256(sizeof(uint64_t) * (size_t)((n + 63) / 64 > 0 ? (n + 63) / 64 : 1));
    W.wrow = off;
    off += up256(sizeof(float) * (size_t)(n > 0 ? n : 1));
    W.total = off;
    return W;
}

struct CalibLayout {
    size_t set, state, hist, sched, grad, total;
    GradWs g;
};

CalibLayout calib_layout(int64_t n, int32_t steps, size_t set_bytes = sizeof(Set))
{
    CalibLayout L;
    L.g = grad_ws(n);
    const size_t ns = (size_t)(steps > 0 ? steps : 1);
    size_t off = 0;
    L.set = off;
    off += up256(set_bytes);
    L.state = off;
    off += up256(sizeof(CalibState));
    L.hist = off;
    off += up256(sizeof(double) * ns);
    L.sched = off;
    off += up256(3 * sizeof(double) * ns);
    L.grad = off;
    off += L.g.total;
    L.total = off;
    return L;
}

constexpr int kBatchMaxBlocks = kGradMaxBlocks;

struct BatchLayout {
    size_t sets, states, opts, descs, meas, items, setn, flagoff, hist, partials, flags, total;
    int nb, nb2, max_items;
    int64_t max_words;
};

BatchLayout batch_layout(int64_t n_total, int32_t n_sets, int32_t steps)
{
    BatchLayout L;
    L.max_items = (int)(n_total / kMinChunk + n_sets + 1);
    L.nb = L.max_items < kBatchMaxBlocks ? L.max_items : kBatchMaxBlocks;
    L.nb2 = grad_layout(n_total).nb2;
    L.max_words = n_total / 64 + n_sets + 1;
    size_t off = 0;
    L.sets = off;
    off += up256(sizeof(Set) * n_sets);
    L.states = off;
    off += up256(sizeof(CalibState) * n_sets);
    L.opts = off;
    off += up256(sizeof(AdamOpts) * n_sets);
    L.descs = off;
    off += up256(sizeof(DescPtrs) * n_sets);
    L.meas = off;
    off += up256(sizeof(float*) * n_sets);
    L.items = off;
    off += up256(sizeof(int32_t) * (size_t)(n_sets + 1));
    L.setn = off;
    off += up256(sizeof(int64_t) * n_sets);
    L.flagoff = off;
    off += up256(sizeof(int64_t) * n_sets);
    L.hist = off;
    off += up256(sizeof(double) * (size_t)n_sets * (size_t)(steps > 0 ? steps : 1));
    L.partials = off;
    off += up256(sizeof(double) * kAcc * (size_t)n_sets * (size_t)(L.nb + L.nb2));
    L.flags = off;
    off += up256(sizeof(uint64_t) * (size_t)L.max_words);
    L.total = off;
    return L;
}

bool ws_ok(void* ws, size_t have, size_t need)
{
    if (need == 0) return true;
    return ws && have >= need && ((uintptr_t)ws & 255u) == 0;
}

// Capture `chunk` steps of a calibration loop on `stream` into an executable
// graph.  `enqueue_step` records one step's launches.
template <typename F>
int32_t capture_steps(hipStream_t stream, int chunk, F enqueue_step, hipGraphExec_t* exec)
{
    hipGraph_t graph = nullptr;
    WM_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int i = 0; i < chunk && err == hipSuccess; ++i) err = enqueue_step();
    hipError_t e2 = hipStreamEndCapture(stream, &graph);
    if (err != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(err);
    }
    if (e2 != hipSuccess) return hip_fail(e2);
    hipError_t e3 = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return hip_fail(e3);
    return WM_OK;
}

// Run `steps` steps as replays of captured graphs of up to kGraphChunk steps.
constexpr int kGraphChunk = 50;

template <typename F>
int32_t run_steps(hipStream_t stream, int steps, F enqueue_step)
{
    const int chunk = steps < kGraphChunk ? steps : kGraphChunk;
    const int full = steps / chunk, rem = steps % chunk;
    hipGraphExec_t g_full = nullptr, g_rem = nullptr;
    int32_t rc = capture_steps(stream, chunk, enqueue_step, &g_full);
    if (rc != WM_OK) return rc;
    if (rem > 0) {
        rc = capture_steps(stream, rem, enqueue_step, &g_rem);
        if (rc != WM_OK) {
            (void)hipGraphExecDestroy(g_full);
            return rc;
        }
    }
    hipError_t e = hipSuccess;
    for (int i = 0; i < full && e == hipSuccess; ++i) e = hipGraphLaunch(g_full, stream);
    if (e == hipSuccess && g_rem) e = hipGraphLaunch(g_rem, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipGraphExecDestroy(g_full);
    if (g_rem) (void)hipGraphExecDestroy(g_rem);
    if (e != hipSuccess) return hip_fail(e);
    return WM_OK;
}

// A capturable stream: the caller's, or for the null stream a library stream
// created once per device (after draining the null stream's earlier work).
std::mutex g_stream_mu;
std::vector<hipStream_t> g_own_streams;

int32_t capture_stream(void* user, hipStream_t* out)
{
    if (user) {
        *out = (hipStream_t)user;
        return WM_OK;
    }
    int dev = 0;
    WM_HIP(hipGetDevice(&dev));
    WM_HIP(hipStreamSynchronize(nullptr));
    std::lock_guard<std::mutex> lk(g_stream_mu);
    if ((int)g_own_streams.size() <= dev) g_own_streams.resize(dev + 1, nullptr);
    if (!g_own_streams[dev]) WM_HIP(hipStreamCreateWithFlags(&g_own_streams[dev], hipStreamNonBlocking));
    *out = g_own_streams[dev];
    return WM_OK;
}


// Device images of a multi-set calibration in a workspace: the per-set
// parameter images, Adam states, options, descriptor and measurement pointer
// tables, and each set's first item (items of `chunk` descriptors, set by
// set).  step() enqueues the sweep, the float64 pass and one
// reduce-and-Adam launch.
struct BatchRun {
    int n_sets = 0, steps = 0, n_items = 0, nb = 0, nb2 = 0;
    int64_t chunk = 0;
    Set* S_dev = nullptr;
    CalibState* st_dev = nullptr;
    AdamOpts* o_dev = nullptr;
    DescPtrs* d_dev = nullptr;
    const float** m_dev = nullptr;
    int32_t* io_dev = nullptr;
    int64_t* n_dev = nullptr;
    int64_t* fo_dev = nullptr;
    double* hist_dev = nullptr;
    double* part_dev = nullptr;
    uint64_t* flags_dev = nullptr;
    hipStream_t s = nullptr;

    hipError_t step() const
    {
        hipError_t e = launch_grad_batched(d_dev, m_dev, S_dev, io_dev, n_items, chunk, n_sets,
                                           n_dev, fo_dev, flags_dev, part_dev, nb, nb2, s);
        if (e != hipSuccess) return e;
        return launch_adam_batched(part_dev + (int64_t)nb * n_sets * kAcc, nb2, n_sets, st_dev,
                                   o_dev, S_dev, steps, hist_dev, s);
    }
};

int32_t batch_prepare(int32_t n_sets, const wm_desc_t* sets, const float* const* measured,
                      const wm_params_t* p0, const wm_calib_opts_t* opts, const BatchLayout& L,
                      const LaunchCfg& cfg, void* ws, hipStream_t s, BatchRun* run)
{
    std::vector<Set> Sh((size_t)n_sets);
    std::vector<CalibState> sth((size_t)n_sets);
    std::vector<AdamOpts> oh((size_t)n_sets);
    std::vector<DescPtrs> dh((size_t)n_sets);
    std::vector<const float*> mh((size_t)n_sets);
    std::vector<int64_t> nh((size_t)n_sets), foh((size_t)n_sets);
    std::vector<int32_t> ioh((size_t)n_sets + 1);
    int64_t words = 0, n_items = 0;
    const int64_t chunk = cfg.chunk;
    if (chunk < 64 || chunk % 64 != 0) return WM_EINVAL;
    for (int k = 0; k < n_sets; ++k) {
        nh[k] = sets[k].n;
        foh[k] = words;
        words += (sets[k].n + 63) / 64;
        Sh[k] = make_set(&p0[k]);
        sth[k] = init_state(&p0[k], opts[k].free_mask);
        oh[k] = adam_of(&opts[k]);
        dh[k] = ptrs_of(&sets[k]);
        mh[k] = measured[k];
        ioh[k] = (int32_t)n_items;
        n_items += (sets[k].n + chunk - 1) / chunk;
        if (n_items > L.max_items) return WM_EINVAL;
    }
    ioh[n_sets] = (int32_t)n_items;
    char* base = (char*)ws;
    run->n_sets = n_sets;
    run->steps = opts[0].steps;
    run->n_items = (int)n_items;
    run->chunk = chunk;
    run->nb = batched_grid(run->n_items, cfg.grid_mult);
    int64_t max_words = 0;
    for (int k = 0; k < n_sets; ++k)
        max_words = std::max<int64_t>(max_words, (sets[k].n + 63) / 64);
    run->nb2 = batched_redo_grid(n_sets, max_words, L.nb2);
    run->S_dev = (Set*)(base + L.sets);
    run->st_dev = (CalibState*)(base + L.states);
    run->o_dev = (AdamOpts*)(base + L.opts);
    run->d_dev = (DescPtrs*)(base + L.descs);
    run->m_dev = (const float**)(base + L.meas);
    run->io_dev = (int32_t*)(base + L.items);
    run->n_dev = (int64_t*)(base + L.setn);
    run->fo_dev = (int64_t*)(base + L.flagoff);
    run->hist_dev = (double*)(base + L.hist);
    run->part_dev = (double*)(base + L.partials);
    run->flags_dev = (uint64_t*)(base + L.flags);
    run->s = s;
    WM_HIP(hipMemcpyAsync(run->S_dev, Sh.data(), sizeof(Set) * n_sets, hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(run->st_dev, sth.data(), sizeof(CalibState) * n_sets, hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(run->o_dev, oh.data(), sizeof(AdamOpts) * n_sets, hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(run->d_dev, dh.data(), sizeof(DescPtrs) * n_sets, hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(run->m_dev, mh.data(), sizeof(float*) * n_sets, hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(run->n_dev, nh.data(), sizeof(int64_t) * n_sets, hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(run->fo_dev, foh.data(), sizeof(int64_t) * n_sets, hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(run->io_dev, ioh.data(), sizeof(int32_t) * (n_sets + 1),
                          hipMemcpyHostToDevice, s));
    WM_HIP(hipStreamSynchronize(s));  // the host images above go out of scope
    return WM_OK;
}

bool batch_args_ok(int32_t n_sets, const wm_desc_t* sets, const float* const* measured,
                   const wm_params_t* p0, const wm_calib_opts_t* opts, int64_t* n_total)
{
    if (n_sets < 1 || n_sets > kMaxSets || !sets || !measured || !p0 || !opts) return false;
    int64_t t = 0;
    for (int k = 0; k < n_sets; ++k) {
        if (!desc_ok(&sets[k]) || (sets[k].n > 0 && !measured[k]) || !params_ok(&p0[k]) ||
            !opts_ok(&opts[k]))
            return false;
        if (!free_slots_ok(&p0[k], opts[k].free_mask)) return false;
        if (opts[k].steps != opts[0].steps) return false;
        t += sets[k].n;
    }
    *n_total = t;
    return true;
}

// median of `reps` event-timed runs (after one warm-up), microseconds
template <typename F>
int32_t time_median(hipStream_t s, int reps, F run, double* us)
{
    hipEvent_t a = nullptr, b = nullptr;
    WM_HIP(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(e);
    }
    std::vector<float> t;
    e = run();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = hipEventRecord(a, s);
        if (e == hipSuccess) e = run();
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e);
    std::sort(t.begin(), t.end());
    *us = 1e3 * (double)t[t.size() / 2];
    return WM_OK;
}

wm_launch_t to_pub(const LaunchCfg& c)
{
    wm_launch_t o;
    o.block = c.block;
    o.per_thread = c.vec;
    o.grid_mult = c.grid_mult;
    o.chunk = c.chunk;
    return o;
}

LaunchCfg from_pub(const wm_launch_t& o)
{
    LaunchCfg c;
    c.block = o.block;
    c.vec = o.per_thread;
    c.grid_mult = o.grid_mult;
    c.chunk = o.chunk;
    return c;
}

// try every candidate, keep the fastest (ties: first), record it
template <typename F>
int32_t tune_over(int op, int64_t n, const std::vector<LaunchCfg>& cands, hipStream_t s, int reps,
                  F run_with, wm_launch_t* best, double* best_us)
{
    double bu = 1e300;
    LaunchCfg bc = cands.front();
    for (const LaunchCfg& c : cands) {
        double us = 0.0;
        int32_t rc = time_median(s, reps, [&]() { return run_with(c); }, &us);
        if (rc != WM_OK) return rc;
        if (us < bu) {
            bu = us;
            bc = c;
        }
    }
    store_cfg(op, n, bc, bu, true);
    if (best) *best = to_pub(bc);
    if (best_us) *best_us = bu;
    return WM_OK;
}

std::vector<LaunchCfg> candidates(int op)
{
    std::vector<LaunchCfg> v;
    const int blocks[4] = {64, 128, 256, 512};
    LaunchCfg c = default_cfg(op);
    if (op == kOpPredict) {
        const int vecs[4] = {1, 2, 4, 8};
        for (int b : blocks)
            for (int vv : vecs) {
                c.block = b;
                c.vec = vv;
                v.push_back(c);
            }
    } else if (op == kOpCalibrateBatched) {
        for (int ch = (int)kMinChunk; ch <= 65536; ch *= 2)
            for (int gm = 1; gm <= 2; ++gm) {
                c.chunk = ch;
                c.grid_mult = gm;
                v.push_back(c);
            }
    } else {
        for (int b : blocks)
            for (int gm = 1; gm <= 4; gm *= 2) {
                c.block = b;
                c.grid_mult = gm;
                v.push_back(c);
            }
    }
    // the default first, so it wins ties
    const LaunchCfg d = default_cfg(op);
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i].block == d.block && v[i].vec == d.vec && v[i].grid_mult == d.grid_mult &&
            v[i].chunk == d.chunk) {
            std::swap(v[0], v[i]);
            break;
        }
    return v;
}

}  // namespace

// ===========================================================================
int32_t wm::record_hip_error(hipError_t e) { return hip_fail(e); }

bool wm::grad_args_ok(const wm_desc_t* desc, const float* w, const wm_params_t* params, const double* out)
{
    if (!desc_ok(desc) || !params_ok(params) || !out) return false;
    return !(desc->n > 0 && !w);
}

extern "C" {

const char* wm_strerror(int32_t s)
{
    switch (s) {
    case WM_OK: return "ok";
    case WM_EINVAL: return "invalid argument";
    case WM_EWORKSPACE: return "workspace missing, too small or misaligned";
    case WM_EHIP: return "HIP runtime error";
    case WM_EDIVERGED: return "calibration diverged";
    case WM_ETOOLARGE: return "input larger than the fixed scratch allows";
    default: return "unknown status";
    }
}

int32_t wm_last_hip_error(void) { return g_last_hip; }

int32_t wm_validate_params(const wm_params_t* p) { return params_ok(p) ? WM_OK : WM_EINVAL; }

size_t wm_workspace_bytes(int32_t op, int64_t n, int32_t n_sets, int32_t steps)
{
    if (n < 0) return 0;
    switch (op) {
    case WM_OP_VJP:
    case WM_OP_LOSS_GRAD:
        return grad_ws(n).total;
    case WM_OP_CALIBRATE:
        if (steps < 1) return 0;
        return calib_layout(n, steps).total;
    case WM_OP_CALIBRATE_BATCHED:
        if (steps < 1 || n_sets < 1 || n_sets > kMaxSets) return 0;
        return batch_layout(n, n_sets, steps).total;
    case WM_OP_FIT_MULTIPLIERS:
        return kFitMultWs;
    default:
        return 0;
    }
}

int32_t wm_bw_validate_params(const wm_bw_params_t* p) { return bw_params_ok(p) ? WM_OK : WM_EINVAL; }

size_t wm_bw_workspace_bytes(int32_t op, int64_t n, int32_t steps)
{
    if (n < 0) return 0;
    if (op == WM_BW_OP_GRAD) return grad_ws(n).total;
    if (op == WM_BW_OP_CALIBRATE && steps >= 1) return calib_layout(n, steps, sizeof(BwSet)).total;
    return 0;
}

int32_t wm_bw_predict(const wm_bw_desc_t* desc, const wm_bw_params_t* params, float* T, int32_t* cta,
                      void* stream)
{
    if (!bw_desc_ok(desc) || !bw_params_ok(params)) return WM_EINVAL;
    if (desc->n == 0) return WM_OK;
    if (!T) return WM_EINVAL;
    const BwSet S = make_bw_set(params);
    WM_HIP(launch_bw_predict(bw_ptrs_of(desc), desc->n, S, T, cta, default_cfg(kOpPredict),
                             (hipStream_t)stream));
    return WM_OK;
}

static int32_t bw_grad_common(int mode, const wm_bw_desc_t* desc, const float* w,
                              const wm_bw_params_t* params, double* out, void* ws, size_t ws_bytes,
                              void* stream)
{
    if (!bw_desc_ok(desc) || !bw_params_ok(params) || !out) return WM_EINVAL;
    if (desc->n > 0 && !w) return WM_EINVAL;
    const GradWs W = grad_ws(desc->n);
    if (!ws_ok(ws, ws_bytes, W.total)) return WM_EWORKSPACE;
    const BwSet S = make_bw_set(params);
    char* base = (char*)ws;
    const LaunchCfg cfg = launch_cfg(mode == 1 ? kOpLossGrad : kOpVjp, desc->n);
    WM_HIP(launch_bw_grad(mode, bw_ptrs_of(desc), desc->n, w, S, nullptr, (double*)(base + W.partials),
                          (uint64_t*)(base + W.flags), W.g, cfg, out, (hipStream_t)stream));
    return WM_OK;
}

int32_t wm_bw_predict_vjp(const wm_bw_desc_t* desc, const wm_bw_params_t* params, const float* dL_dT,
                          double* dL_dtheta, void* ws, size_t ws_bytes, void* stream)
{
    return bw_grad_common(0, desc, dL_dT, params, dL_dtheta, ws, ws_bytes, stream);
}

int32_t wm_bw_loss_grad(const wm_bw_desc_t* desc, const float* measured, const wm_bw_params_t* params,
                        double* out, void* ws, size_t ws_bytes, void* stream)
{
    return bw_grad_common(1, desc, measured, params, out, ws, ws_bytes, stream);
}

int32_t wm_bw_calibrate(const wm_bw_desc_t* desc, const float* measured, const wm_bw_params_t* p0,
                        const wm_calib_opts_t* opts, wm_bw_params_t* p_out, double* loss_hist,
                        void* ws, size_t ws_bytes, void* stream)
{
    // the level orderings name CDNA slots
    if (!bw_desc_ok(desc) || (desc->n > 0 && !measured) || !bw_params_ok(p0) || !opts_ok(opts) ||
        opts->order != 0 || !p_out)
        return WM_EINVAL;
    for (int j = 0; j < WM_N_THETA; ++j)
        if (((opts->free_mask >> j) & 1u) && !(p0->theta[j] > 0.0)) return WM_EINVAL;
    const CalibLayout L = calib_layout(desc->n, opts->steps, sizeof(BwSet));
    if (!ws_ok(ws, ws_bytes, L.total)) return WM_EWORKSPACE;
    hipStream_t s = nullptr;
    int32_t rc = capture_stream(stream, &s);
    if (rc != WM_OK) return rc;
    char* base = (char*)ws;
    BwSet* S_dev = (BwSet*)(base + L.set);
    CalibState* st_dev = (CalibState*)(base + L.state);
    double* hist_dev = (double*)(base + L.hist);
    double* part_dev = (double*)(base + L.grad + L.g.partials);
    uint64_t* flags_dev = (uint64_t*)(base + L.grad + L.g.flags);
    const BwSet S = make_bw_set(p0);
    CalibState st0;
    std::memset(&st0, 0, sizeof(st0));
    for (int j = 0; j < WM_N_THETA; ++j) {
        st0.theta[j] = p0->theta[j];
        st0.theta_ok[j] = p0->theta[j];
        st0.phi[j] = ((opts->free_mask >> j) & 1u) ? std::log(p0->theta[j]) : 0.0;
    }
    AdamOpts ao = adam_of(opts);
    const std::vector<double> sched = adam_table(ao);
    ao.sched = (const double*)(base + L.sched);
    WM_HIP(hipMemcpyAsync(S_dev, &S, sizeof(S), hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(st_dev, &st0, sizeof(st0), hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(base + L.sched, sched.data(), sizeof(double) * sched.size(),
                          hipMemcpyHostToDevice, s));
    WM_HIP(hipStreamSynchronize(s));
    const BwDescPtrs dp = bw_ptrs_of(desc);
    const int64_t n = desc->n;
    const GradLayout G = L.g.g;
    const LaunchCfg cfg = launch_cfg(kOpLossGrad, n);
    double* rows2_dev = part_dev + (int64_t)bw_grad_grid(1, true, n, cfg) * kAcc;
    auto step = [&]() -> hipError_t {
        hipError_t e = launch_bw_grad(1, dp, n, measured, S, S_dev, part_dev, flags_dev, G, cfg,
                                      nullptr, s);
        if (e != hipSuccess) return e;
        return launch_bw_adam(rows2_dev, G.nb2, st_dev, ao, S_dev, hist_dev, s);
    };
    rc = run_steps(s, opts->steps, step);
    if (rc != WM_OK) return rc;
    CalibState fin_st;
    WM_HIP(hipMemcpyAsync(&fin_st, st_dev, sizeof(fin_st), hipMemcpyDeviceToHost, s));
    std::vector<double> hist((size_t)opts->steps);
    WM_HIP(hipMemcpyAsync(hist.data(), hist_dev, sizeof(double) * opts->steps, hipMemcpyDeviceToHost, s));
    WM_HIP(hipStreamSynchronize(s));
    *p_out = *p0;
    const double* th = fin_st.diverged ? fin_st.theta_ok : fin_st.theta;
    for (int j = 0; j < WM_N_THETA; ++j) p_out->theta[j] = th[j];
    if (loss_hist) std::memcpy(loss_hist, hist.data(), sizeof(double) * opts->steps);
    return fin_st.diverged ? WM_EDIVERGED : WM_OK;
}

size_t wm_plan_workspace_bytes(int64_t n, int32_t R)
{
    if (n < 0 || R < 1 || R > kPlanMaxRun) return 0;
    return plan_ws(n, R).total;
}

int32_t wm_fit_multipliers(const float* T, const float* measured, const int32_t* group_off,
                           int64_t n_groups, int64_t n, const uint8_t* train, double* mult,
                           float* T_scaled, double* stats, void* ws, size_t ws_bytes, void* stream)
{
    if (n < 0 || n_groups < 0 || !stats) return WM_EINVAL;
    if (n > 0 && (!T || !measured || !train || !T_scaled)) return WM_EINVAL;
    if (n_groups > 0 && (!group_off || !mult)) return WM_EINVAL;
    if (!ws_ok(ws, ws_bytes, kFitMultWs)) return WM_EWORKSPACE;
    WM_HIP(launch_fit_multipliers(T, measured, group_off, n_groups, n, train, mult, T_scaled,
                                  (double*)ws, stats, (hipStream_t)stream));
    return WM_OK;
}

int32_t wm_plan_fusion(const wm_desc_t* desc, const float* edge, const int32_t* chain_off,
                       int64_t n_chains, int32_t R, const wm_params_t* params, double* total,
                       double* unfused, uint8_t* start, void* ws, size_t ws_bytes, void* stream)
{
    if (!desc_ok(desc) || !params_ok(params) || n_chains < 0 || R < 1 || R > kPlanMaxRun)
        return WM_EINVAL;
    if (n_chains == 0) return WM_OK;
    if (!chain_off || !total || !unfused) return WM_EINVAL;
    if (desc->n > 0 && (!edge || !start)) return WM_EINVAL;
    const PlanWs W = plan_ws(desc->n, R);
    if (!ws_ok(ws, ws_bytes, W.total)) return WM_EWORKSPACE;
    char* base = (char*)ws;
    const Set S = make_set(params);
    PlanBufs wb;
    wb.cost = (double*)(base + W.cost);
    wb.redo = (int64_t*)(base + W.redo);
    wb.cut = (uint8_t*)(base + W.cut);
    wb.cov = (uint8_t*)(base + W.cov);
    wb.n_redo = (uint32_t*)(base + W.n_redo);
    WM_HIP(launch_plan_fusion(ptrs_of(desc), edge, chain_off, n_chains, desc->n, R, S,
                              params->theta + 8, wb, total, unfused, start, (hipStream_t)stream));
    return WM_OK;
}

size_t wm_apps_workspace_bytes(int64_t n, int64_t n_apps)
{
    if (n < 0 || n_apps < 0) return 0;
    return apps_ws(n, n_apps).total;
}

int32_t wm_predict(const wm_desc_t* desc, const wm_params_t* params, float* T, int32_t* occ,
                   void* stream)
{
    if (!desc_ok(desc) || !params_ok(params)) return WM_EINVAL;
    if (desc->n == 0) return WM_OK;
    if (!T) return WM_EINVAL;
    const bool vec = aligned16(desc) && ((uintptr_t)T & 15u) == 0 && ((uintptr_t)occ & 15u) == 0;
    const Set S = make_set(params);
    WM_HIP(launch_predict(ptrs_of(desc), desc->n, S, T, occ, vec, launch_cfg(kOpPredict, desc->n),
                          (hipStream_t)stream));
    return WM_OK;
}

int32_t wm_roofline(const wm_desc_t* desc, const wm_params_t* params, float* T, void* stream)
{
    if (!desc_ok(desc) || !params_ok(params)) return WM_EINVAL;
    if (desc->n == 0) return WM_OK;
    if (!T) return WM_EINVAL;
    const Set S = make_set(params);
    WM_HIP(launch_roofline(ptrs_of(desc), desc->n, S, T, (hipStream_t)stream));
    return WM_OK;
}

static int32_t grad_common(int mode, const wm_desc_t* desc, const float* w, const wm_params_t* params,
                           double* out, void* ws, size_t ws_bytes, void* stream, bool exact = false)
{
    if (!wm::grad_args_ok(desc, w, params, out)) return WM_EINVAL;
    const size_t need = wm_workspace_bytes(mode == 1 ? WM_OP_LOSS_GRAD : WM_OP_VJP, desc->n, 1, 0);
    if (!ws_ok(ws, ws_bytes, need)) return WM_EWORKSPACE;
    const Set S = make_set(params);
    const GradWs W = grad_ws(desc->n);
    char* base = (char*)ws;
    // n == 0 still writes zeros through the (empty) sweep and reduction
    const LaunchCfg cfg = launch_cfg(mode == 1 ? kOpLossGrad : kOpVjp, desc->n);
    if (exact)
        WM_HIP(launch_grad_exact(mode, ptrs_of(desc), desc->n, w, S, (double*)(base + W.partials),
                                 (uint64_t*)(base + W.flags), W.g, cfg.grid_mult, out, (hipStream_t)stream));
    else
        WM_HIP(launch_grad(mode, ptrs_of(desc), desc->n, w, S, nullptr, (double*)(base + W.partials),
                           (uint64_t*)(base + W.flags), W.g, cfg, out, (hipStream_t)stream));
    return WM_OK;
}

int32_t wm_predict_vjp(const wm_desc_t* desc, const wm_params_t* params, const float* dL_dT,
                       double* dL_dtheta, void* ws, size_t ws_bytes, void* stream)
{
    return grad_common(0, desc, dL_dT, params, dL_dtheta, ws, ws_bytes, stream);
}

int32_t wm_loss_grad(const wm_desc_t* desc, const float* measured, const wm_params_t* params,
                     double* out, void* ws, size_t ws_bytes, void* stream)
{
    return grad_common(1, desc, measured, params, out, ws, ws_bytes, stream);
}

int32_t wm_predict_vjp_exact(const wm_desc_t* desc, const wm_params_t* params, const float* dL_dT,
                             double* dL_dtheta, void* ws, size_t ws_bytes, void* stream)
{
    return grad_common(0, desc, dL_dT, params, dL_dtheta, ws, ws_bytes, stream, true);
}

int32_t wm_loss_grad_exact(const wm_desc_t* desc, const float* measured, const wm_params_t* params,
                           double* out, void* ws, size_t ws_bytes, void* stream)
{
    return grad_common(1, desc, measured, params, out, ws, ws_bytes, stream, true);
}

int32_t wm_predict_apps(const wm_desc_t* desc, const wm_segs_t* segs, const wm_params_t* params,
                        const wm_segparams_t* segp, float* T_app, float* T_seg, void* stream)
{
    if (!desc_ok(desc) || !params_ok(params) || !segp_ok(segp) || !segs_ok(segs, desc->n))
        return WM_EINVAL;
    if (segs->n_apps == 0) return WM_OK;
    if (!T_app) return WM_EINVAL;
    const Set S = make_set(params);
    WM_HIP(launch_predict_apps(ptrs_of(desc), segptrs_of(segs), desc->n, segs->n_apps, S,
                               make_segset(segp), T_app, T_seg,
                               launch_cfg(kOpPredictApps, segs->n_apps), (hipStream_t)stream));
    return WM_OK;
}

int32_t wm_apps_loss_grad(const wm_desc_t* desc, const wm_segs_t* segs, const float* measured,
                          const wm_params_t* params, const wm_segparams_t* segp, double* out,
                          void* ws, size_t ws_bytes, void* stream)
{
    if (!desc_ok(desc) || !params_ok(params) || !segp_ok(segp) || !segs_ok(segs, desc->n) || !out)
        return WM_EINVAL;
    if (segs->n_apps > 0 && !measured) return WM_EINVAL;
    const AppsWs W = apps_ws(desc->n, segs->n_apps);
    if (!ws_ok(ws, ws_bytes, W.total)) return WM_EWORKSPACE;
    char* base = (char*)ws;
    const Set S = make_set(params);
    // no applications: the sweeps write zero rows, so out is still written
    WM_HIP(launch_apps_loss_grad(ptrs_of(desc), segptrs_of(segs), desc->n, segs->n_apps, measured,
                                 S, make_segset(segp), (double*)(base + W.rows), (uint64_t*)(base + W.aflags),
                                 (uint64_t*)(base + W.lflags), (uint64_t*)(base + W.rflags), (float*)(base + W.wrow),
                                 launch_cfg(kOpAppsLossGrad, segs->n_apps), out, (hipStream_t)stream));
    return WM_OK;
}

int32_t wm_predict_apps_vjp(const wm_desc_t* desc, const wm_segs_t* segs, const float* dL_dTapp,
                            const wm_params_t* params, const wm_segparams_t* segp, double* out,
                            void* ws, size_t ws_bytes, void* stream)
{
    if (!desc_ok(desc) || !params_ok(params) || !segp_ok(segp) || !segs_ok(segs, desc->n) || !out)
        return WM_EINVAL;
    if (segs->n_apps > 0 && !dL_dTapp) return WM_EINVAL;
    const AppsWs W = apps_ws(desc->n, segs->n_apps);
    if (!ws_ok(ws, ws_bytes, W.total)) return WM_EWORKSPACE;
    char* base = (char*)ws;
    const Set S = make_set(params);
    WM_HIP(launch_apps_vjp(ptrs_of(desc), segptrs_of(segs), desc->n, segs->n_apps, dL_dTapp, S,
                           make_segset(segp), (double*)(base + W.rows), (uint64_t*)(base + W.lflags),
                           (uint64_t*)(base + W.rflags), (float*)(base + W.wrow),
                           launch_cfg(kOpAppsLossGrad, segs->n_apps), out,
                           (hipStream_t)stream));
    return WM_OK;
}

int32_t wm_select_tile(const wm_shapes_t* shapes, const int32_t* cand_off,
                       const uint32_t* cand_code, int64_t n_cand, const wm_params_t* params,
                       int32_t* best, double* best_cost, uint8_t* near_tie, void* stream)
{
    if (!shapes || shapes->n < 0 || !params_ok(params) || n_cand < 0) return WM_EINVAL;
    if (shapes->n == 0) return WM_OK;
    if (!shapes->M || !shapes->N || !shapes->K || !shapes->dtype || !cand_off || !best ||
        !best_cost || !near_tie)
        return WM_EINVAL;
    if (n_cand > 0 && !cand_code) return WM_EINVAL;
    if (n_cand > 0x7fffffffll) return WM_EINVAL;
    ShapePtrs sp;
    sp.M = shapes->M;
    sp.N = shapes->N;
    sp.K = shapes->K;
    sp.dtype = shapes->dtype;
    const Set S = make_set(params);
    WM_HIP(launch_select_tile(sp, cand_off, cand_code, shapes->n, n_cand, S, best, best_cost,
                              near_tie, launch_cfg(kOpSelectTile, shapes->n), (hipStream_t)stream));
    return WM_OK;
}

int32_t wm_tile_costs(const wm_shapes_t* shapes, const int32_t* cand_off, const uint32_t* cand_code,
                      int64_t n_cand, const wm_params_t* params, float* cost, void* stream)
{
    if (!shapes || shapes->n < 0 || !params_ok(params) || n_cand < 0) return WM_EINVAL;
    if (shapes->n == 0) return WM_OK;
    if (!shapes->M || !shapes->N || !shapes->K || !shapes->dtype || !cand_off) return WM_EINVAL;
    if (n_cand > 0 && (!cand_code || !cost)) return WM_EINVAL;
    if (n_cand > 0x7fffffffll) return WM_EINVAL;
    ShapePtrs sp;
    sp.M = shapes->M;
    sp.N = shapes->N;
    sp.K = shapes->K;
    sp.dtype = shapes->dtype;
    const Set S = make_set(params);
    WM_HIP(launch_tile_costs(sp, cand_off, cand_code, shapes->n, n_cand, S, cost, (hipStream_t)stream));
    return WM_OK;
}

int32_t wm_calibrate_resume(const wm_desc_t* desc, const float* measured, const wm_params_t* p0,
                            const wm_calib_opts_t* opts, const wm_calib_state_t* state_in, int32_t run,
                            wm_calib_state_t* state_out, wm_params_t* p_out, double* loss_hist, void* ws,
                            size_t ws_bytes, void* stream)
{
    if (!desc_ok(desc) || (desc->n > 0 && !measured) || !params_ok(p0) || !opts_ok(opts) || !p_out)
        return WM_EINVAL;
    if (run < 1) return WM_EINVAL;
    wm_params_t pc = *p0;
    CalibState st0;
    if (state_in) {
        // the state's parameters must form a valid set with p0's structure
        if (state_in->step < 0 || state_in->step > opts->steps - run) return WM_EINVAL;
        if (state_in->diverged != 0) return WM_EINVAL;   // nothing to resume
        for (int j = 0; j < WM_N_THETA; ++j) pc.theta[j] = state_in->theta[j];
        if (!params_ok(&pc)) return WM_EINVAL;
        std::memset(&st0, 0, sizeof(st0));
        for (int j = 0; j < WM_N_THETA; ++j) {
            st0.theta[j] = state_in->theta[j];
            st0.theta_ok[j] = state_in->theta_ok[j];
            st0.phi[j] = state_in->phi[j];
            st0.m[j] = state_in->m[j];
            st0.v[j] = state_in->v[j];
        }
        st0.t = state_in->step;
        st0.diverged = state_in->diverged;
    } else {
        if (run > opts->steps) return WM_EINVAL;
        st0 = init_state(p0, opts->free_mask);
    }
    if (!free_slots_ok(&pc, opts->free_mask)) return WM_EINVAL;
    const CalibLayout L = calib_layout(desc->n, opts->steps);
    if (!ws_ok(ws, ws_bytes, L.total)) return WM_EWORKSPACE;
    hipStream_t s = nullptr;
    int32_t rc = capture_stream(stream, &s);
    if (rc != WM_OK) return rc;

    char* base = (char*)ws;
    Set* S_dev = (Set*)(base + L.set);
    CalibState* st_dev = (CalibState*)(base + L.state);
    double* hist_dev = (double*)(base + L.hist);
    double* part_dev = (double*)(base + L.grad + L.g.partials);
    uint64_t* flags_dev = (uint64_t*)(base + L.grad + L.g.flags);
    const Set S = make_set(&pc);
    AdamOpts ao = adam_of(opts);
    const std::vector<double> sched = adam_table(ao);
    ao.sched = (const double*)(base + L.sched);
    WM_HIP(hipMemcpyAsync(S_dev, &S, sizeof(S), hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(st_dev, &st0, sizeof(st0), hipMemcpyHostToDevice, s));
    WM_HIP(hipMemcpyAsync(base + L.sched, sched.data(), sizeof(double) * sched.size(),
                          hipMemcpyHostToDevice, s));
    WM_HIP(hipStreamSynchronize(s));

    const DescPtrs dp = ptrs_of(desc);
    const int64_t n = desc->n;
    const GradLayout G = L.g.g;
    const LaunchCfg cfg = launch_cfg(kOpLossGrad, n);
    // the float64 pass folds the sweep's rows: Adam reduces its nb2 rows
    double* rows2_dev = part_dev + (int64_t)grad_grid(1, true, n, cfg) * kAcc;
    auto step = [&]() -> hipError_t {
        hipError_t e = launch_grad(1, dp, n, measured, S, S_dev, part_dev, flags_dev, G, cfg,
                                   nullptr, s);
        if (e != hipSuccess) return e;
        return launch_adam(rows2_dev, G.nb2, st_dev, ao, S_dev, hist_dev, s);
    };
    rc = run_steps(s, run, step);
    if (rc != WM_OK) return rc;

    CalibState st;
    WM_HIP(hipMemcpyAsync(&st, st_dev, sizeof(st), hipMemcpyDeviceToHost, s));
    std::vector<double> hist((size_t)run);
    WM_HIP(hipMemcpyAsync(hist.data(), hist_dev + st0.t, sizeof(double) * run, hipMemcpyDeviceToHost, s));
    WM_HIP(hipStreamSynchronize(s));
    *p_out = pc;
    for (int j = 0; j < WM_N_THETA; ++j) p_out->theta[j] = st.diverged ? st.theta_ok[j] : st.theta[j];
    if (loss_hist) std::memcpy(loss_hist, hist.data(), sizeof(double) * run);
    if (state_out) {
        for (int j = 0; j < WM_N_THETA; ++j) {
            state_out->theta[j] = st.theta[j];
            state_out->theta_ok[j] = st.theta_ok[j];
            state_out->phi[j] = st.phi[j];
            state_out->m[j] = st.m[j];
            state_out->v[j] = st.v[j];
        }
        state_out->step = st.t;
        state_out->diverged = st.diverged;
    }
    return st.diverged ? WM_EDIVERGED : WM_OK;
}

int32_t wm_calibrate(const wm_desc_t* desc, const float* measured, const wm_params_t* p0,
                     const wm_calib_opts_t* opts, wm_params_t* p_out, double* loss_hist, void* ws,
                     size_t ws_bytes, void* stream)
{
    if (!opts_ok(opts)) return WM_EINVAL;
    return wm_calibrate_resume(desc, measured, p0, opts, nullptr, opts->steps, nullptr, p_out, loss_hist, ws,
                               ws_bytes, stream);
}

int32_t wm_calibrate_batched(int32_t n_sets, const wm_desc_t* sets, const float* const* measured,
                             const wm_params_t* p0, const wm_calib_opts_t* opts,
                             wm_params_t* p_out, double* loss_hist, void* ws, size_t ws_bytes,
                             void* stream)
{
    int64_t n_total = 0;
    if (!batch_args_ok(n_sets, sets, measured, p0, opts, &n_total) || !p_out) return WM_EINVAL;
    const int steps = opts[0].steps;
    const BatchLayout L = batch_layout(n_total, n_sets, steps);
    if (!ws_ok(ws, ws_bytes, L.total)) return WM_EWORKSPACE;
    hipStream_t s = nullptr;
    int32_t rc = capture_stream(stream, &s);
    if (rc != WM_OK) return rc;
    BatchRun run;
    rc = batch_prepare(n_sets, sets, measured, p0, opts, L, launch_cfg(kOpCalibrateBatched, n_total),
                       ws, s, &run);
    if (rc != WM_OK) return rc;
    rc = run_steps(s, steps, [&]() { return run.step(); });
    if (rc != WM_OK) return rc;

    std::vector<CalibState> sth((size_t)n_sets);
    WM_HIP(hipMemcpyAsync(sth.data(), run.st_dev, sizeof(CalibState) * n_sets, hipMemcpyDeviceToHost, s));
    std::vector<double> hist((size_t)n_sets * steps);
    WM_HIP(hipMemcpyAsync(hist.data(), run.hist_dev, sizeof(double) * hist.size(),
                          hipMemcpyDeviceToHost, s));
    WM_HIP(hipStreamSynchronize(s));
    bool div = false;
    for (int k = 0; k < n_sets; ++k) {
        p_out[k] = p0[k];
        for (int j = 0; j < WM_N_THETA; ++j)
            p_out[k].theta[j] = sth[k].diverged ? sth[k].theta_ok[j] : sth[k].theta[j];
        div = div || sth[k].diverged;
    }
    if (loss_hist) std::memcpy(loss_hist, hist.data(), sizeof(double) * hist.size());
    return div ? WM_EDIVERGED : WM_OK;
}

// ---- launch configurations and autotuning ----

int32_t wm_get_launch(int32_t op, int64_t n, wm_launch_t* cfg)
{
    if (!cfg || n < 0 || !cfg_valid(op, default_cfg(op))) return WM_EINVAL;
    *cfg = to_pub(launch_cfg(op, n));
    return WM_OK;
}

int32_t wm_set_launch(int32_t op, int64_t n, const wm_launch_t* cfg)
{
    if (!cfg || n < 0) return WM_EINVAL;
    const LaunchCfg c = from_pub(*cfg);
    if (!cfg_valid(op, c)) return WM_EINVAL;
    store_cfg(op, n, c, 0.0, false);
    return WM_OK;
}

int32_t wm_autotune_predict(const wm_desc_t* desc, const wm_params_t* params, float* T,
                            int32_t* occ, void* stream, wm_launch_t* best, double* best_us)
{
    if (!desc_ok(desc) || !params_ok(params) || !T || desc->n < 1) return WM_EINVAL;
    const bool vec = aligned16(desc) && ((uintptr_t)T & 15u) == 0 && ((uintptr_t)occ & 15u) == 0;
    const Set S = make_set(params);
    const DescPtrs dp = ptrs_of(desc);
    const int64_t n = desc->n;
    hipStream_t s = (hipStream_t)stream;
    std::vector<LaunchCfg> cands = candidates(kOpPredict);
    if (!vec) {
        std::vector<LaunchCfg> scal;
        for (const LaunchCfg& c : cands)
            if (c.vec == 1) scal.push_back(c);
        cands = scal;
    }
    return tune_over(kOpPredict, n, cands, s, 10,
                     [&](const LaunchCfg& c) { return launch_predict(dp, n, S, T, occ, vec, c, s); },
                     best, best_us);
}

int32_t wm_autotune_grad(int32_t op, const wm_desc_t* desc, const float* w,
                         const wm_params_t* params, double* out, void* ws, size_t ws_bytes,
                         void* stream, wm_launch_t* best, double* best_us)
{
    if (op != WM_OP_VJP && op != WM_OP_LOSS_GRAD) return WM_EINVAL;
    if (!desc_ok(desc) || !params_ok(params) || !out || !w || desc->n < 1) return WM_EINVAL;
    const int mode = op == WM_OP_LOSS_GRAD ? 1 : 0;
    const GradWs W = grad_ws(desc->n);
    if (!ws_ok(ws, ws_bytes, W.total)) return WM_EWORKSPACE;
    const Set S = make_set(params);
    const DescPtrs dp = ptrs_of(desc);
    const int64_t n = desc->n;
    char* base = (char*)ws;
    hipStream_t s = (hipStream_t)stream;
    return tune_over(op, n, candidates(op), s, 10,
                     [&](const LaunchCfg& c) {
                         return launch_grad(mode, dp, n, w, S, nullptr, (double*)(base + W.partials),
                                            (uint64_t*)(base + W.flags), W.g, c, out, s);
                     },
                     best, best_us);
}

int32_t wm_autotune_apps(int32_t op, const wm_desc_t* desc, const wm_segs_t* segs,
                         const float* measured, const wm_params_t* params,
                         const wm_segparams_t* segp, float* T_app, double* out, void* ws,
                         size_t ws_bytes, void* stream, wm_launch_t* best, double* best_us)
{
    if (op != WM_OP_PREDICT_APPS && op != WM_OP_APPS_LOSS_GRAD) return WM_EINVAL;
    if (!desc_ok(desc) || !params_ok(params) || !segp_ok(segp) || !segs_ok(segs, desc->n) ||
        segs->n_apps < 1)
        return WM_EINVAL;
    const Set S = make_set(params);
    const SegSet Q = make_segset(segp);
    const DescPtrs dp = ptrs_of(desc);
    const SegPtrs sp = segptrs_of(segs);
    const int64_t n = desc->n, na = segs->n_apps;
    hipStream_t s = (hipStream_t)stream;
    if (op == WM_OP_PREDICT_APPS) {
        if (!T_app) return WM_EINVAL;
        return tune_over(op, na, candidates(op), s, 10,
                         [&](const LaunchCfg& c) {
                             return launch_predict_apps(dp, sp, n, na, S, Q, T_app, nullptr, c, s);
                         },
                         best, best_us);
    }
    if (!measured || !out) return WM_EINVAL;
    const AppsWs W = apps_ws(n, na);
    if (!ws_ok(ws, ws_bytes, W.total)) return WM_EWORKSPACE;
    char* base = (char*)ws;
    return tune_over(op, na, candidates(op), s, 10,
                     [&](const LaunchCfg& c) {
                         return launch_apps_loss_grad(dp, sp, n, na, measured, S, Q, (double*)(base + W.rows),
                                                      (uint64_t*)(base + W.aflags), (uint64_t*)(base + W.lflags),
                                                      (uint64_t*)(base + W.rflags), (float*)(base + W.wrow), c,
                                                      out, s);
                     },
                     best, best_us);
}

int32_t wm_autotune_select_tile(const wm_shapes_t* shapes, const int32_t* cand_off,
                                const uint32_t* cand_code, int64_t n_cand,
                                const wm_params_t* params, int32_t* best_idx, double* best_cost,
                                uint8_t* near_tie, void* stream, wm_launch_t* best,
                                double* best_us)
{
    if (!shapes || shapes->n < 1 || !params_ok(params) || n_cand < 0 || n_cand > 0x7fffffffll)
        return WM_EINVAL;
    if (!shapes->M || !shapes->N || !shapes->K || !shapes->dtype || !cand_off || !best_idx ||
        !best_cost || !near_tie || (n_cand > 0 && !cand_code))
        return WM_EINVAL;
    ShapePtrs sp;
    sp.M = shapes->M;
    sp.N = shapes->N;
    sp.K = shapes->K;
    sp.dtype = shapes->dtype;
    const Set S = make_set(params);
    const int64_t n = shapes->n;
    hipStream_t s = (hipStream_t)stream;
    return tune_over(kOpSelectTile, n, candidates(kOpSelectTile), s, 10,
                     [&](const LaunchCfg& c) {
                         return launch_select_tile(sp, cand_off, cand_code, n, n_cand, S, best_idx,
                                                   best_cost, near_tie, c, s);
                     },
                     best, best_us);
}

int32_t wm_autotune_batched(int32_t n_sets, const wm_desc_t* sets, const float* const* measured,
                            const wm_params_t* p0, const wm_calib_opts_t* opts, void* ws,
                            size_t ws_bytes, void* stream, wm_launch_t* best, double* best_us)
{
    int64_t n_total = 0;
    if (!batch_args_ok(n_sets, sets, measured, p0, opts, &n_total)) return WM_EINVAL;
    const BatchLayout L = batch_layout(n_total, n_sets, opts[0].steps);
    if (!ws_ok(ws, ws_bytes, L.total)) return WM_EWORKSPACE;
    hipStream_t s = nullptr;
    int32_t rc = capture_stream(stream, &s);
    if (rc != WM_OK) return rc;
    // every candidate times one calibration step (sweep + reduce-and-Adam)
    // from freshly uploaded images, so the Adam state it perturbs is private
    // to the workspace
    std::vector<LaunchCfg> cands = candidates(kOpCalibrateBatched);
    double bu = 1e300;
    LaunchCfg bc = cands.front();
    for (const LaunchCfg& c : cands) {
        BatchRun run;
        rc = batch_prepare(n_sets, sets, measured, p0, opts, L, c, ws, s, &run);
        if (rc != WM_OK) return rc;
        double us = 0.0;
        rc = time_median(s, 10, [&]() { return run.step(); }, &us);
        if (rc != WM_OK) return rc;
        if (us < bu) {
            bu = us;
            bc = c;
        }
    }
    store_cfg(kOpCalibrateBatched, n_total, bc, bu, true);
    if (best) *best = to_pub(bc);
    if (best_us) *best_us = bu;
    return WM_OK;
}

}  // extern "C"
