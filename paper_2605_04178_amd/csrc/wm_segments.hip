// wm_segments.hip -- workload segments (Sections IV-E, IV-F and V-B): an
// application is a run of segment rows, each a kernel descriptor executed
// n_exec times with n_kern launches per execution, a per-class scale on the
// kernel time and optional host-device transfers (Eq. (15)).  Kernels:
// application totals, and the application-level mean relative error with its
// gradient with respect to theta and the seven segment parameters.
//
// Layout: applications are CSR offsets over the segment rows, which run
// parallel to the descriptor rows.  A block takes `BLOCK` consecutive
// applications; their rows are contiguous, so it streams them with coalesced
// loads in pieces of 8 x BLOCK rows staged in LDS, then each thread adds its own
// application's rows in float64, in row order.
#include "wm_device.hpp"

namespace wm {


struct SegRow {
    float ne, h, dd;
    int32_t nk, c;
};

// KEEP = true: ordinary loads, so that a second pass over the same rows
// finds them in the caches; false: streaming (nontemporal) loads.
template <bool KEEP = false>
__device__ inline SegRow load_seg(const SegPtrs& sg, int64_t i)
{
    SegRow r;
    if (KEEP) {
        r.ne = sg.n_exec[i];
        r.nk = sg.n_kern[i];
        r.c = sg.cls[i];
        r.h = sg.h2d[i];
        r.dd = sg.d2h[i];
    } else {
        r.ne = ntload(sg.n_exec + i);
        r.nk = ntload(sg.n_kern + i);
        r.c = ntload(sg.cls + i);
        r.h = ntload(sg.h2d + i);
        r.dd = ntload(sg.d2h + i);
    }
    return r;
}

__device__ inline bool seg_row_valid(const SegRow& r)
{
    const float inf = __builtin_huge_valf();
    return (r.ne >= 0.0f) & (r.ne < inf) & (r.nk >= 1) & (r.c >= 0) & (r.c <= 3) & (r.h >= 0.0f) &
           (r.h < inf) & (r.dd >= 0.0f) & (r.dd < inf);
}

template <typename R>
__device__ inline R kappa_of(const SegConst<R>& q, int32_t c)
{
    R k = q.kappa[0];
    k = c == 1 ? q.kappa[1] : k;
    k = c == 2 ? q.kappa[2] : k;
    k = c == 3 ? q.kappa[3] : k;
    return k;
}

// Segment time from its kernel time Tk:
//   n_exec (kappa_cls Tk + (n_kern - 1) T_launch
//           + [h2d > 0] (h2d / B_h2d + tau) + [d2h > 0] (d2h / B_d2h + tau)),
// NaN for an invalid row or kernel, +inf for an infeasible kernel.
template <typename R>
__device__ inline R seg_time(R Tk, const SegRow& r, const SegConst<R>& q, R t_launch)
{
    if (!seg_row_valid(r) || !(Tk == Tk)) return (R)__builtin_nan("");
    if (!(Tk < (R)__builtin_huge_val())) return Tk;
    R t = kappa_of(q, r.c) * Tk + (R)(r.nk - 1) * t_launch;
    if (r.h > 0.0f) t += (R)r.h * q.inv_bw_h2d + q.tau;
    if (r.dd > 0.0f) t += (R)r.dd * q.inv_bw_d2h + q.tau;
    return (R)r.ne * t;
}

// Fixed-order block sum of NA float64 accumulators into out[NA].
template <int NA>
__device__ inline void block_sum(double* acc, double* lds /* [waves][NA] */, double* out)
{
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        double v = acc[j];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
        acc[j] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NA; ++j) lds[wid * NA + j] = acc[j];
    }
    __syncthreads();
    if (threadIdx.x < NA) {
        const int nw = blockDim.x >> 6;
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[w * NA + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Application sweep.  A block takes BLOCK consecutive applications (one per
// thread); their rows are staged in LDS in pieces of 8 x BLOCK rows (one
// piece unless the chunk averages more than 8 rows per application).
// MODE 0: T_app[a] (float32) and optionally the segment times.
// MODE 1 (loss) and MODE 2 (vector-Jacobian product, weights dL/dT_app read
// from `meas`): after the application totals, a second row-parallel pass
// writes the adjoint weights wseg[j] = w_a * n_exec_j * kappa_cls(j) for the
// kernel model's vector-Jacobian product, with w_a = sign(T_a - m_a) / m_a
// (MODE 1) or dL/dT_app[a] (MODE 2), and adds w_a times each row's n_exec (n_kern - 1), n_exec Tk (per class),
// n_exec h2d, n_exec d2h and n_exec x transfers; per block one row of
// kAppAcc float64 sums (loss, count, those seven).  In MODE 1 an application
// with |T_a/m_a - 1| <= 1e-5 in this float32 sweep gets zero weights and is
// flagged in aflags (one 64-bit ballot word per 64 applications) for
// k_apps_redo.  Offsets are caller data: they are clamped into [0, n_seg],
// so malformed offsets give unspecified values but no out-of-range access.
template <int BLOCK, int MODE>
__global__ __launch_bounds__(BLOCK) void k_apps(DescPtrs d, SegPtrs sg, int64_t n_seg,
                                               int64_t n_apps, Set S, SegSet Q,
                                               const float* __restrict__ meas,
                                               float* __restrict__ T_app, float* __restrict__ T_seg,
                                               float* __restrict__ wseg, double* __restrict__ rows,
                                               uint64_t* __restrict__ aflags)
{
    constexpr bool LOSS = MODE != 0;  // loss (1) and vector-Jacobian product (2) share the weights pass
    constexpr int CAP = 8 * BLOCK;
    constexpr int LC = LOSS ? CAP : 1;
    __shared__ float ts[CAP];
    __shared__ float ekn[LC];       // n_exec * T_kernel
    __shared__ uint8_t ecl[LC];     // class
    __shared__ uint16_t own[LC];    // application (index in the chunk) of the row
    __shared__ int32_t lo_s[BLOCK], hi_s[BLOCK];
    __shared__ float wa_s[LOSS ? BLOCK : 1];
    __shared__ double red[LOSS ? 8 * kAppAcc : 1];

    double acc[kAppAcc];
#pragma unroll
    for (int j = 0; j < kAppAcc; ++j) acc[j] = 0.0;
    const int tid = threadIdx.x;
    const int64_t nchunks = (n_apps + BLOCK - 1) / BLOCK;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t a = ch * BLOCK + tid;
        const int64_t left = n_apps - ch * BLOCK;
        const int na = left < BLOCK ? (int)left : BLOCK;
        int32_t lo = 0, hi = 0;
        if (tid < na) {
            int64_t x = sg.off[a], y = sg.off[a + 1];
            x = x < 0 ? 0 : (x > n_seg ? n_seg : x);
            y = y < x ? x : (y > n_seg ? n_seg : y);
            lo = (int32_t)x;
            hi = (int32_t)y;
        }
        lo_s[tid] = lo;
        hi_s[tid] = hi;
        __syncthreads();
        const int32_t sb = lo_s[0], se = hi_s[na - 1];
        const bool one_piece = se - sb <= CAP;
        double tot = 0.0;
        for (int32_t pb = sb; pb < se; pb += CAP) {
            const int32_t pe = se - pb < CAP ? se : pb + CAP;
            // rows are visited from a 64-row boundary so that every wave's
            // loads cover whole cache lines (the rows before pb are skipped)
            for (int32_t j = (pb & ~63) + tid; j < pe; j += BLOCK) {
                if (j < pb) continue;
                const Desc<float> x = load_desc(d, j);
                const SegRow r = load_seg<LOSS>(sg, j);
                Eval<float> E;
                evaluate<float, false>(S.st, S.cf, x, E);
                const float t = seg_time<float>(E.T, r, Q.f, S.cf.ov[0]);
                ts[j - pb] = t;
                if (T_seg) __builtin_nontemporal_store(t, T_seg + j);
                if (LOSS) {
                    ekn[j - pb] = r.ne * E.T;
                    ecl[j - pb] = (uint8_t)(r.c & 3);
                }
            }
            __syncthreads();
            if (tid < na) {
                const int32_t jb = lo > pb ? lo : pb, je = hi < pe ? hi : pe;
                for (int32_t j = jb; j < je; ++j) {
                    tot += (double)ts[j - pb];
                    if (LOSS) own[j - pb] = (uint16_t)tid;
                }
            }
            __syncthreads();
        }
        if (!LOSS) {
            if (tid < na) __builtin_nontemporal_store((float)tot, T_app + a);
            __syncthreads();  // lo_s / hi_s are rewritten by the next chunk
            continue;
        }
        float wa = 0.0f;
        bool near = false;
        if (MODE == 2 && tid < na && tot - tot == 0.0) {
            wa = meas[a];  // dL/dT_app
        } else if (MODE == 1 && tid < na) {
            const float mf = meas[a];
            if (tot - tot == 0.0 && mf > 0.0f && mf < __builtin_huge_valf()) {
                const double m = mf, im = 1.0 / m;
                const double T = tot;
                near = __builtin_fabs(T * im - 1.0) <= 1e-5;
                if (!near) {
                    const double w = T > m ? im : (T < m ? -im : 0.0);
                    acc[0] += __builtin_fabs(T - m) * im;
                    acc[1] += 1.0;
                    wa = (float)w;
                }
            }
        }
        if (MODE == 1) {
            const uint64_t fw = __ballot(near);
            if ((tid & 63) == 0 && a < n_apps) aflags[a >> 6] = fw;
        }
        wa_s[tid] = wa;
        __syncthreads();
        // row-parallel pass: weights and the segment-parameter sums.  With one
        // piece the owner, class and n_exec Tk are still in LDS; otherwise the
        // owner is found by binary search and Tk is evaluated again.
        for (int32_t j = (sb & ~63) + tid; j < se; j += BLOCK) {
            if (j < sb) continue;
            int t0;
            float ek;
            int32_t c;
            bool mine = true;
            if (one_piece) {
                t0 = own[j - sb];
                t0 = t0 < na ? t0 : na - 1;  // rows no application owns (bad offsets)
                mine = j >= lo_s[t0] && j < hi_s[t0];
                ek = ekn[j - sb];
                c = ecl[j - sb];
            } else {
                int t1 = na - 1;
                t0 = 0;
                while (t0 < t1) {
                    const int mid = (t0 + t1 + 1) >> 1;
                    if (lo_s[mid] <= j) t0 = mid;
                    else t1 = mid - 1;
                }
                mine = j >= lo_s[t0] && j < hi_s[t0];
                ek = 0.0f;
                c = 0;
            }
            const float wt = mine ? wa_s[t0] : 0.0f;
            float w = 0.0f;
            if (wt != 0.0f) {
                const SegRow r = load_seg<true>(sg, j);
                if (!one_piece) {
                    Eval<float> E;
                    evaluate<float, false>(S.st, S.cf, load_desc(d, j), E);
                    ek = r.ne * E.T;
                    c = r.c;
                }
                w = wt * r.ne * kappa_of(Q.f, c);
                const double wd = wt;
                acc[2] += wd * (double)(r.ne * (float)(r.nk - 1));
                const double v = wd * (double)ek;
                acc[3] += c == 0 ? v : 0.0;
                acc[4] += c == 1 ? v : 0.0;
                acc[5] += c == 2 ? v : 0.0;
                acc[6] += c == 3 ? v : 0.0;
                if (r.h > 0.0f) {
                    acc[7] += wd * (double)(r.ne * r.h);
                    acc[9] += wd * (double)r.ne;
                }
                if (r.dd > 0.0f) {
                    acc[8] += wd * (double)(r.ne * r.dd);
                    acc[9] += wd * (double)r.ne;
                }
            }
            wseg[j] = w;
        }
        __syncthreads();
    }
    if (LOSS) block_sum<kAppAcc>(acc, red, rows + (int64_t)blockIdx.x * kAppAcc);
}

// The applications flagged by k_apps: float64 totals decide the sign; their
// loss and gradient sums go to this kernel's rows and their row weights to
// wseg.  Block b first folds the sweep's rows b, b + gridDim.x, ... (fixed
// order), so the final reduction sees gridDim.x rows.
__global__ __launch_bounds__(256) void k_apps_redo(DescPtrs d, SegPtrs sg, int64_t n_seg,
                                                    int64_t n_apps, Set S, SegSet Q,
                                                    const float* __restrict__ meas,
                                                    const uint64_t* __restrict__ aflags,
                                                    const double* __restrict__ rows1, int nrows1,
                                                    float* __restrict__ wseg,
                                                    double* __restrict__ rows2)
{
    __shared__ double red[4 * kAppAcc];
    double acc[kAppAcc];
#pragma unroll
    for (int j = 0; j < kAppAcc; ++j) acc[j] = 0.0;
    for (int r = blockIdx.x + gridDim.x * threadIdx.x; r < nrows1; r += gridDim.x * blockDim.x) {
#pragma unroll
        for (int j = 0; j < kAppAcc; ++j) acc[j] += rows1[(int64_t)r * kAppAcc + j];
    }
    const int64_t nwords = (n_apps + 63) >> 6;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; wi < nwords; wi += stride) {
        uint64_t fw = aflags[wi];
        while (fw) {
            const int bit = __builtin_ctzll(fw);
            fw &= fw - 1;
            const int64_t a = (wi << 6) + bit;
            int64_t lo = sg.off[a], hi = sg.off[a + 1];
            lo = lo < 0 ? 0 : (lo > n_seg ? n_seg : lo);
            hi = hi < lo ? lo : (hi > n_seg ? n_seg : hi);
            double T = 0.0, sk[4] = {0.0, 0.0, 0.0, 0.0}, sl = 0.0, sh = 0.0, sd = 0.0, sn = 0.0;
            for (int64_t j = lo; j < hi; ++j) {
                Eval<double> E;
                evaluate<double, false>(S.st, S.cd, widen(load_desc(d, j)), E);
                const SegRow r = load_seg(sg, j);
                T += seg_time<double>(E.T, r, Q.d, S.cd.ov[0]);
                const double ne = r.ne;
                const double v = ne * E.T;
                sk[0] += r.c == 0 ? v : 0.0;
                sk[1] += r.c == 1 ? v : 0.0;
                sk[2] += r.c == 2 ? v : 0.0;
                sk[3] += r.c == 3 ? v : 0.0;
                sl += ne * (double)(r.nk - 1);
                sh += r.h > 0.0f ? ne * (double)r.h : 0.0;
                sd += r.dd > 0.0f ? ne * (double)r.dd : 0.0;
                sn += ne * (double)((int)(r.h > 0.0f) + (int)(r.dd > 0.0f));
            }
            const double m = meas[a], im = 1.0 / m;
            float wa = 0.0f;
            if (T - T == 0.0) {
                const double w = T > m ? im : (T < m ? -im : 0.0);
                acc[0] += __builtin_fabs(T - m) * im;
                acc[1] += 1.0;
                acc[2] += w * sl;
                acc[3] += w * sk[0];
                acc[4] += w * sk[1];
                acc[5] += w * sk[2];
                acc[6] += w * sk[3];
                acc[7] += w * sh;
                acc[8] += w * sd;
                acc[9] += w * sn;
                wa = (float)w;
            }
            for (int64_t j = lo; j < hi; ++j)
                wseg[j] = wa != 0.0f ? wa * sg.n_exec[j] * kappa_of(Q.f, sg.cls[j]) : 0.0f;
        }
    }
    block_sum<kAppAcc>(acc, red, rows2 + (int64_t)blockIdx.x * kAppAcc);
}

// Final fixed-order reduction: the gradient sweep's nb2 rows of kAcc columns
// (sum of wseg_j dTk_j/dtheta) and the application sweep's rows of kAppAcc
// columns, into [loss, count, grad theta[24], grad seg params[7]] divided by
// the count.
__global__ __launch_bounds__(256) void k_apps_reduce(const double* __restrict__ grows, int ng,
                                                     const double* __restrict__ arows, int na,
                                                     SegSet Q, int vjp, double* __restrict__ out)
{
    __shared__ double red[4 * kAcc];
    __shared__ double tg[kAcc], ta[kAppAcc];
    {
        double acc[kAcc];
#pragma unroll
        for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
        for (int r = threadIdx.x; r < ng; r += blockDim.x)
#pragma unroll
            for (int j = 0; j < kAcc; ++j) acc[j] += grows[(int64_t)r * kAcc + j];
        block_sum<kAcc>(acc, red, tg);
    }
    {
        double acc[kAppAcc];
#pragma unroll
        for (int j = 0; j < kAppAcc; ++j) acc[j] = 0.0;
        for (int r = threadIdx.x; r < na; r += blockDim.x)
#pragma unroll
            for (int j = 0; j < kAppAcc; ++j) acc[j] += arows[(int64_t)r * kAppAcc + j];
        block_sum<kAppAcc>(acc, red, ta);
    }
    const int t = threadIdx.x;
    if (vjp) {
        // [grad theta[24], grad seg params[7]], plain sums
        if (t >= kTheta + kSegParams) return;
        double v;
        if (t < kTheta) v = tg[2 + t] + (t == 13 ? ta[2] : 0.0);
        else if (t < kTheta + 4) v = ta[3 + (t - kTheta)];
        else if (t == kTheta + 4) v = -ta[7] * Q.inv_bw2_h2d;
        else if (t == kTheta + 5) v = -ta[8] * Q.inv_bw2_d2h;
        else v = ta[9];
        out[t] = v;
        return;
    }
    if (t >= kAppsOut) return;
    const double c = ta[1];
    const double ic = c > 0.0 ? 1.0 / c : 0.0;
    double v;
    if (t == 0) v = ta[0] * ic;
    else if (t == 1) v = c;
    else if (t < kAcc) v = (tg[t] + (t == 2 + 13 ? ta[2] : 0.0)) * ic;
    else if (t < kAcc + 4) v = ta[3 + (t - kAcc)] * ic;
    else if (t == kAcc + 4) v = -ta[7] * Q.inv_bw2_h2d * ic;
    else if (t == kAcc + 5) v = -ta[8] * Q.inv_bw2_d2h * ic;
    else v = ta[9] * ic;
    out[t] = v;
}

template <int BLOCK, int MODE>
static int apps_grid(int64_t n_apps, int grid_mult)
{
    const int64_t chunks = (n_apps + BLOCK - 1) / BLOCK;
    int64_t b = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_apps<BLOCK, MODE>), BLOCK) *
                (grid_mult < 1 ? 1 : grid_mult);
    b = b < chunks ? b : chunks;
    b = b < kAppsMaxBlocks ? b : kAppsMaxBlocks;
    return (int)(b < 1 ? 1 : b);
}

template <int MODE>
static hipError_t apps_t(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg, int64_t n_apps,
                         const Set& S, const SegSet& Q, const float* meas, float* T_app,
                         float* T_seg, float* wseg, double* rows, uint64_t* aflags,
                         const LaunchCfg& c, hipStream_t s)
{
#define WM_APPS_CASE(B)                                                                        \
    case B:                                                                                    \
        k_apps<B, MODE><<<apps_grid<B, MODE>(n_apps, c.grid_mult), B, 0, s>>>(                 \
            d, sg, n_seg, n_apps, S, Q, meas, T_app, T_seg, wseg, rows, aflags);               \
        break;
    switch (c.block) {
        WM_APPS_CASE(64)
        WM_APPS_CASE(128)
        WM_APPS_CASE(256)
        WM_APPS_CASE(512)
    default: return hipErrorInvalidValue;
    }
#undef WM_APPS_CASE
    return hipGetLastError();
}

hipError_t launch_predict_apps(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg, int64_t n_apps,
                               const Set& S, const SegSet& Q, float* T_app, float* T_seg,
                               const LaunchCfg& cfg, hipStream_t stream)
{
    if (n_apps <= 0) return hipSuccess;
    return apps_t<0>(d, sg, n_seg, n_apps, S, Q, nullptr, T_app, T_seg, nullptr, nullptr,
                     nullptr, cfg, stream);
}

// Rows the application sweep of mode MODE writes for n_apps applications
// (at least one).
template <int MODE>
static int apps_rows(int64_t n_apps, const LaunchCfg& c)
{
    switch (c.block) {
    case 64: return apps_grid<64, MODE>(n_apps, c.grid_mult);
    case 128: return apps_grid<128, MODE>(n_apps, c.grid_mult);
    case 512: return apps_grid<512, MODE>(n_apps, c.grid_mult);
    default: return apps_grid<256, MODE>(n_apps, c.grid_mult);
    }
}

int apps_redo_blocks(int64_t n_apps)
{
    const int64_t b = ((n_apps + 63) / 64 + 255) / 256;
    return (int)(b < 1 ? 1 : (b > kRedoMaxBlocks ? kRedoMaxBlocks : b));
}

hipError_t launch_apps_loss_grad(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg,
                                 int64_t n_apps, const float* measured, const Set& S,
                                 const SegSet& Q, float* wseg, double* app_rows, uint64_t* aflags,
                                 double* partials, uint64_t* flags, const GradLayout& L,
                                 const LaunchCfg& cfg, const LaunchCfg& vjp_cfg, double* out,
                                 hipStream_t stream)
{
    hipError_t e = apps_t<1>(d, sg, n_seg, n_apps, S, Q, measured, nullptr, nullptr, wseg,
                             app_rows, aflags, cfg, stream);
    if (e != hipSuccess) return e;
    const int na1 = apps_rows<1>(n_apps, cfg), na2 = apps_redo_blocks(n_apps);
    double* rows2 = app_rows + (int64_t)na1 * kAppAcc;
    k_apps_redo<<<na2, 256, 0, stream>>>(d, sg, n_seg, n_apps, S, Q, measured, aflags, app_rows,
                                         na1, wseg, rows2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_grad(0, d, n_seg, wseg, S, nullptr, partials, flags, L, vjp_cfg, nullptr, stream);
    if (e != hipSuccess) return e;
    const int nb = grad_grid(0, false, n_seg, vjp_cfg);
    k_apps_reduce<<<1, 256, 0, stream>>>(partials + (int64_t)nb * kAcc, L.nb2, rows2, na2, Q, 0, out);
    return hipGetLastError();
}

hipError_t launch_apps_vjp(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg, int64_t n_apps,
                           const float* w_app, const Set& S, const SegSet& Q, float* wseg,
                           double* app_rows, double* partials, uint64_t* flags, const GradLayout& L,
                           const LaunchCfg& cfg, const LaunchCfg& vjp_cfg, double* out,
                           hipStream_t stream)
{
    hipError_t e = apps_t<2>(d, sg, n_seg, n_apps, S, Q, w_app, nullptr, nullptr, wseg, app_rows,
                             nullptr, cfg, stream);
    if (e != hipSuccess) return e;
    e = launch_grad(0, d, n_seg, wseg, S, nullptr, partials, flags, L, vjp_cfg, nullptr, stream);
    if (e != hipSuccess) return e;
    const int nb = grad_grid(0, false, n_seg, vjp_cfg);
    k_apps_reduce<<<1, 256, 0, stream>>>(partials + (int64_t)nb * kAcc, L.nb2, app_rows,
                                         apps_rows<2>(n_apps, cfg), Q, 1, out);
    return hipGetLastError();
}

}  // namespace wm
