// wm_device.hpp -- device-side helpers shared by the kernel files: streaming
// loads of one descriptor row and its float64 image, the fixed-order FP64
// block reductions, and the Adam step on log(theta).
#pragma once

#include "wm_launch.hpp"

namespace wm {

template <typename T>
__device__ inline T ntload(const T* p) { return __builtin_nontemporal_load(p); }

// Parameters read through a pointer into memory that stays constant while
// the kernel runs (a by-value kernel argument in the kernel-argument
// segment, or a set in device memory), laundered so that the optimiser cannot
// see through it: inside a sweep loop each parameter use is then a scalar
// load, served by the scalar cache.  Kept in scalar registers across the loop
// instead, the sixty-odd parameters overflow the 102 scalar registers; the
// compiler spills them to vector-register lanes and reloads each with one
// VALU instruction per descriptor.
template <typename T>
__device__ inline const T& uniform_const(const T* p)
{
    typedef __attribute__((address_space(4))) const T* CP;
    CP q = (CP)p;
    asm volatile("" : "+s"(q));
    return *(const T*)q;
}

// The address of by-value kernel argument `member` in the kernel-argument
// segment.  The arguments lie there in declaration order at their natural
// alignment, as the members of a struct (Mirror) that declares the kernel's
// parameters up to that argument do.  (A mismatch would feed every
// evaluation wrong parameters, which each parity test would show.)
#define WM_KERNARG_PTR(Mirror, member)                                                   \
    reinterpret_cast<const decltype(Mirror::member)*>(                                  \
        (const char*)__builtin_amdgcn_kernarg_segment_ptr() + __builtin_offsetof(Mirror, member))

__device__ inline Desc<float> load_desc(const DescPtrs& d, int64_t i)
{
    Desc<float> x;
    x.F = ntload(d.F + i);
    x.B = ntload(d.B + i);
    x.r1 = ntload(d.r1 + i);
    x.r2 = ntload(d.r2 + i);
    x.r3 = ntload(d.r3 + i);
    x.K = ntload(d.K + i);
    x.u = ntload(d.u + i);
    x.W = ntload(d.W + i);
    x.v = ntload(d.vgpr + i);
    x.s = ntload(d.lds + i);
    x.gp = ntload(d.gpack + i);
    x.G = ntload(d.grid + i);
    return x;
}

__device__ inline Desc<double> widen(const Desc<float>& x)
{
    Desc<double> y;
    y.F = x.F; y.B = x.B; y.r1 = x.r1; y.r2 = x.r2; y.r3 = x.r3; y.K = x.K; y.u = x.u; y.W = x.W;
    y.v = x.v; y.s = x.s; y.gp = x.gp; y.G = x.G;
    return y;
}

// ---------------------------------------------------------------------------
// block reduction of the 26 FP64 accumulators (fixed order)
// ---------------------------------------------------------------------------
// One step of the wave's recursive halving over lane bit m: a lane keeps the
// upper half of its H x 2 remaining columns if its bit m is set, else the
// lower half, and adds the partner lane's copy of the half it keeps.
template <int H>
__device__ inline void halve_columns(double* v, int lane, int m)
{
    const bool hi = (lane & m) != 0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const double send = hi ? v[j] : v[j + H];
        const double keep = hi ? v[j + H] : v[j];
        v[j] = keep + __shfl_xor(send, m, 64);
    }
}

// Block sum of the 26 per-thread accumulators (fixed order).  Within a wave
// the columns are halved over lane bits 5..1 (32 doubles cross lanes, not
// 26 x 6 for one butterfly per column), after which lanes 2c and 2c + 1
// hold column c over 32 lanes each; then the waves' rows are added in LDS.
// Must be called by every thread of the block.  acc is clobbered.
__device__ inline void block_reduce_acc(double* acc, double* lds /* [waves][26] */, double* out)
{
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    static_assert(kAcc <= 32, "the halving covers 32 columns");
    double v[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) v[j] = j < kAcc ? acc[j] : 0.0;
    halve_columns<16>(v, lane, 32);
    halve_columns<8>(v, lane, 16);
    halve_columns<4>(v, lane, 8);
    halve_columns<2>(v, lane, 4);
    halve_columns<1>(v, lane, 2);
    const double s = v[0] + __shfl_xor(v[0], 1, 64);
    const int col = lane >> 1;
    if ((lane & 1) == 0 && col < kAcc) lds[wid * kAcc + col] = s;
    __syncthreads();
    if (threadIdx.x < kAcc) {
        const int nw = blockDim.x >> 6;
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[w * kAcc + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Fixed-order sum of partial rows: thread t adds rows t, t+256, ... of all 26
// columns, then the block tree of block_reduce_acc.
__device__ inline void reduce_partials(const double* __restrict__ partials, int rows, int stride,
                                       double* red /* [waves][26] */, double* tot /* [26] */)
{
    double acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        const double* row = partials + (int64_t)r * stride;
#pragma unroll
        for (int j = 0; j < kAcc; ++j) acc[j] += row[j];
    }
    block_reduce_acc(acc, red, tot);
}

// ---------------------------------------------------------------------------
// device Adam on log(theta)
// ---------------------------------------------------------------------------
// Closest non-decreasing (INC) or non-increasing sequence, in the least-
// squares sense, to the values of lanes base .. base + 3; lane base + i gets
// element i, other lanes keep v.  Element i of the isotonic fit is
// max over a <= i of min over b >= i of the mean of y[a..b] (non-decreasing;
// min and max swap for non-increasing).  Called by all 64 lanes, converged.
template <bool INC>
__device__ inline double isotonic4(double v, int lane, int base)
{
    double y[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = __shfl(v, base + k, 64);
    const int i = lane - base;
    if (i < 0 || i > 3) return v;
    double best = INC ? -HUGE_VAL : HUGE_VAL;
    for (int a = 0; a <= i; ++a) {
        double inner = INC ? HUGE_VAL : -HUGE_VAL, sum = 0.0;
        for (int b = a; b < 4; ++b) {
            sum += y[b];
            if (b < i) continue;
            const double mean = sum / (double)(b - a + 1);
            inner = INC ? fmin(inner, mean) : fmax(inner, mean);
        }
        best = INC ? fmax(best, inner) : fmin(best, inner);
    }
    return best;
}

__device__ inline bool adam_theta_step(CalibState* st, const double* tot, const AdamOpts& o,
                                       double* loss_hist, double* th_out /* LDS [kTheta] */)
{
    // Called by the 64 lanes of one wave, converged; lane j < 24 updates
    // theta_j.  The step index lives in device memory so one captured graph
    // serves every chunk of steps.  Returns true (on every lane) when theta
    // changed; th_out then holds the new theta, visible to the whole wave,
    // and the caller rebuilds its constants from it.
    const int lane = threadIdx.x & 63;
    const int step_index = st->t;
    const int was_diverged = st->diverged;
    const double cnt = tot[1];
    const double loss = cnt > 0.0 ? tot[0] / cnt : 0.0;
    if (lane == 0) {
        st->t = step_index + 1;
        if (loss_hist && step_index < o.steps)
            loss_hist[step_index] = was_diverged ? __builtin_nan("") : loss;
    }
    if (was_diverged) return false;
    const bool mine = lane < kTheta;
    const double g = mine && cnt > 0.0 ? tot[2 + lane] / cnt : 0.0;
    if (!__builtin_isfinite(loss) || __ballot(!__builtin_isfinite(g)) != 0) {
        if (lane == 0) st->diverged = 1;
        return false;
    }
    const double th = mine ? st->theta[lane] : 1.0;
    if (mine) st->theta_ok[lane] = th;
    // the step's schedule: from the host's table (three loads) where there is
    // one, else formed here (three pow calls on the wave's critical path)
    double lr, c1, c2;
    if (o.sched && step_index < o.steps) {
        lr = o.sched[3 * step_index];
        c1 = o.sched[3 * step_index + 1];
        c2 = o.sched[3 * step_index + 2];
    } else {
        adam_schedule(o, step_index, &lr, &c1, &c2);
    }
    double th_new = th;
    bool ok = true;
    const bool fit = mine && ((o.free_mask >> lane) & 1u);
    double phi = fit ? st->phi[lane] : 0.0;
    if (fit) {
        const double gp = th * g;
        const double m = o.beta1 * st->m[lane] + (1.0 - o.beta1) * gp;
        const double v = o.beta2 * st->v[lane] + (1.0 - o.beta2) * gp * gp;
        st->m[lane] = m;
        st->v[lane] = v;
        const double mh = m / c1;
        const double vh = v / c2;
        phi -= lr * mh / (sqrt(vh) + o.eps);
    }
    // constraints: the level orderings (every slot of an ordered group is
    // fitted), then the boxes
    if (o.order & 1) phi = isotonic4<false>(phi, lane, 0);
    if (o.order & 2) phi = isotonic4<true>(phi, lane, 4);
    if (fit) {
        phi = fmin(fmax(phi, o.lo_log[lane]), o.hi_log[lane]);
        st->phi[lane] = phi;
        th_new = exp(phi);
        ok = __builtin_isfinite(th_new) && th_new > 0.0;
    }
    if (__ballot(!ok) != 0) {
        if (lane == 0) st->diverged = 1;
        return false;
    }
    if (mine) {
        st->theta[lane] = th_new;
        th_out[lane] = th_new;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return true;
}


}  // namespace wm
