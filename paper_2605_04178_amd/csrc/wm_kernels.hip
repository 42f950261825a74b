// wm_kernels.hip -- gfx950 kernels of libwavemodel: forward sweep, naive
// roofline, adjoint / loss-gradient with fixed-order FP64 reductions, device
// Adam, occupancy-driven tile selection and the multi-set calibration sweep.
//
// Memory layout: descriptors are structure-of-arrays; the forward kernel
// streams them with 16-byte nontemporal loads (4 descriptors per thread per
// array) and writes T / occ with nontemporal stores, so a sweep larger than
// the 256 MB Infinity Cache does not evict anything useful.  The gradient
// kernels are persistent (grid-stride) and keep 26 FP64 accumulators per
// thread, reduced across the wave with shuffles, across the block through LDS
// and across blocks by a second single-block kernel in a fixed order.
#include "wm_device.hpp"

#include <map>
#include <mutex>
#include <utility>

namespace wm {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// forward sweep
// ---------------------------------------------------------------------------
template <int V> struct VecT {
    typedef float f __attribute__((ext_vector_type(V)));
    typedef int i __attribute__((ext_vector_type(V)));
};

// VEC consecutive descriptors per thread: one VEC-wide nontemporal load per
// array (16 B at VEC = 4), the evaluations, one VEC-wide store of T and occ.
template <int VEC, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_predict(DescPtrs d, int64_t n, Set S,
                                                    float* __restrict__ T, int32_t* __restrict__ occ)
{
    const int64_t i0 = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * VEC;
    if (i0 >= n) return;
    if constexpr (VEC > 1) {
        if (i0 + VEC <= n) {
            typedef typename VecT<VEC>::f fv;
            typedef typename VecT<VEC>::i iv;
            const fv F = ntload((const fv*)(d.F + i0));
            const fv B = ntload((const fv*)(d.B + i0));
            const fv r1 = ntload((const fv*)(d.r1 + i0));
            const fv r2 = ntload((const fv*)(d.r2 + i0));
            const fv r3 = ntload((const fv*)(d.r3 + i0));
            const fv K = ntload((const fv*)(d.K + i0));
            const fv u = ntload((const fv*)(d.u + i0));
            const fv W = ntload((const fv*)(d.W + i0));
            const iv v = ntload((const iv*)(d.vgpr + i0));
            const iv s = ntload((const iv*)(d.lds + i0));
            const iv gp = ntload((const iv*)(d.gpack + i0));
            const iv G = ntload((const iv*)(d.grid + i0));
            fv t;
            iv o;
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                Desc<float> x;
                x.F = F[j]; x.B = B[j]; x.r1 = r1[j]; x.r2 = r2[j]; x.r3 = r3[j];
                x.K = K[j]; x.u = u[j]; x.W = W[j]; x.v = v[j]; x.s = s[j]; x.gp = gp[j]; x.G = G[j];
                Eval<float> E;
                evaluate<float, false>(S.st, S.cf, x, E);
                t[j] = E.T;
                o[j] = E.occ;
            }
            __builtin_nontemporal_store(t, (fv*)(T + i0));
            if (occ) __builtin_nontemporal_store(o, (iv*)(occ + i0));
            return;
        }
    }
    for (int j = 0; j < VEC; ++j) {
        const int64_t i = i0 + j;
        if (i >= n) break;
        Desc<float> x = load_desc(d, i);
        Eval<float> E;
        evaluate<float, false>(S.st, S.cf, x, E);
        __builtin_nontemporal_store(E.T, T + i);
        if (occ) __builtin_nontemporal_store(E.occ, occ + i);
    }
}

__global__ __launch_bounds__(256) void k_roofline(DescPtrs d, int64_t n, Set S,
                                                   float* __restrict__ T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Desc<float> x = load_desc(d, i);
    float r = __builtin_nanf("");
    if (desc_valid(x)) {
        const int dt = (x.gp >> 11) & 7;
        float ip = S.cf.inv_peak[0];
        ip = dt == 1 ? S.cf.inv_peak[1] : ip;
        ip = dt == 2 ? S.cf.inv_peak[2] : ip;
        ip = dt == 3 ? S.cf.inv_peak[3] : ip;
        ip = dt == 4 ? S.cf.inv_peak[4] : ip;
        const float tc = x.F * ip;
        const float tb = x.B * __builtin_amdgcn_rcpf(S.cf.bw[3]);
        r = tc > tb ? tc : tb;
    }
    T[i] = r;
}

template <int VEC, int BLOCK>
static void predict_t(const DescPtrs& d, int64_t n, const Set& S, float* T, int32_t* occ,
                      hipStream_t stream)
{
    const int64_t threads = (n + VEC - 1) / VEC;
    const int64_t blocks = (threads + BLOCK - 1) / BLOCK;
    k_predict<VEC, BLOCK><<<dim3((unsigned)blocks), dim3(BLOCK), 0, stream>>>(d, n, S, T, occ);
}

template <int VEC>
static bool predict_v(int block, const DescPtrs& d, int64_t n, const Set& S, float* T,
                      int32_t* occ, hipStream_t stream)
{
    switch (block) {
    case 64: predict_t<VEC, 64>(d, n, S, T, occ, stream); return true;
    case 128: predict_t<VEC, 128>(d, n, S, T, occ, stream); return true;
    case 256: predict_t<VEC, 256>(d, n, S, T, occ, stream); return true;
    case 512: predict_t<VEC, 512>(d, n, S, T, occ, stream); return true;
    default: return false;
    }
}

hipError_t launch_predict(const DescPtrs& d, int64_t n, const Set& S, float* T, int32_t* occ,
                          bool vec_ok, const LaunchCfg& cfg, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int vec = vec_ok ? cfg.vec : 1;
    bool ok = false;
    switch (vec) {
    case 1: ok = predict_v<1>(cfg.block, d, n, S, T, occ, stream); break;
    case 2: ok = predict_v<2>(cfg.block, d, n, S, T, occ, stream); break;
    case 4: ok = predict_v<4>(cfg.block, d, n, S, T, occ, stream); break;
    case 8: ok = predict_v<8>(cfg.block, d, n, S, T, occ, stream); break;
    }
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_roofline(const DescPtrs& d, int64_t n, const Set& S, float* T, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    k_roofline<<<dim3((unsigned)blocks), dim3(256), 0, stream>>>(d, n, S, T);
    return hipGetLastError();
}

// Weight of one descriptor's Jacobian row in the sum, and its loss term.
// mode 0: dL/dT supplied; mode 1: mean relative error against measured m.
// Returns false if the descriptor does not contribute.
template <int MODE, typename R>
__device__ inline bool weight_of(R T, float wi, double& w, double& loss_term)
{
    if (MODE == 1) {
        if (!(wi > 0.0f && wi < __builtin_huge_valf())) return false;
        // 1/m: float32 reciprocal refined by one float64 Newton step (~1e-14)
        const double m = wi, r0 = (double)__builtin_amdgcn_rcpf(wi);
        const double im = r0 * (2.0 - m * r0), Td = (double)T;
        loss_term = __builtin_fabs(Td - m) * im;
        w = Td > m ? im : (Td < m ? -im : 0.0);
    } else {
        w = wi;
        loss_term = 0.0;
    }
    return true;
}

// Phase 1, float32: accumulate the descriptor's contribution unless it lies
// within 1e-5 of a max/min switch or (mode 1) of T = m; those return true and
// are left to the float64 pass.
template <int MODE>
__device__ inline bool grad_fast(const Set& S, const Desc<float>& x, float wi, double* acc)
{
    Eval<float> E;
    evaluate<float, true>(S.st, S.cf, x, E);
    if (!(E.T < __builtin_huge_valf())) return false;  // invalid (NaN) or infeasible (+inf)
    bool redo = E.near_kink;
    if (MODE == 1 && wi > 0.0f && wi < __builtin_huge_valf()) {
        const float rho = E.T * __builtin_amdgcn_rcpf(wi) - 1.0f;
        redo = redo || (__builtin_fabsf(rho) <= 1e-5f);
    }
    if (redo) return true;
    double w, lt;
    if (!weight_of<MODE>(E.T, wi, w, lt)) return false;
    if (MODE == 1) {
        acc[0] += lt;
        acc[1] += 1.0;
    }
    accumulate_partials<float, double>(S.st, S.cf, E, w, acc);
    return false;
}

// Phase 2, float64: the full contribution of a flagged descriptor.
template <int MODE>
__device__ inline void grad_exact(const Set& S, const Desc<float>& x, float wi, double* acc)
{
    Eval<double> D;
    evaluate<double, true>(S.st, S.cd, widen(x), D);
    if (!(D.T < __builtin_huge_val())) return;
    double w, lt;
    if (!weight_of<MODE>(D.T, wi, w, lt)) return;
    if (MODE == 1) {
        acc[0] += lt;
        acc[1] += 1.0;
    }
    accumulate_partials<double, double>(S.st, S.cd, D, w, acc);
}

// Phase 1 sweep.  The loop runs over wave-aligned groups of 64 consecutive
// descriptors so that every group's redo flags leave as one 64-bit ballot
// word, written exactly once (no clearing needed, order fixed).
template <int MODE, bool PTR, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_grad(DescPtrs d, int64_t n, const float* __restrict__ wv,
                                               Set sv, const Set* __restrict__ sp,
                                               double* __restrict__ partials,
                                               uint64_t* __restrict__ flags)
{
    __shared__ double red[16 * kAcc];
    const Set& S = PTR ? *sp : sv;
    double acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    // software pipeline: the next group's loads are in flight while this
    // group is evaluated
    int64_t base = (int64_t)blockIdx.x * BLOCK + (threadIdx.x & ~63);
    Desc<float> xn;
    float wn = 0.0f;
    if (base + lane < n) {
        xn = load_desc(d, base + lane);
        wn = ntload(wv + base + lane);
    }
    for (; base < n; base += stride) {
        const int64_t i = base + lane;
        const Desc<float> x = xn;
        const float w = wn;
        const int64_t inext = i + stride;
        if (inext < n) {
            xn = load_desc(d, inext);
            wn = ntload(wv + inext);
        }
        bool redo = false;
        if (i < n) redo = grad_fast<MODE>(S, x, w, acc);
        const uint64_t m = __ballot(redo);
        if (lane == 0) flags[base >> 6] = m;
    }
    block_reduce_acc(acc, red, partials + (int64_t)blockIdx.x * kAcc);
}

// Phase 2: (a) block b first folds the phase-1 partial rows b, b + nb2, ...
// (fixed order), so the final single-block reduction only sees nb2 rows;
// (b) it re-evaluates in float64 every descriptor flagged in its flag words.
template <int MODE, bool PTR>
__global__ __launch_bounds__(256) void k_grad_redo(DescPtrs d, int64_t n,
                                                    const float* __restrict__ wv, Set sv,
                                                    const Set* __restrict__ sp,
                                                    const uint64_t* __restrict__ flags,
                                                    const double* __restrict__ rows1, int nrows1,
                                                    double* __restrict__ rows2)
{
    __shared__ double red[16 * kAcc];
    const Set& S = PTR ? *sp : sv;
    double acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
    for (int r = blockIdx.x + gridDim.x * threadIdx.x; r < nrows1; r += gridDim.x * blockDim.x) {
#pragma unroll
        for (int j = 0; j < kAcc; ++j) acc[j] += rows1[(int64_t)r * kAcc + j];
    }
    const int64_t nwords = (n + 63) >> 6;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; wi < nwords; wi += stride) {
        uint64_t m = flags[wi];
        while (m) {
            const int bit = __builtin_ctzll(m);
            m &= m - 1;
            const int64_t i = (wi << 6) + bit;
            grad_exact<MODE>(S, load_desc(d, i), wv[i], acc);
        }
    }
    block_reduce_acc(acc, red, rows2 + (int64_t)blockIdx.x * kAcc);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ partials, int rows,
                                                 double* __restrict__ out)
{
    __shared__ double red[16 * kAcc];
    __shared__ double tot[kAcc];
    reduce_partials(partials, rows, kAcc, red, tot);
    if (threadIdx.x < kAcc) {
        if (MODE == 1) {
            const double c = tot[1];
            const double v = tot[threadIdx.x];
            out[threadIdx.x] = (threadIdx.x == 1 || c == 0.0) ? v : v / c;
        } else if (threadIdx.x >= 2) {
            out[threadIdx.x - 2] = tot[threadIdx.x];
        }
    }
}

hipError_t launch_reduce(int mode, const double* partials, int rows, double* out, hipStream_t stream)
{
    if (mode == 1) k_reduce<1><<<1, 256, 0, stream>>>(partials, rows, out);
    else k_reduce<0><<<1, 256, 0, stream>>>(partials, rows, out);
    return hipGetLastError();
}

GradLayout grad_layout(int64_t n)
{
    GradLayout L;
    int64_t b = (n + 63) / 64;
    L.nb = (int)(b < 1 ? 1 : (b > kGradMaxBlocks ? kGradMaxBlocks : b));
    L.nwords = (n + 63) / 64;
    int64_t b2 = (L.nwords + 255) / 256;
    L.nb2 = (int)(b2 < 1 ? 1 : (b2 > kRedoMaxBlocks ? kRedoMaxBlocks : b2));
    return L;
}

// Blocks of 256 threads that are resident at once on the current device for
// a kernel (occupancy x compute units), cached per device and kernel.  A
// persistent grid of exactly this size has no second, half-empty round.
int resident_blocks(const void* kernel, int block)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_pair(dev, kernel);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1;
    int r = per_cu * cus;
    r = r < 1 ? 1 : r;
    cache[key] = r;
    return r;
}

template <int MODE, bool PTR, int BLOCK>
static int grad_grid_t(int64_t n, int grid_mult)
{
    const GradLayout L = grad_layout(n);
    const int64_t want = (n + BLOCK - 1) / BLOCK;
    int64_t r = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_grad<MODE, PTR, BLOCK>), BLOCK) *
                (grid_mult < 1 ? 1 : grid_mult);
    r = r < want ? r : want;
    r = r < L.nb ? r : L.nb;
    return (int)(r < 1 ? 1 : r);
}

template <int MODE, bool PTR>
static int grad_grid_b(int64_t n, const LaunchCfg& c)
{
    switch (c.block) {
    case 64: return grad_grid_t<MODE, PTR, 64>(n, c.grid_mult);
    case 128: return grad_grid_t<MODE, PTR, 128>(n, c.grid_mult);
    case 512: return grad_grid_t<MODE, PTR, 512>(n, c.grid_mult);
    default: return grad_grid_t<MODE, PTR, 256>(n, c.grid_mult);
    }
}

int grad_grid(int mode, bool ptr, int64_t n, const LaunchCfg& c)
{
    if (mode == 1) return ptr ? grad_grid_b<1, true>(n, c) : grad_grid_b<1, false>(n, c);
    return ptr ? grad_grid_b<0, true>(n, c) : grad_grid_b<0, false>(n, c);
}

template <int MODE, bool PTR>
static bool launch_grad_t(const DescPtrs& d, int64_t n, const float* w, const Set& S,
                          const Set* S_dev, double* partials, uint64_t* flags, int nb,
                          const GradLayout& L, const LaunchCfg& c, hipStream_t stream)
{
    switch (c.block) {
    case 64: k_grad<MODE, PTR, 64><<<nb, 64, 0, stream>>>(d, n, w, S, S_dev, partials, flags); break;
    case 128: k_grad<MODE, PTR, 128><<<nb, 128, 0, stream>>>(d, n, w, S, S_dev, partials, flags); break;
    case 256: k_grad<MODE, PTR, 256><<<nb, 256, 0, stream>>>(d, n, w, S, S_dev, partials, flags); break;
    case 512: k_grad<MODE, PTR, 512><<<nb, 512, 0, stream>>>(d, n, w, S, S_dev, partials, flags); break;
    default: return false;
    }
    k_grad_redo<MODE, PTR><<<L.nb2, 256, 0, stream>>>(d, n, w, S, S_dev, flags, partials, nb,
                                                       partials + (int64_t)nb * kAcc);
    return true;
}

hipError_t launch_grad(int mode, const DescPtrs& d, int64_t n, const float* w, const Set& S,
                       const Set* S_dev, double* partials, uint64_t* flags, const GradLayout& L,
                       const LaunchCfg& c, double* out, hipStream_t stream)
{
    const int nb = grad_grid(mode, S_dev != nullptr, n, c);
    bool ok;
    if (mode == 1)
        ok = S_dev ? launch_grad_t<1, true>(d, n, w, S, S_dev, partials, flags, nb, L, c, stream)
                   : launch_grad_t<1, false>(d, n, w, S, S_dev, partials, flags, nb, L, c, stream);
    else
        ok = S_dev ? launch_grad_t<0, true>(d, n, w, S, S_dev, partials, flags, nb, L, c, stream)
                   : launch_grad_t<0, false>(d, n, w, S, S_dev, partials, flags, nb, L, c, stream);
    if (!ok) return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !out) return e;
    if (mode == 1)
        k_reduce<1><<<1, 256, 0, stream>>>(partials + (int64_t)nb * kAcc, L.nb2, out);
    else
        k_reduce<0><<<1, 256, 0, stream>>>(partials + (int64_t)nb * kAcc, L.nb2, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// device Adam on log(theta)
// ---------------------------------------------------------------------------
__device__ inline void adam_update(CalibState* st, const double* tot, const AdamOpts& o, Set* S,
                                   double* loss_hist)
{
    if (threadIdx.x != 0) return;
    if (adam_theta_step(st, tot, o, loss_hist)) {
        make_const<float>(st->theta, S->st, S->cf);
        make_const<double>(st->theta, S->st, S->cd);
    }
}

__global__ __launch_bounds__(256) void k_adam(const double* __restrict__ partials, int rows,
                                               CalibState* st, AdamOpts o, Set* S,
                                               double* loss_hist)
{
    __shared__ double red[16 * kAcc];
    __shared__ double tot[kAcc];
    reduce_partials(partials, rows, kAcc, red, tot);
    adam_update(st, tot, o, S, loss_hist);
}

hipError_t launch_adam(const double* partials, int rows, CalibState* st, const AdamOpts& o, Set* S,
                       double* loss_hist, hipStream_t stream)
{
    k_adam<<<1, 256, 0, stream>>>(partials, rows, st, o, S, loss_hist);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// multi-set calibration sweep: one persistent launch over a (set, chunk)
// work list; per-block, per-set sums staged in LDS
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_grad_batched(const DescPtrs* __restrict__ sets,
                                                       const float* const* __restrict__ meas,
                                                       const Set* __restrict__ S_all,
                                                       const WorkItem* __restrict__ items,
                                                       int n_items, int n_sets,
                                                       const int64_t* __restrict__ flag_off,
                                                       uint64_t* __restrict__ flags,
                                                       double* __restrict__ partials)
{
    __shared__ double red[16 * kAcc];
    __shared__ double tot[kAcc];
    __shared__ double per_set[kMaxSets * kAcc];
    for (int j = threadIdx.x; j < n_sets * kAcc; j += blockDim.x) per_set[j] = 0.0;
    __syncthreads();
    const int b = blockIdx.x, nb = gridDim.x;
    const int it0 = (int)((int64_t)n_items * b / nb);
    const int it1 = (int)((int64_t)n_items * (b + 1) / nb);
    const int lane = threadIdx.x & 63;
    int cur = -1;
    double acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
    for (int it = it0; it < it1; ++it) {
        const WorkItem w = items[it];
        if (w.set != cur) {
            if (cur >= 0) {
                block_reduce_acc(acc, red, tot);
                if (threadIdx.x < kAcc) per_set[cur * kAcc + threadIdx.x] += tot[threadIdx.x];
                __syncthreads();
#pragma unroll
                for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
            }
            cur = w.set;
        }
        const DescPtrs d = sets[w.set];
        const float* m = meas[w.set];
        const Set& S = S_all[w.set];
        uint64_t* fl = flags + flag_off[w.set];
        // items start at multiples of 64, so each wave covers whole flag words
        for (int64_t base = w.begin + (threadIdx.x & ~63); base < w.end; base += blockDim.x) {
            const int64_t i = base + lane;
            bool redo = false;
            if (i < w.end) redo = grad_fast<1>(S, load_desc(d, i), ntload(m + i), acc);
            const uint64_t msk = __ballot(redo);
            if (lane == 0) fl[base >> 6] = msk;
        }
    }
    if (cur >= 0) {
        block_reduce_acc(acc, red, tot);
        if (threadIdx.x < kAcc) per_set[cur * kAcc + threadIdx.x] += tot[threadIdx.x];
        __syncthreads();
    }
    for (int j = threadIdx.x; j < n_sets * kAcc; j += blockDim.x)
        partials[(int64_t)b * n_sets * kAcc + j] = per_set[j];
}

// Phase 2 for every set in turn (set loop uniform; fixed order): fold the
// phase-1 rows b, b + nb2, ... of the set, then re-evaluate its flagged
// descriptors in float64.
__global__ __launch_bounds__(256) void k_grad_redo_batched(const DescPtrs* __restrict__ sets,
                                                            const float* const* __restrict__ meas,
                                                            const Set* __restrict__ S_all,
                                                            const int64_t* __restrict__ set_n,
                                                            const int64_t* __restrict__ flag_off,
                                                            const uint64_t* __restrict__ flags,
                                                            int n_sets,
                                                            const double* __restrict__ rows1,
                                                            int nrows1,
                                                            double* __restrict__ partials)
{
    __shared__ double red[16 * kAcc];
    __shared__ double tot[kAcc];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int s = 0; s < n_sets; ++s) {
        double acc[kAcc];
#pragma unroll
        for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
        for (int r = blockIdx.x + gridDim.x * threadIdx.x; r < nrows1; r += gridDim.x * blockDim.x) {
            const double* row = rows1 + ((int64_t)r * n_sets + s) * kAcc;
#pragma unroll
            for (int j = 0; j < kAcc; ++j) acc[j] += row[j];
        }
        const DescPtrs d = sets[s];
        const float* m = meas[s];
        const Set& S = S_all[s];
        const uint64_t* fl = flags + flag_off[s];
        const int64_t nwords = (set_n[s] + 63) >> 6;
        for (int64_t wi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; wi < nwords; wi += stride) {
            uint64_t mk = fl[wi];
            while (mk) {
                const int bit = __builtin_ctzll(mk);
                mk &= mk - 1;
                const int64_t i = (wi << 6) + bit;
                grad_exact<1>(S, load_desc(d, i), m[i], acc);
            }
        }
        block_reduce_acc(acc, red, tot);
        if (threadIdx.x < kAcc)
            partials[((int64_t)blockIdx.x * n_sets + s) * kAcc + threadIdx.x] = tot[threadIdx.x];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_adam_batched(const double* __restrict__ partials, int rows,
                                                       int n_sets, CalibState* st,
                                                       const AdamOpts* __restrict__ opts,
                                                       Set* S_all, int steps, double* loss_hist)
{
    __shared__ double red[16 * kAcc];
    __shared__ double tot[kAcc];
    const int s = blockIdx.x;
    reduce_partials(partials + s * kAcc, rows, n_sets * kAcc, red, tot);
    adam_update(st + s, tot, opts[s], S_all + s,
                loss_hist ? loss_hist + (int64_t)s * steps : nullptr);
}

int batched_grid(int n_items, int grid_mult)
{
    const int r = resident_blocks(reinterpret_cast<const void*>(&k_grad_batched), 256) *
                  (grid_mult < 1 ? 1 : grid_mult);
    const int m = n_items < kGradMaxBlocks ? n_items : kGradMaxBlocks;
    return m < 1 ? 1 : (r < m ? r : m);
}

hipError_t launch_grad_batched(const DescPtrs* sets, const float* const* meas, const Set* S_all,
                               const WorkItem* items, int n_items, int n_sets,
                               const int64_t* set_n, const int64_t* flag_off, uint64_t* flags,
                               int64_t total_words, double* partials, int nb, int nb2,
                               hipStream_t stream)
{
    k_grad_batched<<<nb, 256, 0, stream>>>(sets, meas, S_all, items, n_items, n_sets, flag_off,
                                           flags, partials);
    (void)total_words;
    k_grad_redo_batched<<<nb2, 256, 0, stream>>>(sets, meas, S_all, set_n, flag_off, flags, n_sets,
                                                 partials, nb,
                                                 partials + (int64_t)nb * n_sets * kAcc);
    return hipGetLastError();
}

hipError_t launch_adam_batched(const double* partials, int rows, int n_sets, CalibState* st,
                               const AdamOpts* opts, Set* S_all, int steps, double* loss_hist,
                               hipStream_t stream)
{
    k_adam_batched<<<n_sets, 256, 0, stream>>>(partials, rows, n_sets, st, opts, S_all, steps,
                                                loss_hist);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// tile selection
// ---------------------------------------------------------------------------
// GEMM tile -> descriptor (integers exact in 64 bits; F, B rounded to R)
template <typename R>
__device__ inline bool derive_tile(int32_t M, int32_t N, int32_t Kd, int32_t t, uint32_t code,
                                   int wave_shift, Desc<R>& x)
{
    const uint32_t kdc = (code >> 4) & 3u;
    if ((code >> 9) != 0u || kdc == 3u || M < 1 || N < 1 || Kd < 1 || t < 0 || t > 3) return false;
    // tile sizes are powers of two: the ceiling divisions are shifts
    const uint32_t lmt = 5u + (code & 3u), lnt = 5u + ((code >> 2) & 3u), lkd = 4u + kdc;
    const int64_t mt = 1ll << lmt, nt = 1ll << lnt, kd = 1ll << lkd;
    const int64_t wpw = ((code >> 6) & 7u) + 1;
    const int64_t e = 8 >> t;                 // 8, 4, 2, 1 bytes
    const int64_t eo = t == 3 ? 2 : e;        // fp8 writes 16-bit results
    const int64_t acc = t == 0 ? 2 : 1;
    const int64_t gm = ((int64_t)M + mt - 1) >> lmt, gn = ((int64_t)N + nt - 1) >> lnt;
    const int64_t G = gm * gn, Ks = ((int64_t)Kd + kd - 1) >> lkd;
    const int64_t g = wpw << wave_shift;
    if (G > 0x7fffffffll || g > 1024) return false;
    const int64_t Fi = 2 * (gm * mt) * (gn * nt) * (Ks * kd);
    const int64_t Bi = G * Ks * (mt + nt) * kd * e + (int64_t)M * N * eo;
    const int64_t Ui = ((int64_t)M * Kd + (int64_t)Kd * N) * e + (int64_t)M * N * eo;
    x.F = (R)Fi;
    x.B = (R)Bi;
    const R r2 = (R)1 - (R)Ui * Ar<R>::rcp((R)Bi);
    x.r2 = r2 > (R)0 ? r2 : (R)0;
    x.r1 = (R)0;
    x.r3 = (R)0;
    x.K = (R)Ks;
    x.u = (R)1;
    x.W = (R)0;
    // VGPRs: accumulators and the panel share per thread (numerators below
    // 2^19, divisors at most 4096: exact float-reciprocal quotients)
    const uint32_t ga = (uint32_t)g;
    x.v = (int32_t)(udiv_small((uint32_t)(mt * nt * acc) + ga - 1u, ga) +
                    udiv_small((uint32_t)((mt + nt) * kd * e) + 4u * ga - 1u, 4u * ga) + 16u);
    x.s = (int32_t)(2 * (mt + nt) * kd * e);
    x.gp = (int32_t)g | (t << 11);
    x.G = (int32_t)G;
    return true;
}

template <typename R> __device__ inline const Const<R>& cst(const Set& S);
template <> __device__ inline const Const<float>& cst<float>(const Set& S) { return S.cf; }
template <> __device__ inline const Const<double>& cst<double>(const Set& S) { return S.cd; }

// cost of one candidate; invalid codes and infeasible tiles cost +inf
template <typename R>
__device__ inline R tile_cost(const Set& S, int32_t M, int32_t N, int32_t K, int32_t t, uint32_t code)
{
    const R inf = (R)__builtin_huge_val();
    Desc<R> x;
    if (!derive_tile<R>(M, N, K, t, code, S.st.wave_shift, x)) return inf;
    Eval<R> E;
    evaluate<R, false>(S.st, cst<R>(S), x, E);
    return E.T == E.T ? E.T : inf;
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, m, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Orders this wave's LDS stores before its later LDS loads from other lanes
// (the LDS executes one wave's operations in issue order; the fences keep
// the compiler from moving accesses across this point).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// float64 minimum, its lowest local index and the second-smallest value of
// a multiset, accumulated in candidate order (exact ties keep the first)
struct Best2 {
    double c1, c2;
    int32_t j1;
    __device__ inline void add(double cd, int32_t jl)
    {
        if (cd < c1 || (cd == c1 && jl < j1)) {
            c2 = c1;
            c1 = cd;
            j1 = jl;
        } else if (cd < c2) {
            c2 = cd;
        }
    }
};

__device__ inline void write_best(const Best2& r, int64_t i, int32_t* best, double* best_cost,
                                  uint8_t* near_tie)
{
    const double dinf = __builtin_huge_val();
    const bool fin = r.c1 < dinf;
    best[i] = fin ? r.j1 : -1;
    best_cost[i] = r.c1;
    near_tie[i] = (fin && r.c2 < dinf && (r.c2 - r.c1) <= 1e-6 * r.c1) ? 1 : 0;
}

constexpr int kTileQueue = 128;   // queued float64 window candidates per wave
constexpr int kTileSlots = 64;    // shapes per queue (one lane each at the end)

// Per-wave queue of float64 window re-evaluations, shared across shapes.
struct TileQueue {
    int32_t M[kTileSlots], N[kTileSlots], K[kTileSlots], t[kTileSlots];
    int32_t first[kTileSlots];       // first entry of each slot
    int64_t shape[kTileSlots];
    uint32_t key[kTileQueue];        // slot << 8 | local candidate index
    uint32_t code[kTileQueue];
    double cost[kTileQueue];
};

// Evaluates every queued candidate in float64 with all lanes, then one lane
// per shape scans that shape's entries (ascending candidate index) and
// writes its result.  Wave-uniform ns, qn.
__device__ inline void flush_tiles(TileQueue& q, int ns, int qn, const Set& S, int lane,
                                   int32_t* best, double* best_cost, uint8_t* near_tie)
{
    wave_lds_sync();
    for (int e = lane; e < qn; e += 64) {
        const int sl = (int)(q.key[e] >> 8);
        q.cost[e] = tile_cost<double>(S, q.M[sl], q.N[sl], q.K[sl], q.t[sl], q.code[e]);
    }
    wave_lds_sync();
    if (lane < ns) {
        const int e1 = lane + 1 < ns ? q.first[lane + 1] : qn;
        Best2 r{__builtin_huge_val(), __builtin_huge_val(), 0x7fffffff};
        for (int e = q.first[lane]; e < e1; ++e) r.add(q.cost[e], (int32_t)(q.key[e] & 0xffu));
        write_best(r, q.shape[lane], best, best_cost, near_tie);
    }
    wave_lds_sync();   // the queue is refilled next
}

// One wave per shape (persistent over shapes).  Pass 1 takes the float32
// minimum with a packed (cost bits, local index) key.  Every candidate whose
// float32 cost is within kTileWindow of that minimum is re-evaluated in
// float64; the result per shape is the smallest float64 cost (the lowest
// index winning exact ties) and the second-smallest, for the near-tie flag.
// Lists of up to 128 candidates keep their float32 costs and codes in
// registers and queue their window candidates, so that the float64 work of
// many shapes runs on all lanes at once; longer lists re-evaluate their
// window directly, lane-parallel.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_select_tile(ShapePtrs sh, const int32_t* __restrict__ off,
                                                      const uint32_t* __restrict__ code, int64_t n,
                                                      int64_t n_cand,
                                                      Set S, int32_t* __restrict__ best,
                                                      double* __restrict__ best_cost,
                                                      uint8_t* __restrict__ near_tie)
{
    __shared__ TileQueue queues[BLOCK / 64];
    const int lane = threadIdx.x & 63;
    TileQueue& q = queues[threadIdx.x >> 6];
    const int wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * BLOCK + threadIdx.x) >> 6));
    const int nwaves = (int)((gridDim.x * BLOCK) >> 6);
    const double dinf = __builtin_huge_val();
    const float finf = __builtin_huge_valf();
    int ns = 0, qn = 0;
    for (int64_t i = wave; i < n; i += nwaves) {
        const int32_t M = sh.M[i], N = sh.N[i], K = sh.K[i], t = sh.dtype[i];
        // offsets are caller data: clamp them into the candidate array
        int64_t a = off[i], b = off[i + 1];
        a = a < 0 ? 0 : (a > n_cand ? n_cand : a);
        b = b < a ? a : (b > n_cand ? n_cand : b);
        float cc0 = finf, cc1 = finf;
        uint32_t cd0 = 0, cd1 = 0;
        uint64_t key = ~0ull;
        for (int64_t j = a + lane, r = 0; j < b; j += 64, ++r) {
            const uint32_t cj = code[j];
            const float c = tile_cost<float>(S, M, N, K, t, cj);
            cc0 = r == 0 ? c : cc0;
            cc1 = r == 1 ? c : cc1;
            cd0 = r == 0 ? cj : cd0;
            cd1 = r == 1 ? cj : cd1;
            const uint64_t k = ((uint64_t)__float_as_uint(c) << 32) | (uint32_t)(j - a);
            key = k < key ? k : key;
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            const uint64_t o = shfl_xor_u64(key, m);
            key = o < key ? o : key;
        }
        const float c32 = __uint_as_float((uint32_t)(key >> 32));
        if (key == ~0ull || !(c32 < finf)) {
            if (lane == 0) {
                best[i] = -1;
                best_cost[i] = dinf;
                near_tie[i] = 0;
            }
            continue;
        }
        const float thr = c32 * (1.0f + kTileWindow);
        if (b - a <= 128) {
            // lanes past the list hold +inf, which a +inf threshold would admit
            const int64_t len = b - a;
            const bool w0 = lane < len && cc0 <= thr, w1 = 64 + lane < len && cc1 <= thr;
            const uint64_t m0 = __ballot(w0), m1 = __ballot(w1);
            const int n0 = __popcll(m0), cnt = n0 + __popcll(m1);
            if (qn + cnt > kTileQueue || ns == kTileSlots) {
                flush_tiles(q, ns, qn, S, lane, best, best_cost, near_tie);
                ns = 0;
                qn = 0;
            }
            if (lane == 0) {
                q.M[ns] = M;
                q.N[ns] = N;
                q.K[ns] = K;
                q.t[ns] = t;
                q.first[ns] = qn;
                q.shape[ns] = i;
            }
            const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m0 >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)m0, 0u));
            const uint32_t below1 = __builtin_amdgcn_mbcnt_hi((uint32_t)(m1 >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m1, 0u));
            if (w0) {
                const int e = qn + (int)below;
                q.key[e] = ((uint32_t)ns << 8) | (uint32_t)lane;
                q.code[e] = cd0;
            }
            if (w1) {
                const int e = qn + n0 + (int)below1;
                q.key[e] = ((uint32_t)ns << 8) | (uint32_t)(64 + lane);
                q.code[e] = cd1;
            }
            qn += cnt;
            ++ns;
            continue;
        }
        Best2 r{dinf, dinf, 0x7fffffff};
        for (int64_t j = a + lane, rr = 0; j < b; j += 64, ++rr) {
            const float c = rr == 0 ? cc0 : (rr == 1 ? cc1 : tile_cost<float>(S, M, N, K, t, code[j]));
            if (!(c <= thr)) continue;
            r.add(tile_cost<double>(S, M, N, K, t, code[j]), (int32_t)(j - a));
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            const double oc1 = __shfl_xor(r.c1, m, 64);
            const double oc2 = __shfl_xor(r.c2, m, 64);
            const int32_t oj1 = __shfl_xor(r.j1, m, 64);
            if (oc1 < r.c1 || (oc1 == r.c1 && oj1 < r.j1)) {
                r.c2 = r.c1 < oc2 ? r.c1 : oc2;
                r.c1 = oc1;
                r.j1 = oj1;
            } else {
                r.c2 = oc1 < r.c2 ? oc1 : r.c2;
            }
        }
        if (lane == 0) write_best(r, i, best, best_cost, near_tie);
    }
    if (ns > 0) flush_tiles(q, ns, qn, S, lane, best, best_cost, near_tie);
}

template <int BLOCK>
static void select_t(const ShapePtrs& sh, const int32_t* off, const uint32_t* code, int64_t n,
                     int64_t n_cand, const Set& S, int32_t* best, double* best_cost,
                     uint8_t* near_tie, int grid_mult, hipStream_t stream)
{
    const int64_t waves_per_block = BLOCK / 64;
    const int64_t want = (n + waves_per_block - 1) / waves_per_block;
    int64_t b = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_select_tile<BLOCK>), BLOCK) *
                (grid_mult < 1 ? 1 : grid_mult);
    b = b < want ? b : want;
    k_select_tile<BLOCK><<<(int)(b < 1 ? 1 : b), BLOCK, 0, stream>>>(sh, off, code, n, n_cand, S, best,
                                                                     best_cost, near_tie);
}

hipError_t launch_select_tile(const ShapePtrs& sh, const int32_t* off, const uint32_t* code,
                              int64_t n, int64_t n_cand, const Set& S, int32_t* best,
                              double* best_cost, uint8_t* near_tie, const LaunchCfg& c,
                              hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    switch (c.block) {
    case 64: select_t<64>(sh, off, code, n, n_cand, S, best, best_cost, near_tie, c.grid_mult, stream); break;
    case 128: select_t<128>(sh, off, code, n, n_cand, S, best, best_cost, near_tie, c.grid_mult, stream); break;
    case 256: select_t<256>(sh, off, code, n, n_cand, S, best, best_cost, near_tie, c.grid_mult, stream); break;
    case 512: select_t<512>(sh, off, code, n, n_cand, S, best, best_cost, near_tie, c.grid_mult, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wm
