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
// GEMM tile -> descriptor.  Tile sizes are powers of two, so the grid, the
// K steps and the panel sizes are shifts of 32-bit integers (every padded
// extent is below 2^32).  Flops and bytes are real quantities formed in R
// from those exact integers: in double they are exact while below 2^53 and
// never overflow; in float they carry a few ulps, which the float64 window
// of the selection absorbs.
template <typename R>
__device__ inline bool derive_tile(int32_t M, int32_t N, int32_t Kd, int32_t t, uint32_t code,
                                   int wave_shift, Desc<R>& x)
{
#pragma clang fp contract(off)
    const uint32_t kdc = (code >> 4) & 3u;
    if ((code >> 9) != 0u || kdc == 3u || M < 1 || N < 1 || Kd < 1 || t < 0 || t > 3) return false;
    const uint32_t lmt = 5u + (code & 3u), lnt = 5u + ((code >> 2) & 3u), lkd = 4u + kdc;
    const uint32_t wpw = ((code >> 6) & 7u) + 1u;
    const uint32_t le = 3u - (uint32_t)t;          // element bytes 8, 4, 2, 1
    const uint32_t eo = t == 3 ? 2u : (1u << le);  // fp8 writes 16-bit results
    const uint32_t acc = t == 0 ? 2u : 1u;
    const uint32_t gm = ((uint32_t)M + (1u << lmt) - 1u) >> lmt;
    const uint32_t gn = ((uint32_t)N + (1u << lnt) - 1u) >> lnt;
    const uint32_t Ks = ((uint32_t)Kd + (1u << lkd) - 1u) >> lkd;
    const uint64_t G = (uint64_t)gm * gn;
    const uint32_t g = wpw << wave_shift;
    if (G > 0x7fffffffull || g > 1024u) return false;
    const uint32_t pan = ((1u << lmt) + (1u << lnt)) << (lkd + le);   // (mt + nt) kd e <= 2^18
    const R fM = (R)(uint32_t)M, fN = (R)(uint32_t)N, fK = (R)(uint32_t)Kd;
    const R Bi = (R)(uint32_t)G * (R)Ks * (R)pan + fM * fN * (R)eo;
    const R Ui = (fM * fK + fK * fN) * (R)(1u << le) + fM * fN * (R)eo;
    x.F = (R)2 * (R)(gm << lmt) * (R)(gn << lnt) * (R)(Ks << lkd);
    x.B = Bi;
    const R r2 = (R)1 - Ui * Ar<R>::rcp(Bi);
    x.r2 = r2 > (R)0 ? r2 : (R)0;
    x.r1 = (R)0;
    x.r3 = (R)0;
    x.K = (R)Ks;
    x.u = (R)1;
    x.W = (R)0;
    // VGPRs: accumulators and the panel share per thread (numerators below
    // 2^19, divisors at most 4096: exact float-reciprocal quotients)
    x.v = (int32_t)(udiv_small((acc << (lmt + lnt)) + g - 1u, g) +
                    udiv_small(pan + 4u * g - 1u, 4u * g) + 16u);
    x.s = (int32_t)(2u * pan);
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

constexpr int kTileQueue = 256;   // queued float64 window candidates per wave
constexpr int kTileSlots = 64;    // shapes per queue (one lane each at the end)
constexpr int kTileBatch = 8;     // consecutive shapes whose candidates share wavefronts
constexpr int kTileRounds = 12;   // 64-candidate rounds a batch keeps in registers

// Per-wave queue of float64 window re-evaluations, shared across shapes.
// Entries are appended in (slot, local index) order.
struct TileQueue {
    int32_t M[kTileSlots], N[kTileSlots], K[kTileSlots], t[kTileSlots];
    int64_t shape[kTileSlots];
    uint32_t key[kTileQueue];        // slot << 24 | local candidate index
    uint32_t code[kTileQueue];
    double cost[kTileQueue];
    unsigned long long bmin[kTileBatch];   // packed float32 minimum per batch shape
};

__device__ inline uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// first entry in [0, qn) whose slot is >= sl
__device__ inline int first_entry(const TileQueue& q, int qn, uint32_t sl)
{
    int lo = 0, hi = qn;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((q.key[mid] >> 24) < sl) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Evaluates every queued candidate in float64 with all lanes, then one lane
// per shape scans that shape's entries (ascending candidate index) and
// writes its result.  Wave-uniform ns, qn.
__device__ inline void flush_tiles(TileQueue& q, int ns, int qn, const Set& S, int lane,
                                   int32_t* best, double* best_cost, uint8_t* near_tie)
{
    wave_lds_sync();
    for (int e = lane; e < qn; e += 64) {
        const int sl = (int)(q.key[e] >> 24);
        q.cost[e] = tile_cost<double>(S, q.M[sl], q.N[sl], q.K[sl], q.t[sl], q.code[e]);
    }
    wave_lds_sync();
    if (lane < ns) {
        const int e1 = first_entry(q, qn, (uint32_t)lane + 1u);
        Best2 r{__builtin_huge_val(), __builtin_huge_val(), 0x7fffffff};
        for (int e = first_entry(q, qn, (uint32_t)lane); e < e1; ++e)
            r.add(q.cost[e], (int32_t)(q.key[e] & 0xffffffu));
        write_best(r, q.shape[lane], best, best_cost, near_tie);
    }
    wave_lds_sync();   // the queue is refilled next
}

struct TileCtx {
    ShapePtrs sh;
    const int32_t* off;
    const uint32_t* code;
    int64_t n_cand;
    int32_t* best;
    double* best_cost;
    uint8_t* near_tie;
};

__device__ inline void clamp_list(int64_t n_cand, int64_t& a, int64_t& b)
{
    // offsets are caller data: clamp them into the candidate array
    a = a < 0 ? 0 : (a > n_cand ? n_cand : a);
    b = b < a ? a : (b > n_cand ? n_cand : b);
}

// One shape on the whole wave: float32 minimum over its list; lists of up to
// 128 candidates queue their float64 window, longer lists evaluate it here.
__device__ inline void shape_task(const TileCtx& C, const Set& S, TileQueue& q, int& ns, int& qn,
                                  int64_t i, int lane)
{
    const double dinf = __builtin_huge_val();
    const float finf = __builtin_huge_valf();
    const int32_t M = C.sh.M[i], N = C.sh.N[i], K = C.sh.K[i], t = C.sh.dtype[i];
    int64_t a = C.off[i], b = C.off[i + 1];
    clamp_list(C.n_cand, a, b);
    float cc0 = finf, cc1 = finf;
    uint32_t cd0 = 0, cd1 = 0;
    uint64_t key = ~0ull;
    for (int64_t j = a + lane, r = 0; j < b; j += 64, ++r) {
        const uint32_t cj = C.code[j];
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
            C.best[i] = -1;
            C.best_cost[i] = dinf;
            C.near_tie[i] = 0;
        }
        return;
    }
    const float thr = c32 * (1.0f + kTileWindow);
    const int64_t len = b - a;
    if (len <= 128) {
        // lanes past the list hold +inf, which a +inf threshold would admit
        const bool w0 = lane < len && cc0 <= thr, w1 = 64 + lane < len && cc1 <= thr;
        const uint64_t m0 = __ballot(w0), m1 = __ballot(w1);
        const int n0 = __popcll(m0), cnt = n0 + __popcll(m1);
        if (qn + cnt > kTileQueue || ns == kTileSlots) {
            flush_tiles(q, ns, qn, S, lane, C.best, C.best_cost, C.near_tie);
            ns = 0;
            qn = 0;
        }
        if (lane == 0) {
            q.M[ns] = M;
            q.N[ns] = N;
            q.K[ns] = K;
            q.t[ns] = t;
            q.shape[ns] = i;
        }
        if (w0) {
            const int e = qn + (int)lanes_below(m0);
            q.key[e] = ((uint32_t)ns << 24) | (uint32_t)lane;
            q.code[e] = cd0;
        }
        if (w1) {
            const int e = qn + n0 + (int)lanes_below(m1);
            q.key[e] = ((uint32_t)ns << 24) | (uint32_t)(64 + lane);
            q.code[e] = cd1;
        }
        qn += cnt;
        ++ns;
        return;
    }
    Best2 r{dinf, dinf, 0x7fffffff};
    for (int64_t j = a + lane, rr = 0; j < b; j += 64, ++rr) {
        const float c = rr == 0 ? cc0 : (rr == 1 ? cc1 : tile_cost<float>(S, M, N, K, t, C.code[j]));
        if (!(c <= thr)) continue;
        r.add(tile_cost<double>(S, M, N, K, t, C.code[j]), (int32_t)(j - a));
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
    if (lane == 0) write_best(r, i, C.best, C.best_cost, C.near_tie);
}

// kTileBatch consecutive shapes [s0, s0 + kTileBatch) on one wave with their
// candidate lists laid end to end over the lanes, so that short lists do not
// leave lanes idle.  Batches of more than kTileRounds * 64 candidates, or
// whose float64 window would not fit the queue, go shape by shape instead.
__device__ inline void batch_task(const TileCtx& C, const Set& S, TileQueue& q, int& ns, int& qn,
                                  int64_t s0, int64_t n, int lane)
{
    constexpr int SB = kTileBatch;
    const float finf = __builtin_huge_valf();
    // lane k < SB holds shape s0 + k
    const int64_t si = s0 + lane;
    const bool has = lane < SB && si < n;
    int32_t M = 0, N = 0, K = 0, t = 0;
    int64_t a = 0, b = 0;
    if (has) {
        M = C.sh.M[si];
        N = C.sh.N[si];
        K = C.sh.K[si];
        t = C.sh.dtype[si];
        a = C.off[si];
        b = C.off[si + 1];
        clamp_list(C.n_cand, a, b);
    }
    // list lengths, saturated (a batch past kTileRounds * 64 goes shape by shape)
    constexpr int32_t cap = kTileRounds * 64 + 1;
    const int32_t len = (int32_t)(b - a < cap ? b - a : cap);
    int32_t inc = len;   // inclusive prefix over lanes 0..SB-1
#pragma unroll
    for (int d = 1; d < SB; d <<= 1) {
        const int32_t o = __shfl_up(inc, d, 64);
        inc += lane >= d ? o : 0;
    }
    const int32_t T = __builtin_amdgcn_readlane(inc, SB - 1);
    if (T > kTileRounds * 64) {
        for (int k = 0; k < SB && s0 + k < n; ++k) shape_task(C, S, q, ns, qn, s0 + k, lane);
        return;
    }
    const int32_t P = inc - len;   // first virtual position of lane's shape
    int32_t Pk[SB];
#pragma unroll
    for (int k = 0; k < SB; ++k) Pk[k] = __builtin_amdgcn_readlane(P, k);
    if (lane < SB) q.bmin[lane] = ~0ull;
    wave_lds_sync();
    // pass 1: float32 costs (kept in registers) and the per-shape minimum
    const int R = (T + 63) >> 6;
    float creg[kTileRounds];
    uint64_t sbits = 0;   // 3 bits of batch slot per round
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
        creg[r] = finf;
        if (r < R) {
            const int32_t v = r * 64 + lane;
            int32_t sl = 0;
#pragma unroll
            for (int k = 1; k < SB; ++k) sl += v >= Pk[k] ? 1 : 0;
            const int32_t Ms = __shfl(M, sl, 64), Ns = __shfl(N, sl, 64), Ks = __shfl(K, sl, 64);
            const int32_t ts = __shfl(t, sl, 64), Ps = __shfl(P, sl, 64);
            const int64_t as = __shfl(a, sl, 64);
            sbits |= (uint64_t)sl << (3 * r);
            if (v < T) {
                const int32_t jl = v - Ps;
                const float c = tile_cost<float>(S, Ms, Ns, Ks, ts, C.code[as + jl]);
                creg[r] = c;
                __hip_atomic_fetch_min(&q.bmin[sl],
                                       ((unsigned long long)__float_as_uint(c) << 32) | (uint32_t)jl,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
        }
    }
    wave_lds_sync();
    // per shape: threshold, or the empty result when nothing is feasible
    float thr = -finf;
    bool fin = false;
    if (has) {
        const unsigned long long key = q.bmin[lane];
        const float c32 = __uint_as_float((uint32_t)(key >> 32));
        fin = key != ~0ull && c32 < finf;
        if (fin) {
            thr = c32 * (1.0f + kTileWindow);
        } else {
            C.best[si] = -1;
            C.best_cost[si] = __builtin_huge_val();
            C.near_tie[si] = 0;
        }
    }
    const uint64_t fmask = __ballot(fin);
    const int nf = __popcll(fmask);
    // window membership per round
    uint32_t wbits = 0;
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
        if (r < R) {
            const int32_t sl = (int32_t)((sbits >> (3 * r)) & 7u);
            const float th = __shfl(thr, sl, 64);
            // positions past the batch hold +inf, which a +inf threshold would admit
            const bool w = r * 64 + lane < T && creg[r] <= th;
            wbits |= (uint32_t)w << r;
            cnt += __popcll(__ballot(w));
        }
    }
    if (cnt > kTileQueue) {
        for (int k = 0; k < SB && s0 + k < n; ++k) shape_task(C, S, q, ns, qn, s0 + k, lane);
        return;
    }
    if (qn + cnt > kTileQueue || ns + nf > kTileSlots) {
        flush_tiles(q, ns, qn, S, lane, C.best, C.best_cost, C.near_tie);
        ns = 0;
        qn = 0;
    }
    // queue slots for the shapes with a finite minimum, in batch order
    const int32_t qs = ns + (int32_t)lanes_below(fmask);
    if (fin) {
        q.M[qs] = M;
        q.N[qs] = N;
        q.K[qs] = K;
        q.t[qs] = t;
        q.shape[qs] = si;
    }
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
        if (r < R) {
            const int32_t v = r * 64 + lane;
            const int32_t sl = (int32_t)((sbits >> (3 * r)) & 7u);
            const int32_t Ps = __shfl(P, sl, 64), qss = __shfl(qs, sl, 64);
            const int64_t as = __shfl(a, sl, 64);
            const bool w = (wbits >> r) & 1u;
            const uint64_t m = __ballot(w);
            if (w) {
                const int e = qn + (int)lanes_below(m);
                const int32_t jl = v - Ps;
                q.key[e] = ((uint32_t)qss << 24) | (uint32_t)jl;
                q.code[e] = C.code[as + jl];
            }
            qn += __popcll(m);
        }
    }
    ns += nf;
}

// Persistent waves over batches of kTileBatch consecutive shapes.  Pass 1
// takes each shape's float32 minimum with a packed (cost bits, local index)
// key.  Every candidate whose float32 cost is within kTileWindow of that
// minimum is re-evaluated in float64 through a per-wave queue, so that the
// float64 work of many shapes runs on all lanes at once; the result per
// shape is the smallest float64 cost (the lowest index winning exact ties)
// and the second-smallest, for the near-tie flag.
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
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * BLOCK + threadIdx.x) >> 6));
    const int64_t nwaves = (int64_t)((gridDim.x * BLOCK) >> 6);
    const TileCtx C{sh, off, code, n_cand, best, best_cost, near_tie};
    const int64_t nb = (n + kTileBatch - 1) / kTileBatch;
    int ns = 0, qn = 0;
    for (int64_t bt = wave; bt < nb; bt += nwaves) batch_task(C, S, q, ns, qn, bt * kTileBatch, n, lane);
    if (ns > 0) flush_tiles(q, ns, qn, S, lane, best, best_cost, near_tie);
}

template <int BLOCK>
static void select_t(const ShapePtrs& sh, const int32_t* off, const uint32_t* code, int64_t n,
                     int64_t n_cand, const Set& S, int32_t* best, double* best_cost,
                     uint8_t* near_tie, int grid_mult, hipStream_t stream)
{
    const int64_t waves_per_block = BLOCK / 64;
    const int64_t batches = (n + kTileBatch - 1) / kTileBatch;
    const int64_t want = (batches + waves_per_block - 1) / waves_per_block;
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
