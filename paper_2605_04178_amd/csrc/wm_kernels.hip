// wm_kernels.hip -- gfx950 kernels of libwavemodel: forward sweep, naive
// roofline, adjoint / loss-gradient with fixed-order FP64 reductions, device
// Adam and the multi-set calibration sweep.
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
#include <type_traits>
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

// Phase 1, float32: accumulate the descriptor's contribution into the lane's
// float32 partial sums unless it lies within 1e-5 of a max/min switch or
// (mode 1) of T = m; those return true and are left to the float64 pass.
// Mode 1's weight 1/m is a float32 reciprocal refined by one Newton step.
template <int MODE>
__device__ inline bool grad_fast(const Set& S, const Desc<float>& x, float wi, float* acc)
{
    Eval<float> E;
    evaluate<float, true>(S.st, S.cf, x, E);
    if (!(E.T < __builtin_huge_valf())) return false;  // invalid (NaN) or infeasible (+inf)
    float w = wi;
    if (MODE == 1) {
        if (!(wi > 0.0f && wi < __builtin_huge_valf())) return false;
        const float r0 = __builtin_amdgcn_rcpf(wi);
        if (E.near_kink || __builtin_fabsf(E.T * r0 - 1.0f) <= 1e-5f) return true;
        const float r = r0 * (2.0f - wi * r0);
        w = E.T > wi ? r : (E.T < wi ? -r : 0.0f);
        acc[0] += __builtin_fabsf(E.T - wi) * r;
        acc[1] += 1.0f;
    } else if (E.near_kink) {
        return true;
    }
    accumulate_partials<float>(S.st, S.cf, E, w, acc);
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
    accumulate_partials<double>(S.st, S.cd, D, w, acc);
}

// Phase 1 sweep.  The loop runs over wave-aligned groups of 64 consecutive
// descriptors so that every group's redo flags leave as one 64-bit ballot
// word, written exactly once (no clearing needed, order fixed).  X64: every
// descriptor is evaluated and differentiated in float64 (the exact variant);
// nothing is flagged, so the float64 pass only folds the partial rows.
template <int MODE, bool PTR, int BLOCK, bool X64 = false>
__global__ __launch_bounds__(BLOCK) void k_grad(DescPtrs d, int64_t n, const float* __restrict__ wv,
                                               Set sv, const Set* __restrict__ sp,
                                               double* __restrict__ partials,
                                               uint64_t* __restrict__ flags)
{
    __shared__ double red[16 * kAcc];
    const Set& S = PTR ? *sp : sv;
    struct Args { DescPtrs d; int64_t n; const float* wv; Set sv; };
    const Set* sc = PTR ? sp : WM_KERNARG_PTR(Args, sv);   // the set, read in place
    // per-lane partial sums: float32 in the bulk sweep (each lane adds the
    // ~n / (grid threads) descriptors it visits), float64 in the exact
    // variant; float64 from the wave reduction on
    typedef typename std::conditional<X64, double, float>::type A;
    A acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = (A)0;
    const uint32_t lane = threadIdx.x & 63u;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK + (threadIdx.x & ~63); base < n; base += stride) {
        const int64_t i = base + (int64_t)lane;
        bool redo = false;
        if (i < n) {
            const Desc<float> x = load_desc(d, i);
            const float w = ntload(wv + i);
            if constexpr (X64) grad_exact<MODE>(S, x, w, acc);
            else redo = grad_fast<MODE>(uniform_const(sc), x, w, acc);
        }
        const uint64_t m = __ballot(redo);
        if (lane == 0) flags[base >> 6] = m;
    }
    double a64[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) a64[j] = (double)acc[j];
    block_reduce_acc(a64, red, partials + (int64_t)blockIdx.x * kAcc);
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

// The exact variant: float64 sweep (k_grad<MODE, false, 256, true>), the
// row fold of the float64 pass (no flags are set), the fixed-order reduce.
template <int MODE>
static void launch_grad_exact_t(const DescPtrs& d, int64_t n, const float* w, const Set& S, double* partials,
                                uint64_t* flags, const GradLayout& L, int grid_mult, double* out,
                                hipStream_t stream)
{
    const int64_t want = (n + 255) / 256;
    int64_t nb = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_grad<MODE, false, 256, true>), 256) *
                 (grid_mult < 1 ? 1 : grid_mult);
    nb = nb < want ? nb : want;
    nb = nb < L.nb ? nb : L.nb;
    nb = nb < 1 ? 1 : nb;
    k_grad<MODE, false, 256, true><<<(int)nb, 256, 0, stream>>>(d, n, w, S, nullptr, partials, flags);
    k_grad_redo<MODE, false><<<L.nb2, 256, 0, stream>>>(d, n, w, S, nullptr, flags, partials, (int)nb,
                                                        partials + nb * kAcc);
    if (out) k_reduce<MODE><<<1, 256, 0, stream>>>(partials + nb * kAcc, L.nb2, out);
}

hipError_t launch_grad_exact(int mode, const DescPtrs& d, int64_t n, const float* w, const Set& S,
                             double* partials, uint64_t* flags, const GradLayout& L, int grid_mult,
                             double* out, hipStream_t stream)
{
    if (mode == 1) launch_grad_exact_t<1>(d, n, w, S, partials, flags, L, grid_mult, out, stream);
    else launch_grad_exact_t<0>(d, n, w, S, partials, flags, L, grid_mult, out, stream);
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
    __shared__ double th[kTheta];
    if (threadIdx.x >= 64) return;
    // one group of constants per lane, from the new theta in LDS
    if (adam_theta_step(st, tot, o, loss_hist, th) && threadIdx.x < kConstFields) {
        const_field<float>(th, S->st, S->cf, threadIdx.x);
        const_field<double>(th, S->st, S->cd, threadIdx.x);
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
    // one wave when it holds every row (no cross-wave steps in the reduction)
    k_adam<<<1, rows <= 64 ? 64 : 256, 0, stream>>>(partials, rows, st, o, S, loss_hist);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// multi-set calibration sweep: one persistent launch over the sets' items of
// `chunk` descriptors; block b takes the contiguous item range
// [n_items b / nb, n_items (b + 1) / nb), which covers a run of consecutive
// descriptors in each set it touches; per-block, per-set sums staged in LDS
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_grad_batched(
    const DescPtrs* __restrict__ sets, const float* const* __restrict__ meas,
    const Set* __restrict__ S_all, const int32_t* __restrict__ item_off, int n_items,
    int64_t chunk, int n_sets, const int64_t* __restrict__ set_n,
    const int64_t* __restrict__ flag_off, uint64_t* __restrict__ flags,
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
    for (int k = 0; k < n_sets; ++k) {  // uniform over the block
        const int o0 = item_off[k], o1 = item_off[k + 1];
        const int lo = it0 > o0 ? it0 : o0, hi = it1 < o1 ? it1 : o1;
        if (lo >= hi) continue;
        // items start at multiples of chunk (a multiple of 64), so each wave
        // covers whole flag words
        const int64_t nk = set_n[k];
        const int64_t begin = (int64_t)(lo - o0) * chunk;
        const int64_t end_items = (int64_t)(hi - o0) * chunk;
        const int64_t end = end_items < nk ? end_items : nk;
        const DescPtrs d = sets[k];
        const float* m = meas[k];
        uint64_t* fl = flags + flag_off[k];
        float acc[kAcc];
#pragma unroll
        for (int j = 0; j < kAcc; ++j) acc[j] = 0.0f;
        for (int64_t base = begin + (threadIdx.x & ~63); base < end; base += blockDim.x) {
            const int64_t i = base + lane;
            bool redo = false;
            if (i < end) redo = grad_fast<1>(uniform_const(S_all + k), load_desc(d, i), ntload(m + i), acc);
            const uint64_t msk = __ballot(redo);
            if (lane == 0) fl[base >> 6] = msk;
        }
        double a64[kAcc];
#pragma unroll
        for (int j = 0; j < kAcc; ++j) a64[j] = (double)acc[j];
        block_reduce_acc(a64, red, tot);
        if (threadIdx.x < kAcc) per_set[k * kAcc + threadIdx.x] = tot[threadIdx.x];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n_sets * kAcc; j += blockDim.x)
        partials[(int64_t)b * n_sets * kAcc + j] = per_set[j];
}

// Phase 2, block (b, s) for set s = blockIdx.y, so the sets' float64
// re-evaluations run side by side: fold the phase-1 rows b, b + nb2, ... of
// the set (fixed order), then re-evaluate its flagged descriptors in the
// block's share of the flag words.
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
    const int s = blockIdx.y;
    if (s >= n_sets) return;
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

int batched_redo_grid(int n_sets, int64_t max_set_words, int cap)
{
    // the pass is latency-bound (one float64 evaluation chain per flagged
    // descriptor, a few per thousand words), so a second residency round
    // would double its time
    int per = resident_blocks(reinterpret_cast<const void*>(&k_grad_redo_batched), 256) /
              (n_sets < 1 ? 1 : n_sets);
    const int64_t need = (max_set_words + 255) / 256;
    if (need < per) per = (int)need;
    if (cap < per) per = cap;
    return per < 1 ? 1 : per;
}

hipError_t launch_grad_batched(const DescPtrs* sets, const float* const* meas, const Set* S_all,
                               const int32_t* item_off, int n_items, int64_t chunk, int n_sets,
                               const int64_t* set_n, const int64_t* flag_off, uint64_t* flags,
                               double* partials, int nb, int nb2, hipStream_t stream)
{
    k_grad_batched<<<nb, 256, 0, stream>>>(sets, meas, S_all, item_off, n_items, chunk, n_sets,
                                           set_n, flag_off, flags, partials);
    k_grad_redo_batched<<<dim3(nb2, n_sets), 256, 0, stream>>>(sets, meas, S_all, set_n, flag_off, flags, n_sets,
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

}  // namespace wm
