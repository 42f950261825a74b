// wm_blackwell.hip -- the Blackwell stage-centric family (Section IV-A) on
// the same batched machinery as the CDNA model: forward sweep, adjoint /
// loss-gradient sweep with a float64 pass for descriptors near the
// compute / I-O switch or near T = m, fixed-order float64 reductions, and the
// device Adam step (calibration loops are captured as HIP graphs by the API
// layer).  Descriptors are structure-of-arrays: 5 int32 (bM, bN, bK, CTAs,
// flags) and 3 float32 (K-steps, compression ratio, output element bytes),
// 32 bytes each.
#include "bw_launch.hpp"
#include "wm_device.hpp"

namespace wm {

__device__ inline BwDesc load_bw_desc(const BwDescPtrs& d, int64_t i)
{
    BwDesc x;
    x.bM = ntload(d.bM + i);
    x.bN = ntload(d.bN + i);
    x.bK = ntload(d.bK + i);
    x.G = ntload(d.G + i);
    x.fl = ntload(d.flags + i);
    x.Kt = ntload(d.Kt + i);
    x.CR = ntload(d.CR + i);
    x.ob = ntload(d.ob + i);
    return x;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_bw_predict(BwDescPtrs d, int64_t n, BwSet S,
                                                     float* __restrict__ T, int32_t* __restrict__ cta)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    BwEval<float> E;
    evaluate_bw<float, false>(S.st, S.cf, load_bw_desc(d, i), E);
    __builtin_nontemporal_store(E.T, T + i);
    if (cta) __builtin_nontemporal_store(E.cta, cta + i);
}

// mode 0: weight dL/dT; mode 1: measured m (MRE loss).  False if the
// descriptor does not contribute.
template <int MODE, typename R>
__device__ inline bool bw_weight(R T, float wi, double& w, double& lt)
{
    if (MODE == 1) {
        if (!(wi > 0.0f && wi < __builtin_huge_valf())) return false;
        const double m = wi, im = 1.0 / m, Td = (double)T;
        lt = __builtin_fabs(Td - m) * im;
        w = Td > m ? im : (Td < m ? -im : 0.0);
    } else {
        w = wi;
        lt = 0.0;
    }
    return true;
}

// float32 pass: the descriptor's terms go into the lane's float32 partial
// sums unless it sits within 1e-5 of the compute / I-O switch or (mode 1) of
// T = m (returns true: left to the float64 pass)
template <int MODE>
__device__ inline bool bw_grad_fast(const BwSet& S, const BwDesc& x, float wi, float* acc)
{
    BwEval<float> E;
    evaluate_bw<float, true>(S.st, S.cf, x, E);
    if (!(E.T < __builtin_huge_valf())) return false;
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
    bw_accumulate<float, float>(S.cf, E, w, acc);
    return false;
}

template <int MODE>
__device__ inline void bw_grad_exact(const BwSet& S, const BwDesc& x, float wi, double* acc)
{
    BwEval<double> E;
    evaluate_bw<double, false>(S.st, S.cd, x, E);
    if (!(E.T < __builtin_huge_val())) return;
    double w, lt;
    if (!bw_weight<MODE>(E.T, wi, w, lt)) return;
    if (MODE == 1) {
        acc[0] += lt;
        acc[1] += 1.0;
    }
    bw_accumulate<double, double>(S.cd, E, w, acc);
}

// Phase 1: wave-aligned groups of 64 descriptors, one ballot word of redo
// flags per group (written exactly once).
template <int MODE, bool PTR, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_bw_grad(BwDescPtrs d, int64_t n, const float* __restrict__ wv,
                                                  BwSet sv, const BwSet* __restrict__ sp,
                                                  double* __restrict__ partials,
                                                  uint64_t* __restrict__ flags)
{
    __shared__ double red[16 * kAcc];
    const BwSet& S = PTR ? *sp : sv;
    float acc[kAcc];   // the lane's partial sums; float64 from the wave reduction on
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0f;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK + (threadIdx.x & ~63); base < n; base += stride) {
        const int64_t i = base + lane;
        bool redo = false;
        if (i < n) redo = bw_grad_fast<MODE>(S, load_bw_desc(d, i), ntload(wv + i), acc);
        const uint64_t m = __ballot(redo);
        if (lane == 0) flags[base >> 6] = m;
    }
    double a64[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) a64[j] = (double)acc[j];
    block_reduce_acc(a64, red, partials + (int64_t)blockIdx.x * kAcc);
}

// Phase 2: fold the phase-1 rows (fixed order) and redo flagged descriptors
// in float64.
template <int MODE, bool PTR>
__global__ __launch_bounds__(256) void k_bw_grad_redo(BwDescPtrs d, int64_t n,
                                                       const float* __restrict__ wv, BwSet sv,
                                                       const BwSet* __restrict__ sp,
                                                       const uint64_t* __restrict__ flags,
                                                       const double* __restrict__ rows1, int nrows1,
                                                       double* __restrict__ rows2)
{
    __shared__ double red[16 * kAcc];
    const BwSet& S = PTR ? *sp : sv;
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
            bw_grad_exact<MODE>(S, load_bw_desc(d, i), wv[i], acc);
        }
    }
    block_reduce_acc(acc, red, rows2 + (int64_t)blockIdx.x * kAcc);
}

// reduce the phase-2 rows and take one Adam step; rebuild the constants
__global__ __launch_bounds__(256) void k_bw_adam(const double* __restrict__ partials, int rows,
                                                  CalibState* st, AdamOpts o, BwSet* S,
                                                  double* loss_hist)
{
    __shared__ double red[16 * kAcc];
    __shared__ double tot[kAcc];
    reduce_partials(partials, rows, kAcc, red, tot);
    __shared__ double th[kTheta];
    if (threadIdx.x >= 64) return;
    if (adam_theta_step(st, tot, o, loss_hist, th) && threadIdx.x == 0) {
        make_bw_const<float>(th, S->st, S->cf);
        make_bw_const<double>(th, S->st, S->cd);
    }
}

template <int BLOCK>
static void bw_predict_t(const BwDescPtrs& d, int64_t n, const BwSet& S, float* T, int32_t* cta,
                         hipStream_t s)
{
    const int64_t blocks = (n + BLOCK - 1) / BLOCK;
    k_bw_predict<BLOCK><<<(unsigned)blocks, BLOCK, 0, s>>>(d, n, S, T, cta);
}

hipError_t launch_bw_predict(const BwDescPtrs& d, int64_t n, const BwSet& S, float* T, int32_t* cta,
                             const LaunchCfg& c, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    switch (c.block) {
    case 64: bw_predict_t<64>(d, n, S, T, cta, s); break;
    case 128: bw_predict_t<128>(d, n, S, T, cta, s); break;
    case 512: bw_predict_t<512>(d, n, S, T, cta, s); break;
    default: bw_predict_t<256>(d, n, S, T, cta, s); break;
    }
    return hipGetLastError();
}

template <int MODE, bool PTR>
static int bw_grid_t(int64_t n, int grid_mult)
{
    const GradLayout L = grad_layout(n);
    const int64_t want = (n + 255) / 256;
    int64_t r = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_bw_grad<MODE, PTR, 256>), 256) *
                (grid_mult < 1 ? 1 : grid_mult);
    r = r < want ? r : want;
    r = r < L.nb ? r : L.nb;
    return (int)(r < 1 ? 1 : r);
}

int bw_grad_grid(int mode, bool ptr, int64_t n, const LaunchCfg& c)
{
    if (mode == 1) return ptr ? bw_grid_t<1, true>(n, c.grid_mult) : bw_grid_t<1, false>(n, c.grid_mult);
    return ptr ? bw_grid_t<0, true>(n, c.grid_mult) : bw_grid_t<0, false>(n, c.grid_mult);
}

template <int MODE, bool PTR>
static void bw_grad_t(const BwDescPtrs& d, int64_t n, const float* w, const BwSet& S,
                      const BwSet* S_dev, double* partials, uint64_t* flags, int nb,
                      const GradLayout& L, hipStream_t s)
{
    k_bw_grad<MODE, PTR, 256><<<nb, 256, 0, s>>>(d, n, w, S, S_dev, partials, flags);
    k_bw_grad_redo<MODE, PTR><<<L.nb2, 256, 0, s>>>(d, n, w, S, S_dev, flags, partials, nb,
                                                     partials + (int64_t)nb * kAcc);
}

hipError_t launch_bw_grad(int mode, const BwDescPtrs& d, int64_t n, const float* w, const BwSet& S,
                          const BwSet* S_dev, double* partials, uint64_t* flags, const GradLayout& L,
                          const LaunchCfg& c, double* out, hipStream_t s)
{
    const int nb = bw_grad_grid(mode, S_dev != nullptr, n, c);
    if (mode == 1) {
        if (S_dev) bw_grad_t<1, true>(d, n, w, S, S_dev, partials, flags, nb, L, s);
        else bw_grad_t<1, false>(d, n, w, S, S_dev, partials, flags, nb, L, s);
    } else {
        if (S_dev) bw_grad_t<0, true>(d, n, w, S, S_dev, partials, flags, nb, L, s);
        else bw_grad_t<0, false>(d, n, w, S, S_dev, partials, flags, nb, L, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !out) return e;
    return launch_reduce(mode, partials + (int64_t)nb * kAcc, L.nb2, out, s);
}

hipError_t launch_bw_adam(const double* partials, int rows, CalibState* st, const AdamOpts& o,
                          BwSet* S, double* loss_hist, hipStream_t s)
{
    // one wave when it holds every row (no cross-wave steps in the reduction)
    k_bw_adam<<<1, rows <= 64 ? 64 : 256, 0, s>>>(partials, rows, st, o, S, loss_hist);
    return hipGetLastError();
}

}  // namespace wm
