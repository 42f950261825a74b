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
// loads in pieces staged in LDS, and each application's owner thread adds its
// rows in float64, in row order.
#include "wm_device.hpp"

namespace wm {

// the leading parameters of the application kernels, as they lie in the
// kernel-argument segment (the sets are read there in place)
struct AppsArgs {
    DescPtrs d;
    SegPtrs sg;
    int64_t n_seg, n_apps;
    Set S;
    SegSet Q;
};

struct SegRow {
    float ne, h, dd;
    int32_t nk, c;
};

__device__ inline SegRow load_seg(const SegPtrs& sg, int64_t i)
{
    SegRow r;
    r.ne = ntload(sg.n_exec + i);
    r.nk = ntload(sg.n_kern + i);
    r.c = ntload(sg.cls + i);
    r.h = ntload(sg.h2d + i);
    r.dd = ntload(sg.d2h + i);
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
    R k = vreg(q.kappa[0]);
    k = c == 1 ? vreg(q.kappa[1]) : k;
    k = c == 2 ? vreg(q.kappa[2]) : k;
    k = c == 3 ? vreg(q.kappa[3]) : k;
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

// Application totals.  A block takes BLOCK consecutive applications (one per
// thread); their rows are staged in LDS in pieces of 8 x BLOCK rows (one
// piece unless the chunk averages more than 8 rows per application); each
// thread adds its application's segment times in float64, in row order.
// T_app [n_apps] float32, and the segment times if T_seg != nullptr.
// Offsets are caller data: they are clamped into [0, n_seg], so malformed
// offsets give unspecified values but no out-of-range access.
template <int BLOCK, int MODE>
__global__ __launch_bounds__(BLOCK) void k_apps(DescPtrs d, SegPtrs sg, int64_t n_seg,
                                               int64_t n_apps, Set S, SegSet Q,
                                               float* __restrict__ T_app, float* __restrict__ T_seg)
{
    static_assert(MODE == 0, "the loss and its gradient are k_apps_grad");
    constexpr int CAP = 8 * BLOCK;
    const Set* sc = WM_KERNARG_PTR(AppsArgs, S);
    const SegSet* qc = WM_KERNARG_PTR(AppsArgs, Q);
    __shared__ float ts[CAP];
    __shared__ int32_t lo_s[BLOCK], hi_s[BLOCK];
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
        double tot = 0.0;
        // row indices stay below n_seg < 2^31: loops step by offsets within
        // a piece, so no sum can pass 2^31 - 1
        for (int32_t pb = sb; pb < se; pb = se - pb > CAP ? pb + CAP : se) {
            const int32_t pe = se - pb < CAP ? se : pb + CAP;
            // rows are visited from a 64-row boundary so that every wave's
            // loads cover whole cache lines (the rows before pb are skipped)
            for (int32_t jj = (pb & ~63) - pb + tid; jj < pe - pb; jj += BLOCK) {
                if (jj < 0) continue;
                const int32_t j = pb + jj;
                const Desc<float> x = load_desc(d, j);
                const SegRow r = load_seg(sg, j);
                const Set& Sx = uniform_const(sc);
                Eval<float> E;
                evaluate<float, false>(Sx.st, Sx.cf, x, E);
                const float t = seg_time<float>(E.T, r, uniform_const(qc).f, Sx.cf.ov[0]);
                ts[j - pb] = t;
                if (T_seg) __builtin_nontemporal_store(t, T_seg + j);
            }
            __syncthreads();
            if (tid < na) {
                const int32_t jb = lo > pb ? lo : pb, je = hi < pe ? hi : pe;
                for (int32_t j = jb; j < je; ++j) tot += (double)ts[j - pb];
            }
            __syncthreads();
        }
        if (tid < na) __builtin_nontemporal_store((float)tot, T_app + a);
        __syncthreads();  // lo_s / hi_s are rewritten by the next chunk
    }
}

// ---------------------------------------------------------------------------
// application loss (MODE 1) or vector-Jacobian product (MODE 2) in one sweep
// ---------------------------------------------------------------------------
// Per application a weight w_a: MODE 1 sign(T_a - m_a) / m_a over finite
// totals and measurements m_a > 0 (its |T_a - m_a| / m_a and a count go to
// the loss), MODE 2 the supplied dL/dT_app.  A row j of application a then
// contributes w_a n_exec_j kappa_cls(j) dT_kernel,j/dtheta to the theta
// gradient and w_a times n_exec (n_kern - 1), n_exec T_kernel (per class),
// n_exec h2d, n_exec d2h and n_exec x transfers to the segment-parameter sums
// (the derivatives of the segment time, Eq. (15)).  In MODE 1 a total within
// 1e-5 of its measurement gets weight 0 here and is flagged for the float64
// pass (returned in `near`).
template <int MODE, typename LC>
__device__ inline float app_weight(double T, float mv, LC acc, bool& near)
{
    near = false;
    if (!(T - T == 0.0)) return 0.0f;   // NaN or infinite total
    if (MODE == 2) return mv;
    if (!(mv > 0.0f && mv < __builtin_huge_valf())) return 0.0f;
    // 1/m: the float32 reciprocal refined by two float64 Newton steps (~1e-15)
    const double m = mv, r0 = (double)__builtin_amdgcn_rcpf(mv);
    const double r1 = r0 * (2.0 - m * r0);
    const double im = r1 * (2.0 - m * r1);
    if (__builtin_fabs(T * im - 1.0) <= 1e-5) {
        near = true;
        return 0.0f;
    }
    acc[0] += (float)(__builtin_fabs(T - m) * im);
    acc[1] += 1.0f;
    return (float)(T > m ? im : (T < m ? -im : 0.0));
}

// A lane's column of per-lane sums kept in LDS: sum j at p[j * STRIDE], p
// already offset by the lane (STRIDE = the block size, so the lanes of a wave
// hit consecutive words).  Only the lane itself touches its column.
template <int STRIDE>
struct LdsSums {
    float* p;
    __device__ float& operator[](int j) const { return p[j * STRIDE]; }
};

// One row's terms for an application weight wa != 0 and an evaluated
// (finite) kernel: the kernel model's Jacobian row times wa n_exec kappa into
// acc, its seven overhead slots into ovh -- or, within 1e-5 of one of its
// max/min switches, a flag for the float64 pass with that weight kept in
// wrow[j] -- and the segment-parameter sums into sacc.
template <typename OV, typename SA>
__device__ inline void app_row_terms(const Struct& st, const Const<float>& cf, const SegConst<float>& qf,
                                     const Eval<float>& E, const SegRow& r, float wa, int64_t j, float* acc,
                                     OV ovh, SA sacc, uint64_t* rflags, float* wrow)
{
    const float wr = wa * r.ne * kappa_of(qf, r.c);
    if (E.near_kink) {
        wrow[j] = wr;
        atomicOr((unsigned long long*)(rflags + (j >> 6)), 1ull << (j & 63));
    } else {
        accumulate_partials_split<float>(st, cf, E, wr, acc, ovh);
    }
    sacc[0] += wa * (r.ne * (float)(r.nk - 1));
    const float v = wa * (r.ne * E.T);
    sacc[1] += r.c == 0 ? v : 0.0f;
    sacc[2] += r.c == 1 ? v : 0.0f;
    sacc[3] += r.c == 2 ? v : 0.0f;
    sacc[4] += r.c == 3 ? v : 0.0f;
    if (r.h > 0.0f) {
        sacc[5] += wa * (r.ne * r.h);
        sacc[7] += wa * r.ne;
    }
    if (r.dd > 0.0f) {
        sacc[6] += wa * (r.ne * r.dd);
        sacc[7] += wa * r.ne;
    }
}

// float64 sum of one value over the block (fixed order); every thread gets it
template <int BLOCK>
__device__ inline double block_total(double v, double* lds /* [BLOCK / 64] */)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) s += lds[w];
    __syncthreads();
    return s;
}

// The block's kAppRow float64 sums of the lanes' float32 partial sums: the 26
// loss / count / theta columns (slots 0 and 1 from lc, 15 .. 21 from ovh, the
// rest from acc) by the recursive-halving block reduction, the eight segment
// sums by a plain one (fixed order throughout).
template <typename LC, typename OV, typename SA>
__device__ inline void store_row(const float* acc, LC lc, OV ovh, SA sacc, double* lds, double* row)
{
    double a64[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) a64[j] = (double)(j < 2 ? lc[j] : (j >= 15 && j <= 21 ? ovh[j - 15] : acc[j]));
    block_reduce_acc(a64, lds, row);
    double s64[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) s64[j] = (double)sacc[j];
    block_sum<8>(s64, lds, row + kAcc);
}

// The one-pass sweep.  A block takes BLOCK consecutive applications and walks
// them in application-aligned pieces of at most BLOCK rows, one row per
// thread: the thread evaluates its row (kernel model with its derivative
// terms) and keeps it in registers while the owner threads add their
// applications' segment times from LDS in float64 and form the weights; then
// each row thread adds its own row's weighted terms.  So every row is read
// from HBM once.  An application longer than BLOCK rows is flagged in lflags
// (one ballot word per 64 applications) for k_apps_long.  Near-switch rows are flagged in
// rflags (one bit per row; cleared before the launch) with their weight in
// wrow; near-T = m applications (MODE 1) in aflags (one ballot word per 64
// applications, written once).  Per block one row of kAppRow float64 sums:
// loss, count, theta gradient, segment-parameter sums.  Of the lane's float32
// partial sums, the loss and count, the seven overhead slots and the eight
// segment sums sit in LDS columns (they take one add per row or per
// application), the other 17 in registers: 95 VGPRs, five waves per SIMD
// (101 and four with all of them in registers).
template <int BLOCK, int MODE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(5)))
void k_apps_grad(DescPtrs d, SegPtrs sg, int64_t n_seg, int64_t n_apps, Set S, SegSet Q,
                 const float* __restrict__ meas, double* __restrict__ rows, uint64_t* __restrict__ aflags,
                 uint64_t* __restrict__ lflags, uint64_t* __restrict__ rflags, float* __restrict__ wrow)
{
    __shared__ float ts[BLOCK];
    __shared__ uint16_t own[BLOCK];
    __shared__ int32_t lo_s[BLOCK], hi_s[BLOCK];
    __shared__ float wa_s[BLOCK];
    __shared__ double red[(BLOCK / 64) * kAppRow];
    const Set* sc = WM_KERNARG_PTR(AppsArgs, S);
    const SegSet* qc = WM_KERNARG_PTR(AppsArgs, Q);
    __shared__ float sacc_s[8 * BLOCK], lc_s[2 * BLOCK], ov_s[7 * BLOCK];
    float acc[kAcc];   // the lane's partial sums; float64 from the block reduction on
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0f;
    const int tid = threadIdx.x;
    const LdsSums<BLOCK> sacc{sacc_s + tid}, lc{lc_s + tid}, ovh{ov_s + tid};
#pragma unroll
    for (int j = 0; j < 8; ++j) sacc[j] = 0.0f;
#pragma unroll
    for (int j = 0; j < 2; ++j) lc[j] = 0.0f;
#pragma unroll
    for (int j = 0; j < 7; ++j) ovh[j] = 0.0f;
    const float inf = __builtin_huge_valf();
    const int64_t nchunks = (n_apps + BLOCK - 1) / BLOCK;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t a = ch * BLOCK + tid;
        const int64_t left = n_apps - ch * BLOCK;
        const int na = left < BLOCK ? (int)left : BLOCK;
        int32_t lo = 0, hi = 0;
        float mv = 0.0f;   // the application's measurement (MODE 1) or dL/dT_app (MODE 2)
        if (tid < na) {
            int64_t x = sg.off[a], y = sg.off[a + 1];
            x = x < 0 ? 0 : (x > n_seg ? n_seg : x);
            y = y < x ? x : (y > n_seg ? n_seg : y);
            lo = (int32_t)x;
            hi = (int32_t)y;
            mv = meas[a];
        }
        lo_s[tid] = lo;
        hi_s[tid] = hi;
        __syncthreads();
        bool near_mine = false, long_mine = false;
        int t0 = 0;   // first application of the next piece (uniform over the block)
        while (t0 < na) {
            const int32_t p0 = lo_s[t0];
            // an application longer than a piece becomes an empty piece here
            // (one control path, so the loop-carried sums keep one register
            // set) and is left to k_apps_long
            const bool too_long = hi_s[t0] - p0 > BLOCK;
            if (too_long && tid == t0) long_mine = true;
            // the applications t0 .. t1 whose rows end within BLOCK rows of
            // p0: each wave tests 64 candidates per step and takes the run of
            // fits from t0 (a prefix: the ends do not decrease)
            int t1 = t0;
            if (!too_long) {
                for (int base = t0;; base += 64) {
                    const int t = base + (tid & 63);
                    const uint64_t miss = ~__ballot(t < na && hi_s[t] - p0 <= BLOCK);
                    if (miss != 0ull) {
                        t1 = base + __builtin_ctzll(miss) - 1;
                        break;
                    }
                }
            }
            int32_t pend = too_long ? p0 : hi_s[t1];
            pend = pend < p0 ? p0 : (pend - p0 > BLOCK ? p0 + BLOCK : pend);
            const bool row = tid < pend - p0;
            const int64_t j = (int64_t)p0 + tid;
            Eval<float> E;
            SegRow r;
            float tsv = 0.0f;
            if (row) {
                r = load_seg(sg, j);
                const Set& Sx = uniform_const(sc);
                evaluate<float, true>(Sx.st, Sx.cf, load_desc(d, j), E);
                tsv = seg_time<float>(E.T, r, uniform_const(qc).f, Sx.cf.ov[0]);
            }
            ts[tid] = tsv;
            own[tid] = 0xFFFFu;
            __syncthreads();
            if (!too_long && tid >= t0 && tid <= t1) {
                const int32_t jb = lo > p0 ? lo : p0, je = hi < pend ? hi : pend;
                double T = 0.0;
                int32_t k = jb;
                for (; je - k > 3; k += 4) {   // four reads in flight, added in row order
                    const float x0 = ts[k - p0], x1 = ts[k + 1 - p0], x2 = ts[k + 2 - p0], x3 = ts[k + 3 - p0];
                    T += (double)x0;
                    T += (double)x1;
                    T += (double)x2;
                    T += (double)x3;
                }
                for (; k < je; ++k) T += (double)ts[k - p0];
                for (k = jb; k < je; ++k) own[k - p0] = (uint16_t)tid;
                bool nr;
                wa_s[tid] = app_weight<MODE>(T, mv, lc, nr);
                near_mine = near_mine || nr;
            }
            __syncthreads();
            if (row && own[tid] != 0xFFFFu) {
                const float wa = wa_s[own[tid]];
                if (wa != 0.0f && E.T < inf) {
                    const Set& Sx = uniform_const(sc);
                    app_row_terms(Sx.st, Sx.cf, uniform_const(qc).f, E, r, wa, j, acc, ovh, sacc, rflags, wrow);
                }
            }
            __syncthreads();   // ts, own and wa_s are rewritten by the next piece
            t0 = t1 + 1;
        }
        const uint64_t lw = __ballot(long_mine);
        if ((tid & 63) == 0 && a < n_apps) lflags[a >> 6] = lw;
        if (MODE == 1) {
            const uint64_t fw = __ballot(near_mine);
            if ((tid & 63) == 0 && a < n_apps) aflags[a >> 6] = fw;
        }
        __syncthreads();   // lo_s / hi_s are rewritten by the next chunk
    }
    store_row(acc, lc, ovh, sacc, red, rows + (int64_t)blockIdx.x * kAppRow);
}

// Applications longer than a piece (flagged in lflags by the sweep), one at
// a time per block: the block walks the rows once for the total, forms the
// weight, and walks them again for the weighted terms.  Near-T = m
// applications set their aflags bit (after the sweep wrote the words), near-
// switch rows their rflags bit.  Per block one row of kAppRow float64 sums.
template <int MODE>
__global__ __launch_bounds__(256) void k_apps_long(DescPtrs d, SegPtrs sg, int64_t n_seg, int64_t n_apps,
                                                    Set S, SegSet Q, const float* __restrict__ meas,
                                                    const uint64_t* __restrict__ lflags,
                                                    uint64_t* __restrict__ aflags, uint64_t* __restrict__ rflags,
                                                    float* __restrict__ wrow, double* __restrict__ rows)
{
    __shared__ double red[4 * kAppRow];
    __shared__ float wa_s;
    __shared__ uint64_t words[256];
    float acc[kAcc], sacc[8];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) sacc[j] = 0.0f;
    const float inf = __builtin_huge_valf();
    const int64_t nwords = (n_apps + 63) >> 6;
    // block b takes flag words [256 b, 256 b + 256), [256 (b + grid), ...),
    // staged in LDS by one parallel load, then walked in index order
    for (int64_t w0 = (int64_t)blockIdx.x * 256; w0 < nwords; w0 += (int64_t)gridDim.x * 256) {
        const int64_t wt = w0 + threadIdx.x;
        const uint64_t mine = wt < nwords ? lflags[wt] : 0ull;
        words[threadIdx.x] = mine;
        if (!__syncthreads_or(mine != 0ull)) continue;   // no long application in this group
        for (int q = 0; q < 256; ++q) {
        uint64_t fw = words[q];
        const int64_t wi = w0 + q;
        while (fw) {
            const int bit = __builtin_ctzll(fw);
            fw &= fw - 1;
            const int64_t a = (wi << 6) + bit;
            int64_t lo = sg.off[a], hi = sg.off[a + 1];
            lo = lo < 0 ? 0 : (lo > n_seg ? n_seg : lo);
            hi = hi < lo ? lo : (hi > n_seg ? n_seg : hi);
            double part = 0.0;
            for (int64_t j = lo + threadIdx.x; j < hi; j += 256) {
                Eval<float> E;
                evaluate<float, false>(S.st, S.cf, load_desc(d, j), E);
                part += (double)seg_time<float>(E.T, load_seg(sg, j), Q.f, S.cf.ov[0]);
            }
            const double T = block_total<256>(part, red);
            if (threadIdx.x == 0) {
                bool nr;
                wa_s = app_weight<MODE>(T, meas[a], acc, nr);
                if (MODE == 1 && nr) atomicOr((unsigned long long*)(aflags + wi), 1ull << bit);
            }
            __syncthreads();
            const float wa = wa_s;
            __syncthreads();
            if (wa == 0.0f) continue;
            for (int64_t j = lo + threadIdx.x; j < hi; j += 256) {
                Eval<float> E;
                evaluate<float, true>(S.st, S.cf, load_desc(d, j), E);
                if (E.T < inf) app_row_terms(S.st, S.cf, Q.f, E, load_seg(sg, j), wa, j, acc, acc + 15, sacc, rflags, wrow);
            }
        }
        }
        __syncthreads();   // words[] is rewritten by the next group
    }
    store_row(acc, acc, acc + 15, sacc, red, rows + (int64_t)blockIdx.x * kAppRow);
}

// Block sum of kAppRow float64 accumulators (fixed order): the first 26 by
// the halving reduction, the eight segment sums by a plain one.
__device__ inline void block_row(double* acc, double* lds, double* row)
{
    block_reduce_acc(acc, lds, row);
    block_sum<8>(acc + kAcc, lds, row + kAcc);
}

// The final fixed-order reduction of the float64 pass's rows into [loss,
// count, grad theta[24], grad seg params[7]] divided by the count (vjp =
// false), or the plain sums [grad theta[24], grad seg params[7]] (vjp).
// Thread (g, c) for c < kAppRow and g < 7 adds column c of rows g, g + 7,
// ... (34 consecutive threads read one row: coalesced); column c is then the
// sum of its seven partials in g order.  nrows <= kRedoMaxBlocks; called by
// a whole block of 256.
__device__ inline void apps_final(const double* rows, int nrows, const SegSet& Q, bool vjp,
                                  double* part /* [7 * kAppRow] */, double* tot /* [kAppRow] */, double* out)
{
    constexpr int G = 256 / kAppRow;
    constexpr int K = (kRedoMaxBlocks + G - 1) / G;   // rows per thread at most
    const int t = threadIdx.x;
    if (t < G * kAppRow) {
        const int g = t / kAppRow, c = t - g * kAppRow;
        double x[K];   // every load in flight before the in-order additions
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int r = g + k * G;
            x[k] = r < nrows ? rows[(int64_t)r * kAppRow + c] : 0.0;
        }
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) v += x[k];
        part[g * kAppRow + c] = v;
    }
    __syncthreads();
    if (t < kAppRow) {
        double v = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) v += part[g * kAppRow + t];
        tot[t] = v;
    }
    __syncthreads();
    const double* sa = tot + kAcc;   // extra launches, kappa[4], h2d, d2h, transfers
    if (vjp) {
        if (t >= kTheta + kSegParams) return;
        double v;
        if (t < kTheta) v = tot[2 + t] + (t == 13 ? sa[0] : 0.0);
        else if (t < kTheta + 4) v = sa[1 + (t - kTheta)];
        else if (t == kTheta + 4) v = -sa[5] * Q.inv_bw2_h2d;
        else if (t == kTheta + 5) v = -sa[6] * Q.inv_bw2_d2h;
        else v = sa[7];
        out[t] = v;
        return;
    }
    if (t >= kAppsOut) return;
    const double c = tot[1];
    const double ic = c > 0.0 ? 1.0 / c : 0.0;
    double v;
    if (t == 0) v = tot[0] * ic;
    else if (t == 1) v = c;
    else if (t < kAcc) v = (tot[t] + (t == 2 + 13 ? sa[0] : 0.0)) * ic;
    else if (t < kAcc + 4) v = sa[1 + (t - kAcc)] * ic;
    else if (t == kAcc + 4) v = -sa[5] * Q.inv_bw2_h2d * ic;
    else if (t == kAcc + 5) v = -sa[6] * Q.inv_bw2_d2h * ic;
    else v = sa[7] * ic;
    out[t] = v;
}

// The float64 pass: block b folds the sweep's rows b, b + gridDim.x, ...
// (fixed order); then (MODE 1) every application flagged near T = m is done
// in full in float64 by one wave, its lanes over the rows -- total, weight,
// loss, the rows' Jacobian terms and segment sums -- and every row flagged
// near a max/min switch (in an application decided in float32) adds its
// float64 Jacobian row times the weight kept in wrow.  Each block writes one
// row to rows2.
template <int MODE>
__global__ __launch_bounds__(256) void k_apps_grad_redo(DescPtrs d, SegPtrs sg, int64_t n_seg,
                                                         int64_t n_apps, Set S, SegSet Q,
                                                         const float* __restrict__ meas,
                                                         const uint64_t* __restrict__ aflags,
                                                         const uint64_t* __restrict__ rflags,
                                                         const float* __restrict__ wrow,
                                                         const double* __restrict__ rows1, int nrows1,
                                                         double* __restrict__ rows2)
{
    __shared__ double red[4 * kAppRow];
    double acc[kAppRow];
#pragma unroll
    for (int j = 0; j < kAppRow; ++j) acc[j] = 0.0;
    for (int r = blockIdx.x + gridDim.x * threadIdx.x; r < nrows1; r += gridDim.x * blockDim.x) {
#pragma unroll
        for (int j = 0; j < kAppRow; ++j) acc[j] += rows1[(int64_t)r * kAppRow + j];
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    if (MODE == 1) {
        // Each wave loads 64 flag words at once and takes their flagged
        // applications in batches of up to eight, in flag order: lane group
        // grp = lane / 8 does application grp of the batch -- total, weight,
        // loss, the rows' Jacobian terms and segment sums -- its eight lanes
        // over the rows.
        const int64_t nwords = (n_apps + 63) >> 6;
        const int grp = lane >> 3, sub = lane & 7;
        for (int64_t w0 = (t0 >> 6) << 6; w0 < nwords; w0 += stride) {
            const int64_t wl = w0 + lane;
            uint64_t rem = wl < nwords ? aflags[wl] : 0ull;   // this lane's flags not yet taken
            for (uint64_t todo = __ballot(rem != 0ull); todo; todo = __ballot(rem != 0ull)) {
                int64_t my_app = -1;
                for (int nb = 0; nb < 8 && todo; ++nb) {
                    const int q = __builtin_ctzll(todo);
                    const uint64_t fw = __shfl(rem, q, 64);
                    if (grp == nb) my_app = ((w0 + q) << 6) + __builtin_ctzll(fw);
                    if (lane == q) rem &= rem - 1;
                    if ((fw & (fw - 1)) == 0ull) todo &= todo - 1;   // lane q has no more
                }
                int64_t lo = 0, hi = 0;
                if (my_app >= 0) {
                    lo = sg.off[my_app];
                    hi = sg.off[my_app + 1];
                    lo = lo < 0 ? 0 : (lo > n_seg ? n_seg : lo);
                    hi = hi < lo ? lo : (hi > n_seg ? n_seg : hi);
                }
                double part = 0.0;
                for (int64_t j = lo + sub; j < hi; j += 8) {
                    Eval<double> E;
                    evaluate<double, false>(S.st, S.cd, widen(load_desc(d, j)), E);
                    part += seg_time<double>(E.T, load_seg(sg, j), Q.d, S.cd.ov[0]);
                }
                // the group's lanes end with the same (fixed-order) total
                part += __shfl_xor(part, 4, 64);
                part += __shfl_xor(part, 2, 64);
                part += __shfl_xor(part, 1, 64);
                const double T = part;
                if (my_app < 0 || !(T - T == 0.0)) continue;
                const double m = meas[my_app];
                const double im = 1.0 / m;
                const double w = T > m ? im : (T < m ? -im : 0.0);
                if (sub == 0) {
                    acc[0] += __builtin_fabs(T - m) * im;
                    acc[1] += 1.0;
                }
                if (w == 0.0) continue;
                for (int64_t j = lo + sub; j < hi; j += 8) {
                    Eval<double> E;
                    evaluate<double, true>(S.st, S.cd, widen(load_desc(d, j)), E);
                    if (!(E.T < __builtin_huge_val())) continue;
                    const SegRow r = load_seg(sg, j);
                    const double ne = r.ne;
                    accumulate_partials<double>(S.st, S.cd, E, w * ne * kappa_of(Q.d, r.c), acc);
                    double* sa = acc + kAcc;
                    sa[0] += w * (ne * (double)(r.nk - 1));
                    const double v = w * (ne * E.T);
                    sa[1] += r.c == 0 ? v : 0.0;
                    sa[2] += r.c == 1 ? v : 0.0;
                    sa[3] += r.c == 2 ? v : 0.0;
                    sa[4] += r.c == 3 ? v : 0.0;
                    if (r.h > 0.0f) {
                        sa[5] += w * (ne * (double)r.h);
                        sa[7] += w * ne;
                    }
                    if (r.dd > 0.0f) {
                        sa[6] += w * (ne * (double)r.dd);
                        sa[7] += w * ne;
                    }
                }
            }
        }
    }
    const int64_t rwords = (n_seg + 63) >> 6;
    for (int64_t wi = t0; wi < rwords; wi += stride) {
        uint64_t fw = rflags[wi];
        while (fw) {
            const int bit = __builtin_ctzll(fw);
            fw &= fw - 1;
            const int64_t j = (wi << 6) + bit;
            Eval<double> E;
            evaluate<double, true>(S.st, S.cd, widen(load_desc(d, j)), E);
            if (E.T < __builtin_huge_val()) accumulate_partials<double>(S.st, S.cd, E, (double)wrow[j], acc);
        }
    }
    block_row(acc, red, rows2 + (int64_t)blockIdx.x * kAppRow);
}

__global__ __launch_bounds__(256) void k_apps_final(const double* __restrict__ rows, int nrows, SegSet Q,
                                                    int vjp, double* __restrict__ out)
{
    __shared__ double part[(256 / kAppRow) * kAppRow];
    __shared__ double tot[kAppRow];
    apps_final(rows, nrows, Q, vjp != 0, part, tot, out);
}

__global__ __launch_bounds__(256) void k_zero_words(uint64_t* __restrict__ w, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        w[i] = 0;
}

template <int BLOCK, int MODE>
static int apps_grid(int64_t n_apps, int grid_mult)
{
    const int64_t chunks = (n_apps + BLOCK - 1) / BLOCK;
    const void* k = MODE == 0 ? reinterpret_cast<const void*>(&k_apps<BLOCK, 0>)
                              : (MODE == 1 ? reinterpret_cast<const void*>(&k_apps_grad<BLOCK, 1>)
                                           : reinterpret_cast<const void*>(&k_apps_grad<BLOCK, 2>));
    int64_t b = (int64_t)resident_blocks(k, BLOCK) * (grid_mult < 1 ? 1 : grid_mult);
    b = b < chunks ? b : chunks;
    b = b < kAppsMaxBlocks ? b : kAppsMaxBlocks;
    return (int)(b < 1 ? 1 : b);
}

hipError_t launch_predict_apps(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg, int64_t n_apps,
                               const Set& S, const SegSet& Q, float* T_app, float* T_seg,
                               const LaunchCfg& c, hipStream_t s)
{
    if (n_apps <= 0) return hipSuccess;
#define WM_APPS_CASE(B)                                                                               \
    case B:                                                                                           \
        k_apps<B, 0><<<apps_grid<B, 0>(n_apps, c.grid_mult), B, 0, s>>>(d, sg, n_seg, n_apps, S, Q,  \
                                                                       T_app, T_seg);                \
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

int apps_redo_blocks(int64_t n_apps, int64_t n_seg)
{
    const int64_t words = ((n_apps > n_seg ? n_apps : n_seg) + 63) / 64;
    const int64_t b = (words + 255) / 256;
    return (int)(b < 1 ? 1 : (b > kRedoMaxBlocks ? kRedoMaxBlocks : b));
}

template <int MODE>
static hipError_t apps_grad_t(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg, int64_t n_apps,
                              const float* meas, const Set& S, const SegSet& Q, double* rows,
                              uint64_t* aflags, uint64_t* lflags, uint64_t* rflags, float* wrow,
                              const LaunchCfg& c, double* out, hipStream_t s)
{
    const int64_t rwords = (n_seg + 63) / 64;
    if (rwords > 0) {
        const int64_t zb = (rwords + 255) / 256;
        k_zero_words<<<(int)(zb < 1024 ? zb : 1024), 256, 0, s>>>(rflags, rwords);
    }
    int nb1 = 1;
#define WM_APPS_CASE(B)                                                                               \
    case B:                                                                                           \
        nb1 = apps_grid<B, MODE>(n_apps, c.grid_mult);                                               \
        k_apps_grad<B, MODE><<<nb1, B, 0, s>>>(d, sg, n_seg, n_apps, S, Q, meas, rows, aflags, lflags, \
                                               rflags, wrow);                                        \
        break;
    switch (c.block) {
        WM_APPS_CASE(64)
        WM_APPS_CASE(128)
        WM_APPS_CASE(256)
        WM_APPS_CASE(512)
    default: return hipErrorInvalidValue;
    }
#undef WM_APPS_CASE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_apps_long<MODE><<<kAppsLongBlocks, 256, 0, s>>>(d, sg, n_seg, n_apps, S, Q, meas, lflags, aflags, rflags,
                                                      wrow, rows + (int64_t)nb1 * kAppRow);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nb2 = apps_redo_blocks(n_apps, n_seg);
    const int nrows1 = nb1 + kAppsLongBlocks;
    double* rows2 = rows + (int64_t)nrows1 * kAppRow;
    k_apps_grad_redo<MODE><<<nb2, 256, 0, s>>>(d, sg, n_seg, n_apps, S, Q, meas, aflags, rflags, wrow, rows,
                                               nrows1, rows2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_apps_final<<<1, 256, 0, s>>>(rows2, nb2, Q, MODE == 2 ? 1 : 0, out);
    return hipGetLastError();
}

hipError_t launch_apps_loss_grad(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg, int64_t n_apps,
                                 const float* measured, const Set& S, const SegSet& Q, double* rows,
                                 uint64_t* aflags, uint64_t* lflags, uint64_t* rflags, float* wrow,
                                 const LaunchCfg& cfg, double* out, hipStream_t stream)
{
    return apps_grad_t<1>(d, sg, n_seg, n_apps, measured, S, Q, rows, aflags, lflags, rflags, wrow, cfg, out,
                          stream);
}

hipError_t launch_apps_vjp(const DescPtrs& d, const SegPtrs& sg, int64_t n_seg, int64_t n_apps,
                           const float* w_app, const Set& S, const SegSet& Q, double* rows, uint64_t* lflags,
                           uint64_t* rflags, float* wrow, const LaunchCfg& cfg, double* out, hipStream_t stream)
{
    return apps_grad_t<2>(d, sg, n_seg, n_apps, w_app, S, Q, rows, nullptr, lflags, rflags, wrow, cfg, out,
                          stream);
}

}  // namespace wm
