// wm_planning.hip -- per-group calibration multipliers and kernel-fusion
// planning on top of the model.
//
// Multipliers (Section IV-D: optional per-case multipliers with train /
// holdout separation): for each group of rows, the multiplier that minimises
// the training mean relative error of mult * T is a weighted median of the
// ratios m/T (weights T/m).  One wave per group evaluates every candidate's
// cumulative weight against all the group's rows, so no sort is needed.
//
// Fusion (Section IV-B: a fused kernel is modelled with the combined flops
// and bytes plus tau_fusion): a chain of kernels is cut into runs of at most
// R consecutive kernels.  One thread per row extends the fusion sums of the
// runs starting there one row at a time (float64 sums) and evaluates each
// run's combined descriptor in float32; one thread per chain runs the prefix
// dynamic programme over those costs in float64.  Chains where float32 could
// decide differently from float64 (a decision within a small relative
// margin, or a run float32 cannot represent) are redone in float64, one wave
// per chain, so plans match a float64 evaluation except at its own ties.
#include "wm_device.hpp"

namespace wm {

// ---------------------------------------------------------------------------
// multipliers
// ---------------------------------------------------------------------------
__device__ inline bool mult_ok(double T, double m)
{
    const double inf = __builtin_huge_val();
    return T > 0.0 && T < inf && m > 0.0 && m < inf;
}

template <int NA>
__device__ inline void wave_sum(double* acc)
{
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        double v = acc[j];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
        acc[j] = v;
    }
}

// The wave's index in the grid, in a form the compiler sees as the same on
// every lane (so that what depends on it stays in scalar registers and
// loops over it are scalar-controlled).
__device__ inline int64_t wave_id()
{
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    return (int64_t)blockIdx.x * (int64_t)(blockDim.x >> 6) + w;
}

// Lane k's value of x (k wave-uniform); every lane active.
__device__ inline int64_t read_lane64(int64_t x, int k)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, k);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)x >> 32), k);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ inline double read_lane_f64(double x, int k)
{
    return __builtin_bit_cast(double, read_lane64(__builtin_bit_cast(int64_t, x), k));
}

__device__ inline float read_lane_f32(float x, int k)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, x), k));
}

// Rows i in [a, b) of one group: the training loss and count, the held-out
// loss and count (float64, per lane), and T_scaled = mu T_i.
__device__ inline void mult_apply(double mu, float t, float m, bool tr, int64_t i,
                                  float* __restrict__ T_scaled, double* st)
{
    T_scaled[i] = (float)(mu * (double)t);
    if (!mult_ok(t, m)) return;
    const double e = __builtin_fabs(mu * (double)t - (double)m) / (double)m;
    if (tr) {
        st[0] += e;
        st[1] += 1.0;
    } else {
        st[2] += e;
        st[3] += 1.0;
    }
}

// A group of any size on the whole wave.  Candidate k (a valid training row)
// is the multiplier when its cumulative weight C_k = sum of w_i over valid
// training rows with (x_i, i) <= (x_k, k) reaches half the total and no
// smaller candidate does; the smallest such (x_k, k) wins.  Lanes take 64
// candidates at a time and the group's rows 64 at a time: a lane prepares
// its row once (x_i = m/T in float32 and float64, w_i = T/m in float64, 0
// for rows that do not count), then every row is broadcast to the lanes by
// lane reads.  The order (x_i, i) <= (x_k, k) is decided on the float32
// ratios, which round monotonically, and on the float64 ratios where the
// float32 ones tie; C_k and the total are float64 sums in row order.
__device__ inline void fit_group_scan(int64_t g, int64_t a, int64_t b, const float* __restrict__ T,
                                      const float* __restrict__ meas, const uint8_t* __restrict__ train,
                                      double* __restrict__ mult, float* __restrict__ T_scaled, double* st)
{
    const int lane = threadIdx.x & 63;
    const double dinf = __builtin_huge_val();
    const float finf = __builtin_huge_valf();
    double Wt = 0.0;   // total training weight, row order
    double bx = dinf;
    int64_t bk = INT64_MAX;
    for (int64_t k0 = a; k0 < b; k0 += 64) {
        // this lane's candidate
        const int64_t k = k0 + lane;
        float xfk = finf;
        double xdk = dinf, wk = 0.0;
        if (k < b) {
            const float tk = T[k], mk = meas[k];
            if (train[k] && mult_ok(tk, mk)) {
                xfk = mk / tk;
                xdk = (double)mk / (double)tk;
                wk = (double)tk / (double)mk;
            }
        }
        double C = 0.0;
        for (int64_t i0 = a; i0 < b; i0 += 64) {
            // this lane's row (the candidate's own when the chunks coincide)
            const int64_t i = i0 + lane;
            float xfi = xfk;
            double xdi = xdk, wi = wk;
            if (i0 != k0) {
                xfi = finf;
                xdi = dinf;
                wi = 0.0;
                if (i < b) {
                    const float ti = T[i], mi = meas[i];
                    if (train[i] && mult_ok(ti, mi)) {
                        xfi = mi / ti;
                        xdi = (double)mi / (double)ti;
                        wi = (double)ti / (double)mi;
                    }
                }
            }
            const int cnt = b - i0 < 64 ? (int)(b - i0) : 64;
            for (int r = 0; r < cnt; ++r) {
                const float xf = read_lane_f32(xfi, r);
                const double w = read_lane_f64(wi, r);
                if (k0 == a) Wt += w;
                bool before = xf < xfk;
                const bool tie = xf == xfk;
                if (__ballot(tie) != 0ull) {
                    const double xd = read_lane_f64(xdi, r);
                    if (tie) before = xd < xdk || (xd == xdk && i0 + r <= k);
                }
                C += before ? w : 0.0;
            }
        }
        if (xdk < dinf && C >= 0.5 * Wt && (xdk < bx || (xdk == bx && k < bk))) {
            bx = xdk;
            bk = k;
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const double ox = __shfl_xor(bx, m, 64);
        const int64_t ok = __shfl_xor(bk, m, 64);
        if (ox < bx || (ox == bx && ok < bk)) {
            bx = ox;
            bk = ok;
        }
    }
    const double mu = bk == INT64_MAX ? 1.0 : bx;
    if (lane == 0) mult[g] = mu;
    for (int64_t i = a + lane; i < b; i += 64) mult_apply(mu, T[i], meas[i], train[i] != 0, i, T_scaled, st);
}

// Groups of at most W rows (W = 32: two groups side by side in the wave
// halves; W = 64: one group), row a_s + l on lane l of segment s.  The
// segment sorts its keys (x_i, i) ascending by a bitonic network across its
// lanes (rows that do not count carry x = +inf and w = 0, so they sort
// last), takes each sorted key's weight from its row's lane, and forms the
// inclusive cumulative weights by a float64 prefix sum; the multiplier is the
// first sorted x whose cumulative weight reaches half the segment's total.
// The prefix sum adds in tree order, so C can differ from the row-order sum
// in the last bits; where that moves the choice, the two ratios' objectives
// are equal to rounding (the objective is flat between them when C equals
// half the total).  g1 < 0: the upper half has no group.
template <int W>
__device__ inline void fit_groups_sorted(int64_t g0, int64_t a0, int64_t b0, int64_t g1, int64_t a1,
                                         int64_t b1, const float* __restrict__ T,
                                         const float* __restrict__ meas, const uint8_t* __restrict__ train,
                                         double* __restrict__ mult, float* __restrict__ T_scaled, double* st)
{
    const int lane = threadIdx.x & 63;
    const int seg = W == 64 ? 0 : lane >> 5;
    const int l = lane & (W - 1);
    const int64_t g = seg ? g1 : g0, a = seg ? a1 : a0, b = seg ? b1 : b0;
    const int64_t i = a + l;
    const bool in = g >= 0 && i < b;
    const double dinf = __builtin_huge_val();
    float t = 0.0f, m = 0.0f;
    bool tr = false;
    double x = dinf, w = 0.0;
    if (in) {
        t = T[i];
        m = meas[i];
        tr = train[i] != 0;
        if (tr && mult_ok(t, m)) {
            x = (double)m / (double)t;
            w = (double)t / (double)m;
        }
    }
    // bitonic sort of the unique keys (x, l) within each segment
    double sx = x;
    int si = l;
#pragma unroll
    for (int k = 2; k <= W; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const double px = __shfl_xor(sx, j, 64);
            const int pi = __shfl_xor(si, j, 64);
            const bool p_less = px < sx || (px == sx && pi < si);
            // the lower lane of a pair keeps the smaller key in an ascending
            // block, the larger one in a descending block
            const bool keep_min = ((l & j) == 0) == ((l & k) == 0);
            if (keep_min == p_less) {
                sx = px;
                si = pi;
            }
        }
    }
    const int base = seg * W;
    double c = __shfl(w, base + si, 64);
#pragma unroll
    for (int d = 1; d < W; d <<= 1) {
        const double u = __shfl_up(c, d, W);
        if (l >= d) c += u;
    }
    const double tot = __shfl(c, base + W - 1, 64);
    uint64_t hit = __ballot(sx < dinf && c >= 0.5 * tot);
    if (W == 32) hit = (hit >> base) & 0xFFFFFFFFull;
    const int jl = hit != 0ull ? __builtin_ctzll(hit) : 0;
    const double xj = __shfl(sx, base + jl, 64);
    const double mu = hit != 0ull ? xj : 1.0;
    if (g >= 0 && l == 0) mult[g] = mu;
    if (in) mult_apply(mu, t, m, tr, i, T_scaled, st);
}

// One wave per pair of consecutive groups (persistent): two groups of at
// most 32 rows share the wave by halves; otherwise each group in turn, up to
// 64 rows by the sorted form, beyond by the candidate scan.  Group bounds are
// clamped into [0, n].  Per wave the stats (training loss, count, held-out
// loss, count) accumulate in float64 and each block writes their sums to
// its row.
__device__ inline void group_bounds(const int32_t* __restrict__ off, int64_t g, int64_t n, int64_t& a, int64_t& b)
{
    a = off[g];
    b = off[g + 1];
    a = a < 0 ? 0 : (a > n ? n : a);
    b = b < a ? a : (b > n ? n : b);
}

__global__ __launch_bounds__(256) void k_fit_mult(const float* __restrict__ T,
                                                   const float* __restrict__ meas,
                                                   const int32_t* __restrict__ off,
                                                   int64_t n_groups, int64_t n,
                                                   const uint8_t* __restrict__ train,
                                                   double* __restrict__ mult,
                                                   float* __restrict__ T_scaled,
                                                   double* __restrict__ rows)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = wave_id();
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t npairs = (n_groups + 1) >> 1;
    double st[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t q = wave; q < npairs; q += nwaves) {
        const int64_t g0 = 2 * q, g1 = 2 * q + 1 < n_groups ? 2 * q + 1 : -1;
        int64_t a0, b0, a1 = 0, b1 = 0;
        group_bounds(off, g0, n, a0, b0);
        if (g1 >= 0) group_bounds(off, g1, n, a1, b1);
        if (b0 - a0 <= 32 && b1 - a1 <= 32) {
            fit_groups_sorted<32>(g0, a0, b0, g1, a1, b1, T, meas, train, mult, T_scaled, st);
            continue;
        }
        for (int h = 0; h < 2; ++h) {
            const int64_t g = h ? g1 : g0, a = h ? a1 : a0, b = h ? b1 : b0;
            if (g < 0) continue;
            if (b - a <= 64)
                fit_groups_sorted<64>(g, a, b, -1, 0, 0, T, meas, train, mult, T_scaled, st);
            else
                fit_group_scan(g, a, b, T, meas, train, mult, T_scaled, st);
        }
    }
    // the block's four waves, then one row per block (fixed order)
    __shared__ double red[4][4];
    wave_sum<4>(st);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) red[threadIdx.x >> 6][j] = st[j];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w][threadIdx.x];
        rows[(int64_t)blockIdx.x * 4 + threadIdx.x] = v;
    }
}

__global__ __launch_bounds__(256) void k_fit_mult_reduce(const double* __restrict__ rows, int64_t nrows,
                                                          double* __restrict__ out)
{
    __shared__ double red[4][4];
    double st[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t r = threadIdx.x; r < nrows; r += blockDim.x)
#pragma unroll
        for (int j = 0; j < 4; ++j) st[j] += rows[r * 4 + j];
    wave_sum<4>(st);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[threadIdx.x >> 6][j] = st[j];
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

int fit_mult_grid(int64_t n_groups)
{
    const int64_t want = ((n_groups + 1) / 2 + 3) / 4;  // a pair of groups per wave, 4 waves per block
    int64_t b = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_fit_mult), 256) * 2;
    b = b < want ? b : want;
    b = b < kFitMultMaxBlocks ? b : kFitMultMaxBlocks;
    return (int)(b < 1 ? 1 : b);
}

hipError_t launch_fit_multipliers(const float* T, const float* meas, const int32_t* off,
                                  int64_t n_groups, int64_t n, const uint8_t* train, double* mult,
                                  float* T_scaled, double* rows, double* stats, hipStream_t s)
{
    const int nb = fit_mult_grid(n_groups);
    k_fit_mult<<<nb, 256, 0, s>>>(T, meas, off, n_groups, n, train, mult, T_scaled, rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_fit_mult_reduce<<<1, 256, 0, s>>>(rows, (int64_t)nb, stats);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fusion planning
// ---------------------------------------------------------------------------
// One descriptor row through the caches: the fusion kernels read each row
// once per run that holds it, so these loads are not marked streaming.
__device__ inline Desc<float> load_row(const DescPtrs& d, int64_t i)
{
    Desc<float> x;
    x.F = d.F[i];
    x.B = d.B[i];
    x.r1 = d.r1[i];
    x.r2 = d.r2[i];
    x.r3 = d.r3[i];
    x.K = d.K[i];
    x.u = d.u[i];
    x.W = d.W[i];
    x.v = d.vgpr[i];
    x.s = d.lds[i];
    x.gp = d.gpack[i];
    x.G = d.grid[i];
    return x;
}

// The combined descriptor of rows a .. a+len-1 (len >= 2), float64:
//   F = sum F;  B = max(sum B - 2 sum edges, 0);  r_l byte-weighted;
//   K = sum K;  W = max(sum W - sum edges, 0);  dtype of the first row with
//   the largest F;  u keeps the summed compute time F_k / (u_k P_k) (capped
//   at 1, 1 when F = 0);  VGPRs, LDS, workgroup size, grid, concurrent
//   kernels and devices the largest;  host syncs summed (<= 15);  fused.
// Returns false if a row or an edge is invalid.
__device__ inline bool fuse_rows(const DescPtrs& d, const float* __restrict__ edge,
                                 const double* peak, int64_t a, int32_t len, Desc<double>& o)
{
#pragma clang fp contract(off)
    double F = 0.0, Bs = 0.0, E = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0, K = 0.0, Ws = 0.0, tc = 0.0,
           Fmax = -1.0;
    int32_t v = 0, s = 0, g = 0, G = 0, nc = 0, nd = 0, ns = 0, dt = 0;
    for (int32_t q = 0; q < len; ++q) {
        const int64_t k = a + q;
        const Desc<float> x = load_row(d, k);
        if (!desc_valid(x)) return false;
        if (q < len - 1) {
            const float ek = edge[k];
            if (!(ek >= 0.0f && ek < __builtin_huge_valf())) return false;
            E += (double)ek;
        }
        const double Fk = x.F, Bk = x.B;
        const int32_t dtk = (x.gp >> 11) & 7;
        F += Fk;
        Bs += Bk;
        r1 += (double)x.r1 * Bk;
        r2 += (double)x.r2 * Bk;
        r3 += (double)x.r3 * Bk;
        K += (double)x.K;
        Ws += (double)x.W;
        if (Fk > 0.0) tc += Fk / ((double)x.u * peak[dtk]);
        if (Fk > Fmax) {
            Fmax = Fk;
            dt = dtk;
        }
        v = x.v > v ? x.v : v;
        s = x.s > s ? x.s : s;
        g = (x.gp & 2047) > g ? (x.gp & 2047) : g;
        G = x.G > G ? x.G : G;
        nc = ((x.gp >> 14) & 7) > nc ? ((x.gp >> 14) & 7) : nc;
        nd = ((x.gp >> 17) & 7) > nd ? ((x.gp >> 17) & 7) : nd;
        ns += (x.gp >> 21) & 15;
    }
    o.F = F;
    o.B = Bs - 2.0 * E > 0.0 ? Bs - 2.0 * E : 0.0;
    o.r1 = Bs > 0.0 ? r1 / Bs : 0.0;
    o.r2 = Bs > 0.0 ? r2 / Bs : 0.0;
    o.r3 = Bs > 0.0 ? r3 / Bs : 0.0;
    o.K = K;
    o.W = Ws - E > 0.0 ? Ws - E : 0.0;
    if (F > 0.0) {
        const double u = F / (peak[dt] * tc);
        o.u = u < 1.0 ? u : 1.0;
    } else {
        o.u = 1.0;
    }
    o.v = v;
    o.s = s;
    o.G = G;
    ns = ns < 15 ? ns : 15;
    o.gp = g | (dt << 11) | (nc << 14) | (nd << 17) | (1 << 20) | (ns << 21);
    return true;
}

struct Peaks {
    double p[5];
};

// Running float64 sums of a run of rows, extended one row at a time in row
// order (the order fuse_rows adds them in, so a run's sums are the same).
struct FuseSum {
    double F, Bs, E, r1, r2, r3, K, Ws, tc;
    float Fmax;
    int32_t v, s, g, G, nc, nd, ns, dt;
};

__device__ inline void fuse_begin(FuseSum& a)
{
    a.F = a.Bs = a.E = a.r1 = a.r2 = a.r3 = a.K = a.Ws = a.tc = 0.0;
    a.Fmax = -1.0f;
    a.v = a.s = a.g = a.G = a.nc = a.nd = a.ns = a.dt = 0;
}

// Adds row x; tk = its compute time F / (u P_dtype) (float32, only summed).
__device__ inline void fuse_add(FuseSum& a, const Desc<float>& x, float tk)
{
#pragma clang fp contract(off)
    const double Bk = x.B;
    const int32_t gp = x.gp;
    const int32_t dtk = (gp >> 11) & 7;
    a.F += (double)x.F;
    a.Bs += Bk;
    a.r1 += (double)x.r1 * Bk;
    a.r2 += (double)x.r2 * Bk;
    a.r3 += (double)x.r3 * Bk;
    a.K += (double)x.K;
    a.Ws += (double)x.W;
    if (x.F > 0.0f) a.tc += (double)tk;
    if (x.F > a.Fmax) {
        a.Fmax = x.F;
        a.dt = dtk;
    }
    a.v = x.v > a.v ? x.v : a.v;
    a.s = x.s > a.s ? x.s : a.s;
    a.g = (gp & 2047) > a.g ? (gp & 2047) : a.g;
    a.G = x.G > a.G ? x.G : a.G;
    a.nc = ((gp >> 14) & 7) > a.nc ? ((gp >> 14) & 7) : a.nc;
    a.nd = ((gp >> 17) & 7) > a.nd ? ((gp >> 17) & 7) : a.nd;
    a.ns += (gp >> 21) & 15;
}

// The fused descriptor of the run so far (two or more rows), formed in
// float64 as fuse_rows does and rounded to float32; Wd gets the float64
// working set.
__device__ inline Desc<float> fuse_narrow(const FuseSum& a, double peak_dt, double& Wd)
{
#pragma clang fp contract(off)
    Desc<float> o;
    o.F = (float)a.F;
    o.B = (float)(a.Bs - 2.0 * a.E > 0.0 ? a.Bs - 2.0 * a.E : 0.0);
    const double iB = a.Bs > 0.0 ? 1.0 / a.Bs : 0.0;
    o.r1 = (float)(a.r1 * iB);
    o.r2 = (float)(a.r2 * iB);
    o.r3 = (float)(a.r3 * iB);
    o.K = (float)a.K;
    Wd = a.Ws - a.E > 0.0 ? a.Ws - a.E : 0.0;
    o.W = (float)Wd;
    if (a.F > 0.0) {
        const double u = a.F / (peak_dt * a.tc);
        o.u = (float)(u < 1.0 ? u : 1.0);
    } else {
        o.u = 1.0f;
    }
    o.v = a.v;
    o.s = a.s;
    o.G = a.G;
    const int32_t ns = a.ns < 15 ? a.ns : 15;
    o.gp = a.g | (a.dt << 11) | (a.nc << 14) | (a.nd << 17) | (1 << 20) | (ns << 21);
    return o;
}

// Coverage byte per row: bits 0-5 the number of runs costed from the row
// (at most 32), bit 7 set when one of them is uncertain in float32.
constexpr uint8_t kPlanCount = 0x3f;
constexpr uint8_t kPlanUncertain = 0x80;

// One thread per row s: the runs of 1 .. m rows starting at s, m = min(R,
// rows left in s's chain), their fusion sums extended one row per step in
// float64 and each fused descriptor evaluated in float32 (the row itself for
// the run of one); cost[(s + len - 1) * R + len - 1] gets the time (+inf for
// runs holding an invalid row or edge and for NaN).  A run is uncertain when
// float32 cannot stand for float64: its float32 time is not finite while its
// rows are valid (and the kernel is not simply infeasible), the time is
// negative, or its working set lies within 1e-6 of the LLC capacity, where
// the hit rate of Table "hlcc-piecewise" jumps.
struct FuseArgs {   // k_fuse_costs's parameters, in order
    DescPtrs d;
    const float* edge;
    const int32_t* off;
    int64_t n_chains, n;
    int32_t R;
    Set S;
    Peaks pk;
    PlanBufs wb;
};

constexpr int kFuseBlock = 256;   // k_fuse_costs' block: one row per thread
constexpr int kFuseTileR = 8;     // run lengths up to this many are staged in LDS

__global__ __launch_bounds__(kFuseBlock) void k_fuse_costs(DescPtrs d, const float* __restrict__ edge,
                                                     const int32_t* __restrict__ off,
                                                     int64_t n_chains, int64_t n, int32_t R, Set S,
                                                     Peaks pk, PlanBufs wb)
{
    // parameters read in place (scalar loads at each use), not held in
    // scalar registers across the run loop
    const Set* sc = WM_KERNARG_PTR(FuseArgs, S);
    const Peaks* pc = WM_KERNARG_PTR(FuseArgs, pk);
    const int tl = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * kFuseBlock;
    const int64_t s = s0 + tl;
    if (s == 0) *wb.n_redo = 0u;   // the queue of the planning pass that follows
    // R <= kFuseTileR: the block's costs are staged in LDS and written out
    // row by row (consecutive lanes, consecutive addresses); a lane's own
    // stores to rows s .. s + R - 1 at entry q would touch R * 8-byte pieces
    // of 64 lines each and leave the L2 as that many partial writes
    __shared__ double tile[(kFuseBlock + kFuseTileR - 1) * kFuseTileR];
    __shared__ uint8_t m_s[kFuseBlock], h0_s[kFuseBlock];
    const bool staged = R <= kFuseTileR;
    // the chain holding s: the last c with off[c] <= s (offsets clamped into
    // [0, n] and non-decreasing)
    auto at = [&](int64_t c) -> int64_t {
        const int64_t v = off[c];
        return v < 0 ? 0 : (v > n ? n : v);
    };
    // h0: row s's entries q >= h0 would end runs that start before its chain
    // (never read; written +inf when staged, so that the rows go out whole)
    int32_t m = 0, h0 = 0;
    if (s < n && at(0) <= s) {
        int64_t lo = 0, hi = n_chains;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (at(mid) <= s) lo = mid; else hi = mid;
        }
        const int64_t b = at(lo + 1);
        if (s < b) {
            m = (int32_t)(b - s < (int64_t)R ? b - s : (int64_t)R);
            const int64_t back = s - at(lo) + 1;
            h0 = back < (int64_t)R ? (int32_t)back : R;
        }
    }
    const float inf = __builtin_huge_valf();
    FuseSum fs;
    fuse_begin(fs);
    bool ok = true, unc = false;
    // the next row (and the edge into it) is loaded while this one is
    // evaluated
    Desc<float> xn;
    float en = 0.0f;
    if (m > 0) xn = load_row(d, s);
    for (int32_t q = 0; q < m; ++q) {
        const int64_t k = s + q;
        const Desc<float> x = xn;
        const float ek = en;
        if (q + 1 < m) {
            xn = load_row(d, k + 1);
            en = edge[k];
        }
        if (q > 0) {
            ok = ok && ek >= 0.0f && ek < inf;
            fs.E += (double)ek;
        }
        ok = ok && desc_valid(x);
        float t = inf;
        if (ok) {
            const Set& P = uniform_const(sc);
            const Peaks& K = uniform_const(pc);
            const int32_t dtk = (x.gp >> 11) & 7;
            double pkk = vreg(K.p[0]);
            pkk = dtk == 1 ? vreg(K.p[1]) : pkk;
            pkk = dtk == 2 ? vreg(K.p[2]) : pkk;
            pkk = dtk == 3 ? vreg(K.p[3]) : pkk;
            pkk = dtk == 4 ? vreg(K.p[4]) : pkk;
            fuse_add(fs, x, x.F / (x.u * (float)pkk));
            double Wd = (double)x.W;
            Desc<float> y = x;
            if (q > 0) {
                double pd = vreg(K.p[0]);
                pd = fs.dt == 1 ? vreg(K.p[1]) : pd;
                pd = fs.dt == 2 ? vreg(K.p[2]) : pd;
                pd = fs.dt == 3 ? vreg(K.p[3]) : pd;
                pd = fs.dt == 4 ? vreg(K.p[4]) : pd;
                y = fuse_narrow(fs, pd, Wd);
            }
            Eval<float> E;
            evaluate<float, false>(P.st, P.cf, y, E);
            t = E.T;
            const bool fin = __builtin_isfinite(t);
            unc = unc || (!fin && E.occ != 0) || (fin && t < 0.0f);
            if (P.st.n_levels == 4 && Wd > 0.0) {
                const double c_llc = P.cd.c_llc;
                const double dw = Wd * (1.0 / 1048576.0) - c_llc;
                unc = unc || (dw < 0.0 ? -dw : dw) <= 1e-6 * c_llc;
            }
            t = t == t ? t : inf;
        }
        if (staged) tile[(tl + q) * R + q] = (double)t;
        else wb.cost[k * R + q] = (double)t;
    }
    if (s < n) wb.cov[s] = (uint8_t)(m | (unc ? kPlanUncertain : 0));
    if (!staged) return;
    if (s < n)
        for (int32_t q = h0; q < R; ++q) tile[tl * R + q] = __builtin_huge_val();
    m_s[tl] = (uint8_t)m;
    h0_s[tl] = (uint8_t)h0;
    __syncthreads();
    // Entry (r, q) of a row here comes from the run starting at r - q: from
    // this tile when q <= r (a run of a start here, or row r's +inf when that
    // run leaves its chain) or when q >= h0[r] (+inf); the previous block
    // writes the rest (runs that start in its rows).  r = idx / R exactly
    // (idx < 2^12, R <= 8: the float quotient is at least 1/16 from an integer).
    const float inv_r = 1.0f / (float)R;
    const int64_t left = n - s0;
    const int nrow = left < kFuseBlock ? (int)left : kFuseBlock;
    for (int idx = tl; idx < nrow * R; idx += kFuseBlock) {
        const int r = (int)(((float)idx + 0.5f) * inv_r), q = idx - r * R;
        if (q <= r || q >= (int)h0_s[r]) wb.cost[s0 * R + idx] = tile[idx];
    }
    // runs that start here and end in the next block's first R - 1 rows
    for (int idx = tl; idx < (R - 1) * R; idx += kFuseBlock) {
        const int i = (int)(((float)idx + 0.5f) * inv_r), q = idx - i * R;
        const int st = kFuseBlock + i - q;   // their start, a row here when q > i
        if (q > i && q < (int)m_s[st] && s0 + kFuseBlock + i < n)
            wb.cost[(s0 + kFuseBlock + i) * R + q] = tile[(kFuseBlock + i) * R + q];
    }
}

// Decision margin below which a float32 plan is re-decided in float64.  A
// decision compares two sums of run times, each off by at most the float32
// model's relative error e relative to itself, so it can only flip within
// 2e; the largest e measured on fused runs against the float64 model is
// about 3e-7, so 1e-5 is some 17 times 2e (a test holds it to at least 4).
constexpr double kPlanWindow = 1e-5;

// The dynamic programme runs on groups of GS lanes (GS the power of two >= R),
// one chain per group: lane gl of a group stands for the run of gl + 1 rows
// ending at the current row j and holds prev = best over the rows before
// that run, so that a step is prev + cost, a group minimum (shortest run on
// ties, as a sequential scan with strict improvement picks) and a shift of
// prev by one lane.  Groups of one wave step together over their chains.
template <int GS>
struct PlanGroup {
    int gl, base;   // lane in group, group's first lane
    int64_t c;      // chain (or -1)
    int64_t a, L;   // first row, rows
};

template <int GS>
__device__ inline PlanGroup<GS> plan_group(int64_t c, int64_t n_chains, const int32_t* off,
                                           int64_t n)
{
    PlanGroup<GS> g;
    const int lane = threadIdx.x & 63;
    g.gl = lane & (GS - 1);
    g.base = lane - g.gl;
    g.c = c >= 0 && c < n_chains ? c : -1;
    g.a = 0;
    g.L = 0;
    if (g.c >= 0) {
        int64_t a = off[c], b = off[c + 1];
        a = a < 0 ? 0 : (a > n ? n : a);
        b = b < a ? a : (b > n ? n : b);
        g.a = a;
        g.L = b - a;
    }
    return g;
}

template <int GS>
__device__ inline uint64_t group_mask(const PlanGroup<GS>& g)
{
    return (GS == 64 ? ~0ull : ((1ull << GS) - 1ull)) << g.base;
}

// Lane moves inside a row of 16 lanes (DPP): CTRL 0x140 mirrors the row,
// 0x141 mirrors each half row, 0x4E and 0xB1 swap lanes 2 and 1 apart in each
// quad; 0x138 shifts the wave up by one lane (lane 0 keeps its value).
template <int CTRL>
__device__ inline int32_t dpp32(int32_t x)
{
    return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ inline double dpp64(double x)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)dpp32<CTRL>((int32_t)(uint32_t)u);
    const uint32_t hi = (uint32_t)dpp32<CTRL>((int32_t)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The partner of step k of the group reduction: lanes 16 apart (GS = 32),
// the row mirror (GS >= 16), the half-row mirror (GS >= 8), then 2 and 1 apart
// in the quad; each step doubles the lanes a value covers.
template <int STEP>
__device__ inline double partner(double v)
{
    if constexpr (STEP == 16) return __shfl_xor(v, 16, 64);
    else if constexpr (STEP == 8) return dpp64<0x140>(v);
    else if constexpr (STEP == 4) return dpp64<0x141>(v);
    else if constexpr (STEP == 2) return dpp64<0x4E>(v);
    else return dpp64<0xB1>(v);
}

template <int STEP>
__device__ inline int32_t partner(int32_t v)
{
    if constexpr (STEP == 16) return __shfl_xor(v, 16, 64);
    else if constexpr (STEP == 8) return dpp32<0x140>(v);
    else if constexpr (STEP == 4) return dpp32<0x141>(v);
    else if constexpr (STEP == 2) return dpp32<0x4E>(v);
    else return dpp32<0xB1>(v);
}

template <int STEP>
__device__ inline void argmin_step(double& v, int32_t& len)
{
    const double ov = partner<STEP>(v);
    const int32_t ol = partner<STEP>(len);
    const bool take = (ov < v) | ((ov == v) & (ol < len));
    v = take ? ov : v;
    len = take ? ol : len;
}

// Minimum of (v, len) over the group, ties to the shorter run.
template <int GS>
__device__ inline void group_argmin(double& v, int32_t& len)
{
    if constexpr (GS >= 32) argmin_step<16>(v, len);
    if constexpr (GS >= 16) argmin_step<8>(v, len);
    if constexpr (GS >= 8) argmin_step<4>(v, len);
    if constexpr (GS >= 4) argmin_step<2>(v, len);
    if constexpr (GS >= 2) argmin_step<1>(v, len);
}

template <int GS>
__device__ inline double group_min(double v)
{
    if constexpr (GS >= 32) { const double o = partner<16>(v); v = o < v ? o : v; }
    if constexpr (GS >= 16) { const double o = partner<8>(v); v = o < v ? o : v; }
    if constexpr (GS >= 8) { const double o = partner<4>(v); v = o < v ? o : v; }
    if constexpr (GS >= 4) { const double o = partner<2>(v); v = o < v ? o : v; }
    if constexpr (GS >= 2) { const double o = partner<1>(v); v = o < v ? o : v; }
    return v;
}

// Rows of costs a group loads ahead of its steps (one wait per batch), and
// windows of GS rows whose cut lengths stay in registers (cut bytes of
// rows beyond them go through memory).
constexpr int kPlanBatch = 16;
constexpr int kPlanRegWin = 4;

// Per-lane state of a group's programme: prev (best over the rows before
// this lane's run), the all-singles sum (first lane), best[j], the cut
// length of row w * GS + gl in cutw[w].
struct PlanState {
    double prev, single, best;
    int32_t cutw[kPlanRegWin];
};

// One step of the programme at row j of the group's chain (all lanes of the
// wave call it; `live` marks groups still inside their chain).  t is this
// lane's run cost (ignored where the run is longer than R or than j + 1
// rows).  Updates prev, the all-singles sum (on the group's first lane, whose
// run is the row alone), best and the cut length of row j; with MARGIN,
// `close` is set when the runner-up is within kPlanWindow.
template <int GS, bool MARGIN>
__device__ inline void plan_step(const PlanGroup<GS>& g, int32_t R, int64_t j, bool live,
                                 double t, PlanState& ps, bool& close, uint8_t* __restrict__ cut)
{
    const double inf = __builtin_huge_val();
    const int32_t len = g.gl + 1;
    const bool valid = live & (len <= R) & (len <= j + 1);
    const double v = valid ? ps.prev + t : inf;
    if (valid && g.gl == 0) ps.single += t;
    double bj = v;
    int32_t cj = len;
    group_argmin<GS>(bj, cj);
    if (MARGIN) {
        const double sj = group_min<GS>(len == cj ? inf : v);
        close = close | (live & (sj < inf) & (sj - bj <= kPlanWindow * sj));
    }
    if (live) {
        if (j < (int64_t)kPlanRegWin * GS) {
#pragma unroll
            for (int w = 0; w < kPlanRegWin; ++w)
                if (j == (int64_t)w * GS + g.gl) ps.cutw[w] = cj;
        } else if (g.gl == 0) {
            cut[g.a + j] = (uint8_t)cj;
        }
        ps.best = bj;
    }
    const double up = dpp64<0x138>(ps.prev);   // lane - 1's prev
    ps.prev = g.gl == 0 ? bj : up;
}

// The programme over the group's chain, costs from wb.cost.  With COV, the
// chain's coverage bytes are read with the first batch of costs and `run`
// is narrowed to covered chains without an uncertain run (covered and unc
// report them); without, `run` is taken as given.
template <int GS, bool MARGIN, bool COV>
__device__ inline void plan_run(const PlanGroup<GS>& g, bool& run, int32_t R, const PlanBufs& wb,
                                PlanState& ps, bool& close, bool& covered, bool& unc)
{
    const double inf = __builtin_huge_val();
    const int32_t len = g.gl + 1;
    ps.prev = ps.single = ps.best = 0.0;
#pragma unroll
    for (int w = 0; w < kPlanRegWin; ++w) ps.cutw[w] = 1;
    covered = true;
    unc = false;
    for (int64_t j0 = 0; __ballot(run && j0 < g.L) != 0ull; j0 += kPlanBatch) {
        double t[kPlanBatch];
#pragma unroll
        for (int k = 0; k < kPlanBatch; ++k) {
            const int64_t j = j0 + k;
            t[k] = run && j < g.L && len <= R && len <= j + 1 ? wb.cost[(g.a + j) * R + g.gl] : inf;
        }
        if (COV && j0 == 0) {
            // coverage and uncertain runs, GS rows at a time (loads in flight
            // with the costs above)
            const uint64_t gm = group_mask(g);
            bool bad = false, u = false;
            for (int64_t i = g.gl; i < g.L; i += GS) {
                const uint8_t cv = wb.cov[g.a + i];
                const int64_t want = g.L - i < (int64_t)R ? g.L - i : (int64_t)R;
                bad = bad || (int64_t)(cv & kPlanCount) != want;
                u = u || (cv & kPlanUncertain) != 0;
            }
            covered = (__ballot(bad) & gm) == 0ull;
            unc = (__ballot(u) & gm) != 0ull;
            run = run && covered && !unc;
        }
#pragma unroll 1
        for (int k = 0; k < kPlanBatch; ++k) {
            const int64_t j = j0 + k;
            plan_step<GS, MARGIN>(g, R, j, run && j < g.L, t[k], ps, close, wb.cut);
        }
    }
}

// Start flags of the chosen plan: the run starts found by following the cut
// lengths back from the chain's end, window by window (rows w * GS .. w * GS
// + GS - 1, the window's cut lengths in the group's lanes, the chase by
// shuffles).  `live` marks groups that write their chain's flags.
template <int GS>
__device__ inline void plan_starts(const PlanGroup<GS>& g, bool live, const PlanState& ps,
                                   const uint8_t* __restrict__ cut, uint8_t* __restrict__ start)
{
    const int64_t nw = live ? (g.L + GS - 1) / GS : 0;   // windows of the chain
    // cut bytes beyond the register windows were stored by the group's first
    // lanes: make them visible to the loads below
    if (__ballot(nw > kPlanRegWin) != 0ull) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    int64_t w = nw - 1;
    int64_t jj = live ? g.L : 0;   // the next run start found (row in the chain)
    while (__ballot(w >= 0) != 0ull) {
        const int64_t w0 = w >= 0 ? w * GS : 0;
        const int64_t row = w0 + g.gl;
        const bool mine = w >= 0 && row < g.L;
        int32_t cv = 1;
#pragma unroll
        for (int k = 0; k < kPlanRegWin; ++k) cv = w == k ? ps.cutw[k] : cv;
        if (mine && w >= kPlanRegWin) cv = cut[g.a + row];
        bool flag = mine && row == jj;
        while (__ballot(w >= 0 && jj > w0) != 0ull) {
            const int64_t r = w >= 0 && jj > w0 ? jj - 1 - w0 : 0;
            const int32_t Lr = __shfl(cv, g.base + (int)r, 64);
            if (w >= 0 && jj > w0) {
                jj -= Lr;
                flag = flag || (mine && row == jj);
            }
        }
        if (mine) start[g.a + row] = flag ? 1 : 0;
        --w;
    }
}

// Float32 pass: one group per chain steps through the costs of
// k_fuse_costs.  A chain whose rows were not all costed as its own (offsets
// that are not non-decreasing) gets NaN totals and no start flags; a chain
// holding an uncertain run or a close decision is queued for the float64
// redo; the rest get their totals and start flags.
constexpr int kPlanBlock = 256;    // threads per block of the planning pass (5 blocks per CU)

template <int GS>
__global__ __launch_bounds__(kPlanBlock) void k_plan(const int32_t* __restrict__ off,
                                                      int64_t n_chains, int64_t n, int32_t R,
                                                      PlanBufs wb, double* __restrict__ total,
                                                      double* __restrict__ unfused,
                                                      uint8_t* __restrict__ start)
{
    __shared__ uint32_t wave_q[kPlanBlock / 64 + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GS;
    const PlanGroup<GS> g = plan_group<GS>(gid, n_chains, off, n);
    const uint64_t gm = group_mask(g);
    PlanState ps;
    bool run = g.c >= 0, close = false, covered, unc;
    plan_run<GS, true, true>(g, run, R, wb, ps, close, covered, unc);
    close = unc || (__ballot(close) & gm) != 0ull;
    const bool done = g.c >= 0 && covered && !close;
    // queue slots: one atomic per block, the waves' shares by a prefix in LDS
    const bool queue = g.c >= 0 && covered && close && g.gl == 0;
    const uint64_t qm = __ballot(queue);
    if (lane == 0) wave_q[wid] = (uint32_t)__builtin_popcountll(qm);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sum = 0u;
        for (int w = 0; w < kPlanBlock / 64; ++w) {
            const uint32_t c = wave_q[w];
            wave_q[w] = sum;
            sum += c;
        }
        wave_q[kPlanBlock / 64] = sum != 0u ? atomicAdd(wb.n_redo, sum) : 0u;
    }
    __syncthreads();
    const uint32_t slot = wave_q[kPlanBlock / 64] + wave_q[wid] +
                          (uint32_t)__builtin_popcountll(qm & ((1ull << lane) - 1ull));
    if (g.c >= 0 && g.gl == 0) {
        if (!covered) {
            total[g.c] = __builtin_nan("");
            unfused[g.c] = __builtin_nan("");
        } else if (done) {
            total[g.c] = ps.best;
            unfused[g.c] = ps.single;
        } else if ((int64_t)slot < n) {
            // non-empty chains that partition the rows number at most n
            wb.redo[slot] = g.c;
        } else {
            total[g.c] = __builtin_nan("");
            unfused[g.c] = __builtin_nan("");
        }
    }
    plan_starts(g, done, ps, wb.cut, start);
}

// The queue's length, clamped to what the queue can hold.
__device__ inline int64_t redo_count(const PlanBufs& wb, int64_t n_chains, int64_t n)
{
    int64_t nq = *wb.n_redo;
    nq = nq < n_chains ? nq : n_chains;
    return nq < n ? nq : n;
}

// Float64 redo, costs: each wave takes E <= kRedoChains queued chains (E
// the queue's length over the grid's waves, so that every wave has work
// before any takes several) and lays their (run length, run end) candidates
// end to end over its lanes, ordered by length so that neighbouring lanes
// fuse the same number of rows; each run is formed by fuse_rows and
// evaluated with the float64 model, and the costs replace the chains'
// float32 ones.
constexpr int kRedoChains = 8;

struct RedoArgs {   // k_redo_costs's parameters, in order
    DescPtrs d;
    const float* edge;
    const int32_t* off;
    int64_t n_chains, n;
    int32_t R;
    Set S;
    Peaks pk;
};

__global__ __launch_bounds__(256) void k_redo_costs(DescPtrs d, const float* __restrict__ edge,
                                                     const int32_t* __restrict__ off,
                                                     int64_t n_chains, int64_t n, int32_t R, Set S,
                                                     Peaks pk, PlanBufs wb)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = wave_id();
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const double inf = __builtin_huge_val();
    const int64_t nq = redo_count(wb, n_chains, n);
    int64_t E = (nq + nwaves - 1) / nwaves;
    E = E < 1 ? 1 : (E > kRedoChains ? kRedoChains : E);
    for (int64_t e0 = wave * E; e0 < nq; e0 += nwaves * E) {
        // lanes 0 .. E-1: a chain each, its rows and candidate count
        int64_t a = 0, L = 0, cnt = 0;
        if (lane < E && e0 + lane < nq) {
            const int64_t c = wb.redo[e0 + lane];
            if (c >= 0 && c < n_chains) {
                a = off[c];
                int64_t b = off[c + 1];
                a = a < 0 ? 0 : (a > n ? n : a);
                b = b < a ? a : (b > n ? n : b);
                L = b - a;
                const int64_t r = L < (int64_t)R ? L : (int64_t)R;
                cnt = r * L - r * (r - 1) / 2;   // sum over len <= r of L - len + 1
            }
        }
        // inclusive prefix of the counts over the first kRedoChains lanes
        int64_t inc = cnt;
#pragma unroll
        for (int m = 1; m < kRedoChains; m <<= 1) {
            const int64_t o = __shfl_up(inc, m, 64);
            inc += lane >= m ? o : 0;
        }
        // the chains' running ends, first rows and lengths, read while every
        // lane is active (wave-uniform, so in scalar registers)
        int64_t ends[kRedoChains], as[kRedoChains], Ls[kRedoChains];
#pragma unroll
        for (int k = 0; k < kRedoChains; ++k) {
            ends[k] = read_lane64(inc, k);
            as[k] = read_lane64(a, k);
            Ls[k] = read_lane64(L, k);
        }
        for (int64_t q = lane; q < ends[kRedoChains - 1]; q += 64) {
            int64_t r = q, ca = as[0], cL = Ls[0];
#pragma unroll
            for (int i = 1; i < kRedoChains; ++i) {
                if (q >= ends[i - 1]) {
                    r = q - ends[i - 1];
                    ca = as[i];
                    cL = Ls[i];
                }
            }
            // r -> (len, j): lengths in increasing order, ends j = len-1 .. L-1
            int32_t len = 1;
            while (len < R && r >= cL - len + 1) {
                r -= cL - len + 1;
                ++len;
            }
            const int64_t j = len - 1 + r;
            if (j >= cL) continue;   // r is below the chain's count, so never
            const int64_t s0 = ca + j - len + 1;
            Desc<double> x;
            bool ok;
            if (len == 1) {
                x = widen(load_row(d, s0));
                ok = true;
            } else {
                ok = fuse_rows(d, edge, uniform_const(WM_KERNARG_PTR(RedoArgs, pk)).p, s0, len, x);
            }
            double t = inf;
            if (ok) {
                const Set& P = uniform_const(WM_KERNARG_PTR(RedoArgs, S));
                Eval<double> E;
                evaluate<double, false>(P.st, P.cd, x, E);
                t = E.T == E.T ? E.T : inf;
            }
            wb.cost[(ca + j) * R + (len - 1)] = t;
        }
    }
}

// Float64 redo, plans: one group per queued chain, the programme over the
// float64 costs.
template <int GS>
__global__ __launch_bounds__(256) void k_redo_plan(const int32_t* __restrict__ off,
                                                    int64_t n_chains, int64_t n, int32_t R,
                                                    PlanBufs wb, double* __restrict__ total,
                                                    double* __restrict__ unfused,
                                                    uint8_t* __restrict__ start)
{
    const int64_t nq = redo_count(wb, n_chains, n);
    const int64_t gpw = 64 / GS;   // groups per wave
    const int64_t wave = wave_id();
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int lane = threadIdx.x & 63;
    for (int64_t e0 = wave * gpw; e0 < nq; e0 += nwaves * gpw) {
        const int64_t e = e0 + lane / GS;
        const int64_t c = e < nq ? wb.redo[e] : -1;
        const PlanGroup<GS> g = plan_group<GS>(c, n_chains, off, n);
        PlanState ps;
        bool run = g.c >= 0, unused = false, covered, unc;
        plan_run<GS, false, false>(g, run, R, wb, ps, unused, covered, unc);
        if (g.c >= 0 && g.gl == 0) {
            total[g.c] = ps.best;
            unfused[g.c] = ps.single;
        }
        plan_starts(g, g.c >= 0, ps, wb.cut, start);
    }
}

template <int GS>
static hipError_t plan_launch(const int32_t* off, int64_t n_chains, int64_t n, int32_t R,
                              const PlanBufs& wb, double* total, double* unfused, uint8_t* start,
                              bool redo, hipStream_t s)
{
    if (!redo) {
        const int64_t per_block = kPlanBlock / GS;   // chains per block
        const int64_t nb = (n_chains + per_block - 1) / per_block;
        k_plan<GS><<<(unsigned)nb, kPlanBlock, 0, s>>>(off, n_chains, n, R, wb, total, unfused,
                                                        start);
    } else {
        const int64_t want = (n_chains + 256 / GS - 1) / (256 / GS);
        int64_t b = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_redo_plan<GS>), 256);
        b = b < want ? b : want;
        b = b < 1 ? 1 : b;
        k_redo_plan<GS><<<(unsigned)b, 256, 0, s>>>(off, n_chains, n, R, wb, total, unfused, start);
    }
    return hipGetLastError();
}

static hipError_t plan_dispatch(int32_t gs, const int32_t* off, int64_t n_chains, int64_t n,
                                int32_t R, const PlanBufs& wb, double* total, double* unfused,
                                uint8_t* start, bool redo, hipStream_t s)
{
    switch (gs) {
    case 1: return plan_launch<1>(off, n_chains, n, R, wb, total, unfused, start, redo, s);
    case 2: return plan_launch<2>(off, n_chains, n, R, wb, total, unfused, start, redo, s);
    case 4: return plan_launch<4>(off, n_chains, n, R, wb, total, unfused, start, redo, s);
    case 8: return plan_launch<8>(off, n_chains, n, R, wb, total, unfused, start, redo, s);
    case 16: return plan_launch<16>(off, n_chains, n, R, wb, total, unfused, start, redo, s);
    default: return plan_launch<32>(off, n_chains, n, R, wb, total, unfused, start, redo, s);
    }
}

hipError_t launch_plan_fusion(const DescPtrs& d, const float* edge, const int32_t* off,
                              int64_t n_chains, int64_t n, int32_t R, const Set& S,
                              const double* peaks, const PlanBufs& wb, double* total,
                              double* unfused, uint8_t* start, hipStream_t s)
{
    if (n_chains <= 0) return hipSuccess;
    Peaks pk;
    for (int t = 0; t < 5; ++t) pk.p[t] = peaks[t];
    int32_t gs = 1;
    while (gs < R) gs <<= 1;   // R <= 32
    // at least one block, so that the queue's length is cleared even with no rows
    const int64_t nb = n > 0 ? (n + kFuseBlock - 1) / kFuseBlock : 1;
    k_fuse_costs<<<(unsigned)nb, kFuseBlock, 0, s>>>(d, edge, off, n_chains, n, R, S, pk, wb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = plan_dispatch(gs, off, n_chains, n, R, wb, total, unfused, start, false, s);
    if (e != hipSuccess) return e;
    const int64_t want = (n_chains + 3) / 4;
    int64_t nb3 = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_redo_costs), 256) * 2;
    nb3 = nb3 < want ? nb3 : want;
    nb3 = nb3 < 1 ? 1 : nb3;
    k_redo_costs<<<(unsigned)nb3, 256, 0, s>>>(d, edge, off, n_chains, n, R, S, pk, wb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return plan_dispatch(gs, off, n_chains, n, R, wb, total, unfused, start, true, s);
}

}  // namespace wm
