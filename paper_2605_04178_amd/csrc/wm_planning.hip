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
// R consecutive kernels; every (run end, run length) candidate is turned into
// a combined descriptor and evaluated in float64 (one wave per chain, lanes
// over candidates), then one thread per chain runs the prefix dynamic
// programme over those costs.
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

// One wave per group (persistent).  Candidate k (a valid training row) is
// the multiplier when its cumulative weight C_k = sum of w_i over valid
// training rows with (x_i, i) <= (x_k, k) reaches half the total and no
// smaller candidate does; the smallest such (x_k, k) wins.  Per wave the
// stats (training loss, count, held-out loss, count) accumulate in float64;
// lane 0 of each wave writes them to its row.
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
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    double st[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t g = wave; g < n_groups; g += nwaves) {
        int64_t a = off[g], b = off[g + 1];
        a = a < 0 ? 0 : (a > n ? n : a);
        b = b < a ? a : (b > n ? n : b);
        // total training weight (row order)
        double Wt = 0.0;
        for (int64_t i = a + lane; i < b; i += 64) {
            const double t = T[i], m = meas[i];
            if (train[i] && mult_ok(t, m)) Wt += t / m;
        }
        {
            double v[1] = {Wt};
            wave_sum<1>(v);
            Wt = v[0];
        }
        // best candidate: smallest (x_k, k) with C_k >= W/2
        double bx = __builtin_huge_val();
        int64_t bk = INT64_MAX;
        for (int64_t k = a + lane; k < b; k += 64) {
            const double tk = T[k], mk = meas[k];
            if (!(train[k] && mult_ok(tk, mk))) continue;
            const double xk = mk / tk;
            double C = 0.0;
            for (int64_t i = a; i < b; ++i) {
                const double t = T[i], m = meas[i];
                if (!(train[i] && mult_ok(t, m))) continue;
                const double xi = m / t;
                if (xi < xk || (xi == xk && i <= k)) C += t / m;
            }
            if (C >= 0.5 * Wt && (xk < bx || (xk == bx && k < bk))) {
                bx = xk;
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
        for (int64_t i = a + lane; i < b; i += 64) {
            const double t = T[i], m = meas[i];
            T_scaled[i] = (float)(mu * t);
            if (!mult_ok(t, m)) continue;
            const double e = __builtin_fabs(mu * t - m) / m;
            if (train[i]) {
                st[0] += e;
                st[1] += 1.0;
            } else {
                st[2] += e;
                st[3] += 1.0;
            }
        }
    }
    wave_sum<4>(st);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) rows[wave * 4 + j] = st[j];
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
    const int64_t want = (n_groups + 3) / 4;  // 4 waves per block
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
    k_fit_mult_reduce<<<1, 256, 0, s>>>(rows, (int64_t)nb * 4, stats);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fusion planning
// ---------------------------------------------------------------------------
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
        const Desc<float> x = load_desc(d, k);
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

// One wave per chain: cost[(row) * R + len - 1] for every run of len rows
// ending at that row (float64; +inf for runs that leave the chain or hold an
// invalid row or edge, and for NaN times).
__global__ __launch_bounds__(256) void k_fuse_costs(DescPtrs d, const float* __restrict__ edge,
                                                     const int32_t* __restrict__ off,
                                                     int64_t n_chains, int64_t n, int32_t R, Set S,
                                                     Peaks pk, double* __restrict__ cost)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const double inf = __builtin_huge_val();
    for (int64_t c = wave; c < n_chains; c += nwaves) {
        int64_t a = off[c], b = off[c + 1];
        a = a < 0 ? 0 : (a > n ? n : a);
        b = b < a ? a : (b > n ? n : b);
        const int64_t ncand = (b - a) * R;
        for (int64_t q = lane; q < ncand; q += 64) {
            const int64_t j = q / R;                 // row in the chain (run end)
            const int32_t len = (int32_t)(q - j * R) + 1;
            double t = inf;
            if (len <= j + 1) {
                const int64_t s0 = a + j - len + 1;
                Desc<double> x;
                bool ok;
                if (len == 1) {
                    x = widen(load_desc(d, s0));
                    ok = true;
                } else {
                    ok = fuse_rows(d, edge, pk.p, s0, len, x);
                }
                if (ok) {
                    Eval<double> E;
                    evaluate<double, false>(S.st, S.cd, x, E);
                    t = E.T == E.T ? E.T : inf;
                }
            }
            cost[(a + j) * R + (len - 1)] = t;
        }
    }
}

// One thread per chain: best[j] = min over len (1 .. R, shortest first,
// strict improvement) of best[j - len] + cost(run of len rows ending at j).
// The run lengths of the chosen plan are kept in `cut` (one byte per row of
// workspace) for the backward pass that writes the start flags.
__global__ __launch_bounds__(256) void k_plan(const int32_t* __restrict__ off, int64_t n_chains,
                                               int64_t n, int32_t R,
                                               const double* __restrict__ cost,
                                               double* __restrict__ best_ws,
                                               uint8_t* __restrict__ cut,
                                               double* __restrict__ total,
                                               double* __restrict__ unfused,
                                               uint8_t* __restrict__ start)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chains) return;
    int64_t a = off[c], b = off[c + 1];
    a = a < 0 ? 0 : (a > n ? n : a);
    b = b < a ? a : (b > n ? n : b);
    const double inf = __builtin_huge_val();
    double single = 0.0;
    // best_ws[a + j] holds best over the first j + 1 rows
    for (int64_t j = 0; j < b - a; ++j) {
        double bj = inf;
        int32_t cj = 1;
        for (int32_t len = 1; len <= R && len <= j + 1; ++len) {
            const double t = cost[(a + j) * R + (len - 1)];
            if (len == 1) single += t;
            const double prev = j + 1 - len == 0 ? 0.0 : best_ws[a + j - len];
            const double v = prev + t;
            if (v < bj) {
                bj = v;
                cj = len;
            }
        }
        best_ws[a + j] = bj;
        cut[a + j] = (uint8_t)cj;
    }
    total[c] = b > a ? best_ws[b - 1] : 0.0;
    unfused[c] = single;
    for (int64_t i = a; i < b; ++i) start[i] = 0;
    int64_t j = b - a;
    while (j > 0) {
        const int32_t L = cut[a + j - 1];
        start[a + j - L] = 1;
        j -= L;
    }
}

hipError_t launch_plan_fusion(const DescPtrs& d, const float* edge, const int32_t* off,
                              int64_t n_chains, int64_t n, int32_t R, const Set& S,
                              const double* peaks, double* cost, double* best, uint8_t* cut,
                              double* total, double* unfused, uint8_t* start, hipStream_t s)
{
    if (n_chains <= 0) return hipSuccess;
    Peaks pk;
    for (int t = 0; t < 5; ++t) pk.p[t] = peaks[t];
    const int64_t want = (n_chains + 3) / 4;
    int64_t nb = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_fuse_costs), 256) * 2;
    nb = nb < want ? nb : want;
    nb = nb < 1 ? 1 : nb;
    k_fuse_costs<<<(int)nb, 256, 0, s>>>(d, edge, off, n_chains, n, R, S, pk, cost);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb2 = (n_chains + 255) / 256;
    k_plan<<<(unsigned)nb2, 256, 0, s>>>(off, n_chains, n, R, cost, best, cut, total, unfused, start);
    return hipGetLastError();
}

}  // namespace wm
