// wm_model.hpp -- per-descriptor evaluation of the CDNA wavefront-centric
// execution-time model (Section IV-B), templated on the arithmetic type:
// float for the bulk sweeps, double for the rare re-evaluations that decide a
// subgradient, a loss sign or a near-tied tile.
//
// The terms, in the order they are evaluated:
//   occupancy  o = min(VGPR limit, wave-slot limit, LDS limit) workgroups/CU,
//              generalising the VGPR-limited wavefront count of Section IV-B;
//   rounds     n_r = ceil(G / (N_CU o)), the N_ctas/(N_CU W_eff) of Eq. (14);
//   traffic    served fractions s_l = h_l prod_{m<l}(1 - h_m) (Eq. (10)), the
//              LLC hit rate from Table "hlcc-piecewise" when W > 0, the HBM
//              bandwidth blended by Eq. (16);
//   stages     T_c = F/(u P) (Eq. (11)), T_b = B / sum s_l BW_l,
//              T_lat = n_r (B / (G k L_w)) sum s_l Lat_l / f (Eq. (10) x rounds);
//   combine    max of the stages (Eq. (1), Eq. (14)) or the occupancy-overlap
//              step (Eq. (9), Eq. (12)), plus the overheads of Eq. (13),
//              Eq. (14), the interference / multi-GPU / fusion terms of
//              Section IV-B and the per-sync term of Section IV-E.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define WM_HD __host__ __device__ inline

namespace wm {

constexpr int kTheta = 24;
constexpr int kAcc = 26;  // loss, count, 24 gradient slots

// structural integers of a parameter set, as the kernels use them
struct Struct {
    int32_t n_levels, n_cu, n_simd, wave_shift, vgpr_simd, vgpr_gran_mask, waves_simd, lds_cu,
        lds_gran_mask, mwp, cwp, combine, bytes_inflight_wave, pad_;
    double f_clk, w_lo_mib, c_llc_mib;
};

// theta-derived constants in the arithmetic type R
template <typename R>
struct Const {
    R inv_peak[5];
    R bw[4];     // L1, L2, LLC, HBM
    R latf[4];   // Lat_l / f_clk, seconds
    R ov[7];     // T_launch, tau_wg, tau_bar, tau_interf, tau_gpu, tau_fusion, tau_sync
    R alpha, beta;
    R blend_k;   // -log2(e) / w0: exp(-W/w0) = exp2(W * blend_k)
    R bp_minus_bw;
    R dw0_coef;  // (B_peak - BW_HBM) / w0^2 (0 without the blend): dS/dw0 = s_hbm e W dw0_coef
    R inv_lw;    // 1 / bytes in flight per wave
    R inv_f;     // 1 / f_clk
    R w_lo, c_llc, inv_span;  // MiB
    int32_t blend_on, pad_;
};

// Everything a kernel needs about one parameter set.
struct Set {
    Struct st;
    Const<float> cf;
    Const<double> cd;
};

// One group k of the theta-derived constants (k < kConstFields), so that a
// device rebuild can give each group to its own lane.
constexpr int kConstFields = 21;
template <typename R>
WM_HD void const_field(const double* th, const Struct& s, Const<R>& c, int k)
{
    const bool blend = th[22] > 0.0;
    if (k < 5) {
        c.inv_peak[k] = (R)(1.0 / th[8 + k]);
    } else if (k < 9) {
        const int l = k - 5;
        c.bw[l] = (R)th[l];
        c.latf[l] = (R)(th[4 + l] / s.f_clk);
    } else if (k < 16) {
        c.ov[k - 9] = (R)th[13 + (k - 9)];
    } else if (k == 16) {
        c.alpha = (R)th[20];
        c.beta = (R)th[21];
        c.blend_on = blend ? 1 : 0;
        c.pad_ = 0;
        c.w_lo = (R)s.w_lo_mib;
        c.c_llc = (R)s.c_llc_mib;
    } else if (k == 17) {
        c.dw0_coef = blend ? (R)((th[23] - th[3]) / (th[22] * th[22])) : (R)0;
    } else if (k == 18) {
        c.blend_k = blend ? (R)(-1.4426950408889634 / th[22]) : (R)0;
    } else if (k == 19) {
        c.bp_minus_bw = (R)(th[23] - th[3]);
        c.inv_lw = (R)(1.0 / (double)s.bytes_inflight_wave);
    } else if (k == 20) {
        c.inv_f = (R)(1.0 / s.f_clk);
        c.inv_span = (R)(1.0 / (s.c_llc_mib - s.w_lo_mib));
    }
}

template <typename R>
WM_HD void make_const(const double* th, const Struct& s, Const<R>& c)
{
    for (int k = 0; k < kConstFields; ++k) const_field<R>(th, s, c, k);
}

// ---------------------------------------------------------------------------
// arithmetic helpers: hardware reciprocal in float, IEEE division in double
// ---------------------------------------------------------------------------
template <typename R> struct Ar;
template <> struct Ar<float> {
    static __device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    // hardware base-2 logarithm / exponential (v_log_f32, v_exp_f32)
    static __device__ inline float lg2(float x) { return __builtin_amdgcn_logf(x); }
    static __device__ inline float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
};
template <> struct Ar<double> {
    static __device__ inline double rcp(double x) { return 1.0 / x; }
    static __device__ inline double lg2(double x) { return log2(x); }
    static __device__ inline double ex2(double x) { return exp2(x); }
};

// floor(a / b) for a < 2^24, 1 <= b < 2^24 and a quotient below 2^21: the
// float estimate a * rcp(b) is within 0.37 of a / b (rcp 1 ulp, product
// 0.5 ulp), so truncation is off by at most one, which the remainder fixes.
__device__ inline uint32_t udiv_small(uint32_t a, uint32_t b)
{
    uint32_t q = (uint32_t)((float)a * __builtin_amdgcn_rcpf((float)b));
    const int32_t r = (int32_t)(a - __umul24(q, b));   // q, b < 2^24: low 32 bits
    q = r < 0 ? q - 1u : (r >= (int32_t)b ? q + 1u : q);
    return q;
}

// floor(a / b) for integers a < 2^21 and 1 <= b < 2^24 without a remainder
// correction.  With q = floor(a / b), the value (a + 1/2) / b lies in
// [q + 1/(2b), q + 1 - 1/(2b)].  a + 1/2 and b are exact in float, the
// hardware reciprocal is within 1 ulp (2^-23 relative) and the product adds
// one rounding (2^-24), so the estimate is within (a + 1/2)/b * 1.51 * 2^-23
// of (a + 1/2) / b, which is below 1/(2b) whenever a + 1/2 < 2.7e6: the
// estimate stays strictly inside (q, q + 1) and truncation gives q.
__device__ inline uint32_t udiv21(uint32_t a, uint32_t b)
{
    return (uint32_t)(((float)a + 0.5f) * __builtin_amdgcn_rcpf((float)b));
}

// x finite and >= 0 (-0 included): one class test instead of two compares
__device__ inline bool finite_nonneg(float x) { return __builtin_amdgcn_classf(x, 0x1E0); }
__device__ inline bool finite_nonneg(double x) { return x >= 0.0 && x < __builtin_huge_val(); }

// A copy of v in a register that the optimiser cannot see through.  A
// per-lane select among parameters (the peak of the descriptor's dtype, the
// h_LLC exponent of its regime, the scale of a segment's class) written on
// such copies stays a register select; on the parameters themselves the
// compiler may turn it into a per-lane indexed load from the kernel-argument
// segment, a vector memory access with its latency inside the evaluation.
// float (the bulk sweeps): a scalar register, which v_cndmask reads
// directly -- the sweeps' parameter sets are wave-uniform, and a divergent
// one would not compile; double (the rare re-evaluations): a vector register.
__device__ inline float vreg(float v)
{
    asm("" : "+s"(v));
    return v;
}
__device__ inline double vreg(double v)
{
    asm("" : "+v"(v));
    return v;
}

template <typename R>
struct Desc {
    R F, B, r1, r2, r3, K, u, W;
    int32_t v, s, gp, G;
};

// ---------------------------------------------------------------------------
// occupancy (exact integers)
// ---------------------------------------------------------------------------
struct Occ {
    int32_t o, k;
};

__device__ inline Occ occupancy(const Struct& st, int32_t v, int32_t s, int32_t g)
{
    // the first two dividends are below 2^21 by the parameter limits
    // (VGPR_SIMD <= 65536, N_SIMD * waves <= 1024): udiv21 is exact; the LDS
    // dividend reaches 2^24 and takes udiv_small
    Occ r;
    r.k = (g + (1 << st.wave_shift) - 1) >> st.wave_shift;
    int32_t w = 0;
    if (v <= st.vgpr_simd) {
        int32_t va = (v + st.vgpr_gran_mask) & ~st.vgpr_gran_mask;
        w = (int32_t)udiv21((uint32_t)st.vgpr_simd, (uint32_t)va);
        w = w < st.waves_simd ? w : st.waves_simd;
    }
    int32_t o = (int32_t)udiv21(__umul24((uint32_t)st.n_simd, (uint32_t)w), (uint32_t)r.k);
    if (s > 0) {
        int32_t ol = 0;
        if (s <= st.lds_cu) {
            int32_t sa = (s + st.lds_gran_mask) & ~st.lds_gran_mask;
            // o_l only matters below o_w <= 1024: cap it there so the quotient stays small
            ol = (sa <= (st.lds_cu >> 10)) ? 1024 : (int32_t)udiv_small((uint32_t)st.lds_cu, (uint32_t)sa);
        }
        o = o < ol ? o : ol;
    }
    r.o = o;
    return r;
}

template <typename R>
__device__ inline bool desc_valid(const Desc<R>& d)
{
    const bool fF = finite_nonneg(d.F), fB = finite_nonneg(d.B), fK = finite_nonneg(d.K),
               fW = finite_nonneg(d.W);
    bool ok = fF & fB & fK & fW & (d.u > (R)0) & (d.u <= (R)1) &
              (d.r1 >= (R)0) & (d.r1 <= (R)1) & (d.r2 >= (R)0) & (d.r2 <= (R)1) &
              (d.r3 >= (R)0) & (d.r3 <= (R)1) & (d.v >= 1) & (d.s >= 0) & (d.G >= 1) &
              ((uint32_t)d.gp < (1u << 25));
    int32_t g = d.gp & 2047;
    int32_t dt = (d.gp >> 11) & 7;
    ok = ok & (g >= 1) & (g <= 1024) & (dt <= 4);
    return ok;
}

// ---------------------------------------------------------------------------
// one evaluation
// ---------------------------------------------------------------------------
template <typename R>
struct Eval {
    R T;
    int32_t occ;       // -1 invalid, 0 infeasible, else o
    int32_t dt, nr, G;
    int32_t cnt[4];    // n_conc - 1, n_dev - 1, fused, n_sync
    int32_t llc_regime;  // 0 none/resident, 1 transition, 2 streaming
    R h3, s1, s2, s3, sh, a12, S, Lf, e, bwh, W;
    R Tc, Tb, Tlat, Tm;
    R wc, wb, wl;      // dT/dT_c, dT/dT_b, dT/dT_lat
    R nrK, base_log;   // n_r K; ln(base) (transition) or ln(C/W_MiB) (streaming)
    R q;               // n_r * B / (G k L_w): serialised load batches
    R ip, iS;          // 1 / P of the descriptor's dtype, 1 / S
    bool near_kink;    // within 1e-5 relative of a max/min switch
};

// TILE: the descriptor comes from derive_tile, so it is valid by
// construction and has r1 = r3 = 0, W = 0, u = 1 and no concurrency, device,
// fusion or sync counts; the terms those zeros and ones cancel are skipped.
template <typename R, bool FULL, bool TILE = false>
__device__ inline void evaluate(const Struct& st, const Const<R>& c, const Desc<R>& d, Eval<R>& E)
{
    typedef Ar<R> A;
    E.T = (R)__builtin_nan("");
    E.occ = -1;
    if (!TILE && !desc_valid(d)) return;
    const int32_t g = d.gp & 2047;
    const int32_t dt = (d.gp >> 11) & 7;
    E.dt = dt;
    E.cnt[0] = TILE ? 0 : (d.gp >> 14) & 7;
    E.cnt[1] = TILE ? 0 : (d.gp >> 17) & 7;
    E.cnt[2] = TILE ? 0 : (d.gp >> 20) & 1;
    E.cnt[3] = TILE ? 0 : (d.gp >> 21) & 15;
    E.G = d.G;

    Occ oc = occupancy(st, d.v, d.s, g);
    E.occ = oc.o;
    if (oc.o == 0) {
        E.T = (R)__builtin_huge_val();
        return;
    }
    // n_cu <= 65536 and o <= 1024: 24-bit multiplies are exact
    const uint32_t per_round = __umul24((uint32_t)st.n_cu, (uint32_t)oc.o);
    const uint32_t num = (uint32_t)d.G + per_round - 1u;
    // udiv21 is exact below 2^21 (per_round <= num is then below 2^21 too);
    // larger counts (grids beyond ~2^21 workgroups) take an exact division,
    // behind a branch that the whole wave skips unless one of its lanes needs it
    const bool big = num >= (1u << 21);
    uint32_t nru = udiv21(big ? 0u : num, big ? 1u : per_round);
    if (__builtin_expect(__ballot(big) != 0, 0)) {
        if (big) nru = num / per_round;
    }
    const int32_t nr = (int32_t)nru;
    E.nr = nr;

    // traffic split: with W > 0 and an LLC, h_LLC(W) replaces r3
    // (Table "hlcc-piecewise"): 1 below W_lo, base^alpha in the transition
    // zone, (C/W)^beta above C -- one log2/exp2 pair for every regime
    R h3 = d.r3;
    E.llc_regime = 0;
    E.base_log = (R)0;
    if (!TILE && st.n_levels == 4 && d.W > (R)0) {
        const R Wm = d.W * (R)(1.0 / 1048576.0);
        const int reg = Wm < c.w_lo ? 0 : (Wm <= c.c_llc ? 1 : 2);
        // (1 - (W - W_lo)/(C - W_lo)) written as (C - W)/(C - W_lo): same
        // value, no cancellation near C
        R x = reg == 1 ? (c.c_llc - Wm) * c.inv_span : c.c_llc * A::rcp(Wm);
        x = reg == 0 ? (R)1 : x;
        const R y = reg == 1 ? vreg(c.alpha) : vreg(c.beta);
        const R l2 = A::lg2(x);
        h3 = x > (R)0 ? A::ex2(y * l2) : (R)0;
        E.llc_regime = reg;
        if (FULL) E.base_log = x > (R)0 ? l2 * (R)0.69314718055994531 : (R)0;
    }
    const R m1 = TILE ? (R)1 : (R)1 - d.r1;
    const R s1 = TILE ? (R)0 : d.r1;
    const R s2 = TILE ? d.r2 : m1 * d.r2;
    const R a12 = TILE ? (R)1 - d.r2 : m1 * ((R)1 - d.r2);
    R s3 = (R)0, sh = a12;
    if (!TILE && st.n_levels == 4) {
        s3 = a12 * h3;
        sh = a12 * ((R)1 - h3);
    }
    // Eq. (16) blend of the HBM bandwidth
    R e = (R)0, bwh = c.bw[3];
    if (!TILE && c.blend_on && d.W > (R)0) {
        e = A::ex2(d.W * c.blend_k);
        bwh = c.bw[3] + c.bp_minus_bw * e;
    }
    const R S = TILE ? s2 * c.bw[1] + sh * bwh : s1 * c.bw[0] + s2 * c.bw[1] + s3 * c.bw[2] + sh * bwh;
    const R Lf = TILE ? s2 * c.latf[1] + sh * c.latf[3]
                      : s1 * c.latf[0] + s2 * c.latf[1] + s3 * c.latf[2] + sh * c.latf[3];

    // stage times
    R ip;
    if (TILE) {   // dtype uniform over the wave: scalar selects
        ip = c.inv_peak[0];
        ip = dt == 1 ? c.inv_peak[1] : ip;
        ip = dt == 2 ? c.inv_peak[2] : ip;
        ip = dt == 3 ? c.inv_peak[3] : ip;
        ip = dt == 4 ? c.inv_peak[4] : ip;
    } else {
        ip = vreg(c.inv_peak[0]);
        ip = dt == 1 ? vreg(c.inv_peak[1]) : ip;
        ip = dt == 2 ? vreg(c.inv_peak[2]) : ip;
        ip = dt == 3 ? vreg(c.inv_peak[3]) : ip;
        ip = dt == 4 ? vreg(c.inv_peak[4]) : ip;
    }
    const R Tc = TILE ? d.F * ip : d.F * ip * A::rcp(d.u);
    const R iS = A::rcp(S);
    const R Tb = d.B * iS;
    const R q = (R)nr * d.B * A::rcp((R)d.G * (R)oc.k) * c.inv_lw;
    const R Tlat = q * Lf;

    const R nrK = (R)nr * d.K;
    const R Tov = TILE ? c.ov[0] + c.ov[1] * (R)d.G + c.ov[2] * nrK
                       : c.ov[0] + c.ov[1] * (R)d.G + c.ov[2] * nrK + (R)E.cnt[0] * c.ov[3] +
                             (R)E.cnt[1] * c.ov[4] + (R)E.cnt[2] * c.ov[5] + (R)E.cnt[3] * c.ov[6];

    R wc = (R)0, wb = (R)0, wl = (R)0, step;
    const bool mem_b = Tb >= Tlat;
    const R Tm = mem_b ? Tb : Tlat;
    bool near = false;
    const R tol = (R)1e-5;
    if (st.combine == 0) {
        if (Tc >= Tb && Tc >= Tlat) {
            step = Tc;
            wc = (R)1;
            if (FULL) near = (Tc - Tm) <= tol * Tc;
        } else {
            step = Tm;
            if (mem_b) wb = (R)1; else wl = (R)1;
            if (FULL) {
                const R second = Tc > (mem_b ? Tlat : Tb) ? Tc : (mem_b ? Tlat : Tb);
                near = (Tm - second) <= tol * Tm;
            }
        }
    } else {
        int32_t neff = (int32_t)__umul24((uint32_t)oc.o, (uint32_t)oc.k);
        if (st.mwp > 0) neff = neff < st.mwp ? neff : st.mwp;
        if (st.cwp > 0) neff = neff < st.cwp ? neff : st.cwp;
        const R a = (R)(neff - 1);
        R dTc, dTm;
        R eta;
        if (neff == 1) {
            eta = (R)0;
            dTc = (R)1;
            dTm = (R)1;
        } else if (a * Tc >= Tm) {
            eta = (R)1;
            dTc = (R)0.5;
            dTm = (R)0.5;
        } else {
            eta = a * Tc * A::rcp(Tm);
            const R den = Tm + a * Tc;
            const R iden2 = A::rcp(den * den);
            dTc = Tm * Tm * ((R)1 - a) * iden2;
            dTm = (Tm * Tm + (R)2 * a * Tm * Tc + a * Tc * Tc) * iden2;
        }
        const R num = Tm + Tc;
        step = num == (R)0 ? (R)0 : num * A::rcp((R)1 + eta);
        wc = dTc;
        if (mem_b) wb = dTm; else wl = dTm;
        if (FULL) {
            const R mn = mem_b ? Tlat : Tb;
            near = (Tm - mn) <= tol * Tm;
            if (neff > 1) {
                const R sw = a * Tc - Tm;
                near = near || ((sw < (R)0 ? -sw : sw) <= tol * Tm);
            }
        }
    }
    E.T = Tov + step;
    if (FULL) {
        E.h3 = h3; E.s1 = s1; E.s2 = s2; E.s3 = s3; E.sh = sh; E.a12 = a12;
        E.S = S; E.Lf = Lf; E.e = e; E.bwh = bwh; E.W = d.W;
        E.Tc = Tc; E.Tb = Tb; E.Tlat = Tlat; E.Tm = Tm;
        E.wc = wc; E.wb = wb; E.wl = wl; E.nrK = nrK; E.q = q; E.ip = ip; E.iS = iS;
        E.near_kink = near;
    }
}

// dT/dtheta_j of an evaluated descriptor times `w`, added into acc[2 + j].
// The weight is folded into each stage's coefficient once, so every slot
// costs one multiply-add.  R is the accumulator type too: float for the
// bulk sweeps (per-lane partial sums, reduced in float64 across lanes,
// waves and blocks), double for the float64 re-evaluations.  The split form
// adds the seven overhead slots (acc[15 .. 21]) into ovh[0 .. 6] instead, so
// that a sweep can keep those sums apart (in LDS); acc and ovh are anything
// indexable by slot.
template <typename R, typename A, typename B>
__device__ inline void accumulate_partials_split(const Struct& st, const Const<R>& c, const Eval<R>& E, R w, A acc,
                                                 B ovh)
{
    // overhead slots: data only
    ovh[0] += w;
    ovh[1] += w * (R)E.G;
    ovh[2] += w * E.nrK;
    ovh[3] += w * (R)E.cnt[0];
    ovh[4] += w * (R)E.cnt[1];
    ovh[5] += w * (R)E.cnt[2];
    ovh[6] += w * (R)E.cnt[3];
    // compute: d(F/(uP))/dP = -T_c / P
    const R gP = -(w * E.wc) * E.Tc * E.ip;
    acc[2 + 8] += E.dt == 0 ? gP : (R)0;
    acc[2 + 9] += E.dt == 1 ? gP : (R)0;
    acc[2 + 10] += E.dt == 2 ? gP : (R)0;
    acc[2 + 11] += E.dt == 3 ? gP : (R)0;
    acc[2 + 12] += E.dt == 4 ? gP : (R)0;
    // bandwidth: dT_b/dX = -(T_b / S) dS/dX.  Without the working-set blend
    // e = 0, which zeroes the B_peak and w0 terms; outside the h_LLC regimes
    // base_log = 0 -- so every slot is updated unconditionally.
    const R cb = -(w * E.wb) * E.Tb * E.iS;
    const R cbh = cb * E.sh;
    acc[2 + 0] += cb * E.s1;
    acc[2 + 1] += cb * E.s2;
    acc[2 + 2] += cb * E.s3;
    acc[2 + 3] += cbh * ((R)1 - E.e);
    acc[2 + 23] += cbh * E.e;
    acc[2 + 22] += (cbh * E.e) * (E.W * c.dw0_coef);
    // latency: T_lat = q * sum s_l Lat_l / f
    const R clq = (w * E.wl) * E.q;
    const R cl = clq * c.inv_f;
    acc[2 + 4] += cl * E.s1;
    acc[2 + 5] += cl * E.s2;
    acc[2 + 6] += cl * E.s3;
    acc[2 + 7] += cl * E.sh;
    // h_LLC(W) exponents through s3 and s_hbm
    const R dTdh = E.a12 * (cb * (c.bw[2] - E.bwh) + clq * (c.latf[2] - c.latf[3]));
    const R gh = dTdh * E.h3 * E.base_log;
    acc[2 + 20] += E.llc_regime == 1 ? gh : (R)0;
    acc[2 + 21] += E.llc_regime == 2 ? gh : (R)0;
}

template <typename R>
__device__ inline void accumulate_partials(const Struct& st, const Const<R>& c, const Eval<R>& E, R w, R* acc)
{
    accumulate_partials_split<R>(st, c, E, w, acc, acc + 15);
}

}  // namespace wm
