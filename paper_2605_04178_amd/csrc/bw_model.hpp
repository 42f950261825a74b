// bw_model.hpp -- per-descriptor evaluation of the Blackwell stage-centric
// execution-time model (Section IV-A), templated on the arithmetic type:
// float for the bulk sweeps, double for the re-evaluations that decide a
// subgradient or a loss sign.
//
// One descriptor is one tile kernel (bM x bN x bK tile, Kt K-steps, G CTAs,
// flags: dtype, 2-SM pair, TMEM strategy, multicast participants, barriers,
// compressed operands; compression ratio; output element bytes).  Per
// K-step:
//   T_TMEM    = (acc + [strategy B] A tile) / BW_TMEM_read + L_mma / f
//               + acc / BW_TMEM_write                                Eq. (2)
//   T_compute = 2 bM bN bK / (R_TC[dtype] S_mode) + T_TMEM
//               + (L_alloc + L_dealloc) / f / Kt                     Eq. (3)
//   T_tma     = L_TMA / f + (M_A / P_A + M_B' / P_B) / B_TMA          Eq. (4)
//               (M_B' = M_B / 2 for a 2-SM pair, Eq. (6))
//   T_decomp  = [compressed] (M_A + M_B) / (CR BW_link eta_DE)
//               + [FP4] ((M_A + M_B) / R_decomp + L_setup / f)        Eq. (5)
//   T_dsm     = [pair] M_B / 2 / BW_dsmem                            Eq. (6)
//   T_sync    = N_bar L_mbar / f + [pair] L_commit / f
//   T_io      = eps (T_tma + T_decomp + T_dsm) + T_sync              Eq. (7)
//   T_step    = max(T_compute, T_io) + T_sync + O_misc               Eq. (8)
// and the kernel T = T_launch + n_r (Kt T_step + T_store), T_store = bM bN
// ob / B_gmem + L_store / f, n_r = ceil(G / (N_SM c)), c = min(max_cta,
// floor(TMEM / accumulator bytes)) (0 = the accumulator does not fit: +inf).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wm_model.hpp"

namespace wm {

constexpr int kBwTheta = 24;

struct BwStruct {
    int32_t n_sm, max_cta;
    int64_t tmem_bytes;
    double f_clk;
};

// theta-derived constants in the arithmetic type R
template <typename R>
struct BwConst {
    R inv_tr, inv_tw;      // 1 / TMEM read, write rate
    R lmma;                // L_mma / f
    R inv_rtc[5];          // 1 / R_TC per dtype
    R s2sm, inv_s2sm;
    R ltma, inv_btma;
    R lmbar, lcommit;      // L / f
    R inv_link, inv_eta;   // 1 / BW_link, 1 / eta_DE
    R inv_rdec, lsetup;
    R eps;
    R inv_gmem, lstore;
    R ltmgmt, omisc, tlaunch, inv_dsm;
    R inv_f;
};

struct BwSet {
    BwStruct st;
    BwConst<float> cf;
    BwConst<double> cd;
};

template <typename R>
WM_HD void make_bw_const(const double* th, const BwStruct& s, BwConst<R>& c)
{
    const double f = s.f_clk;
    c.inv_tr = (R)(1.0 / th[0]);
    c.inv_tw = (R)(1.0 / th[1]);
    c.lmma = (R)(th[2] / f);
    for (int t = 0; t < 5; ++t) c.inv_rtc[t] = (R)(1.0 / th[3 + t]);
    c.s2sm = (R)th[8];
    c.inv_s2sm = (R)(1.0 / th[8]);
    c.ltma = (R)(th[9] / f);
    c.inv_btma = (R)(1.0 / th[10]);
    c.lmbar = (R)(th[11] / f);
    c.lcommit = (R)(th[12] / f);
    c.inv_link = (R)(1.0 / th[13]);
    c.inv_eta = (R)(1.0 / th[14]);
    c.inv_rdec = (R)(1.0 / th[15]);
    c.lsetup = (R)(th[16] / f);
    c.eps = (R)th[17];
    c.inv_gmem = (R)(1.0 / th[18]);
    c.lstore = (R)(th[19] / f);
    c.ltmgmt = (R)(th[20] / f);
    c.omisc = (R)th[21];
    c.tlaunch = (R)th[22];
    c.inv_dsm = (R)(1.0 / th[23]);
    c.inv_f = (R)(1.0 / f);
}

struct BwDesc {
    int32_t bM, bN, bK, G, fl;
    float Kt, CR, ob;
};

template <typename R>
struct BwEval {
    R T;
    int32_t cta;           // -1 invalid, 0 does not fit in TMEM, else CTAs per SM
    int32_t dt, pair, comp, nbar, nr;
    bool compute_bound;
    bool near_kink;        // |T_compute - T_io| within 1e-5 relative
    R Kt, MA, MB, Dread, Dacc, Tmma, ta_tb, Tde, Dab, io_raw, ob_bytes;
};

__device__ inline bool bw_desc_valid(const BwDesc& d)
{
    const float inf = __builtin_huge_valf();
    return (d.bM >= 1) & (d.bN >= 1) & (d.bK >= 1) & (d.G >= 1) & (d.fl >= 0) &
           ((d.fl >> 17) == 0) & ((d.fl & 7) <= 4) & (d.Kt >= 1.0f) & (d.Kt < inf) &
           (d.CR >= 1.0f) & (d.CR < inf) & (d.ob > 0.0f) & (d.ob < inf);
}

// a / b: the hardware reciprocal (1 ulp) in the float sweeps, IEEE
// division in the float64 re-evaluations
__device__ inline float bw_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double bw_div(double a, double b) { return a / b; }

// min(floor(a / b), cap) for 1 <= b <= a < 2^30 and cap <= 64.  The float
// estimate a * rcp(b) (a and b rounded to 24 bits, rcp 1 ulp, one product
// rounding: relative error below 2^-21) is within one of floor(a / b)
// whenever that quotient is below 2^20, and at or above cap + 1 whenever the
// quotient is larger than cap + 1; so after clamping the estimate to cap + 1
// one correction by the exact 64-bit remainder gives the quotient or a value
// above cap, which the final min clamps.
__device__ inline uint32_t udiv_capped(uint32_t a, uint32_t b, uint32_t cap)
{
    const float qf = (float)a * __builtin_amdgcn_rcpf((float)b);
    uint32_t q = qf >= (float)(cap + 1u) ? cap + 1u : (uint32_t)qf;
    const uint64_t prod = (uint64_t)q * b;
    q = prod > a ? q - 1u : (a - prod >= b ? q + 1u : q);
    return q < cap ? q : cap;
}

template <typename R, bool FULL>
__device__ inline void evaluate_bw(const BwStruct& st, const BwConst<R>& c, const BwDesc& d,
                                   BwEval<R>& E)
{
    E.T = (R)__builtin_nan("");
    E.cta = -1;
    E.near_kink = false;
    if (!bw_desc_valid(d)) return;
    const int32_t dt = d.fl & 7;
    const int32_t pair = (d.fl >> 3) & 1, stratB = (d.fl >> 4) & 1;
    const int32_t PA = ((d.fl >> 5) & 15) + 1, PB = ((d.fl >> 9) & 15) + 1;
    const int32_t nbar = (d.fl >> 13) & 7, comp = (d.fl >> 16) & 1;
    E.dt = dt;
    E.pair = pair;
    E.comp = comp;
    E.nbar = nbar;

    // residency: accumulator bytes (8 per element for FP64, else 4); TMEM is
    // below 2^30 bytes, so once the accumulator fits every quotient is a
    // 32-bit one (n_sm * cta <= 2^22, G < 2^31).  An extent above the TMEM
    // size cannot fit; otherwise both are below 2^30 and the product, at
    // most 2^63, is exact in 64 unsigned bits.
    const bool too_wide = (uint32_t)d.bM > (uint32_t)st.tmem_bytes || (uint32_t)d.bN > (uint32_t)st.tmem_bytes;
    const uint64_t acc = too_wide ? ~(uint64_t)0 : (uint64_t)d.bM * (uint64_t)d.bN * (dt == 0 ? 8u : 4u);
    const uint32_t cta = acc > (uint64_t)st.tmem_bytes
                             ? 0u
                             : udiv_capped((uint32_t)st.tmem_bytes, (uint32_t)acc, (uint32_t)st.max_cta);
    E.cta = (int32_t)cta;
    if (cta < 1) {
        E.T = (R)__builtin_huge_val();
        return;
    }
    // rounds: per_round = n_sm * cta <= 2^22; udiv21 where the numerator is
    // below 2^21, an exact division (behind a branch the wave skips unless a
    // lane needs it) for the larger grids
    const uint32_t per_round = (uint32_t)st.n_sm * cta;
    const uint32_t num = (uint32_t)d.G + per_round - 1u;
    const bool big = num >= (1u << 21);
    uint32_t nr = udiv21(big ? 0u : num, big ? 1u : per_round);
    if (__builtin_expect(__ballot(big) != 0, 0)) {
        if (big) nr = num / per_round;
    }
    E.nr = (int32_t)nr;

    // element bytes 8, 4, 2, 1, 1/2 for dtypes 0..4 (exact powers of two)
    const R e = (R)__builtin_ldexp(1.0, 3 - dt);
    const R Kt = (R)d.Kt;
    E.Kt = Kt;
    const R MA = (R)d.bM * (R)d.bK * e;
    const R MB = (R)d.bN * (R)d.bK * e;
    E.MA = MA;
    E.MB = MB;
    const R Dacc = (R)acc;
    E.Dacc = Dacc;

    // Eq. (2), Eq. (3)
    const R Dread = Dacc + (stratB ? MA : (R)0);
    E.Dread = Dread;
    const R Ttmem = Dread * c.inv_tr + c.lmma + Dacc * c.inv_tw;
    const R Tmgmt = bw_div(c.ltmgmt, Kt);
    const R fl = (R)2 * (R)d.bM * (R)d.bN * (R)d.bK;
    R inv_rtc = c.inv_rtc[0];
    inv_rtc = dt == 1 ? c.inv_rtc[1] : inv_rtc;
    inv_rtc = dt == 2 ? c.inv_rtc[2] : inv_rtc;
    inv_rtc = dt == 3 ? c.inv_rtc[3] : inv_rtc;
    inv_rtc = dt == 4 ? c.inv_rtc[4] : inv_rtc;
    const R Tmma = fl * inv_rtc * (pair ? c.inv_s2sm : (R)1);
    E.Tmma = Tmma;
    const R Tcomp = Tmma + Ttmem + Tmgmt;

    // Eq. (4), Eq. (6)
    const R ta_tb = bw_div(MA, (R)PA) + bw_div(pair ? (R)0.5 * MB : MB, (R)PB);
    E.ta_tb = ta_tb;
    const R Ttma = c.ltma + ta_tb * c.inv_btma;
    const R Tdsm = pair ? (R)0.5 * MB * c.inv_dsm : (R)0;

    // Eq. (5)
    const R Dab = MA + MB;
    E.Dab = Dab;
    const R Tde = comp ? bw_div(Dab, (R)d.CR) * c.inv_link * c.inv_eta : (R)0;
    E.Tde = Tde;
    const R Tup = dt == 4 ? Dab * c.inv_rdec + c.lsetup : (R)0;

    // sync, Eq. (7), Eq. (8)
    const R Tsync = (R)nbar * c.lmbar + (pair ? c.lcommit : (R)0);
    const R io_raw = Ttma + Tde + Tup + Tdsm;
    E.io_raw = io_raw;
    const R Tio = c.eps * io_raw + Tsync;
    E.compute_bound = Tcomp >= Tio;
    const R Tm = E.compute_bound ? Tcomp : Tio;
    const R Tstep = Tm + Tsync + c.omisc;
    E.ob_bytes = (R)d.bM * (R)d.bN * (R)d.ob;
    const R Tstore = E.ob_bytes * c.inv_gmem + c.lstore;
    E.T = c.tlaunch + (R)nr * (Kt * Tstep + Tstore);
    if (FULL) {
        const R hi = Tcomp > Tio ? Tcomp : Tio;
        const R gap = Tcomp > Tio ? Tcomp - Tio : Tio - Tcomp;
        E.near_kink = gap <= (R)1e-5 * hi;
    }
}

// w * dT/dtheta added to acc[2 + j] (24 slots; inactive terms add exact zeros).
template <typename R, typename A>
__device__ inline void bw_accumulate(const BwConst<R>& c, const BwEval<R>& E, A w, A* acc)
{
    const A nr = (A)E.nr, Kt = (A)E.Kt;
    const A cs = w * nr * Kt;
    const A inv_f = (A)c.inv_f;
    A* g = acc + 2;
    g[22] += w;                                             // T_launch
    g[21] += cs;                                            // O_misc
    g[18] += -w * nr * (A)E.ob_bytes * (A)c.inv_gmem * (A)c.inv_gmem;
    g[19] += w * nr * inv_f;                                // L_store
    const A ws = cs * (E.compute_bound ? (A)1 : (A)2);
    g[11] += ws * (A)E.nbar * inv_f;                        // L_mbar
    g[12] += E.pair ? ws * inv_f : (A)0;                    // L_commit
    const A wc = E.compute_bound ? cs : (A)0;
    const A wi = E.compute_bound ? (A)0 : cs;
    g[0] += -wc * (A)E.Dread * (A)c.inv_tr * (A)c.inv_tr;
    g[1] += -wc * (A)E.Dacc * (A)c.inv_tw * (A)c.inv_tw;
    g[2] += wc * inv_f;
    // once per round, not per K step: wc inv_f / Kt with the K steps cancelled
    g[20] += E.compute_bound ? w * nr * inv_f : (A)0;
    // d/dR_TC[dt] of Tmma = -Tmma / R_TC[dt]
    const A dR = -wc * (A)E.Tmma * (A)c.inv_rtc[E.dt];
    g[3] += E.dt == 0 ? dR : (A)0;
    g[4] += E.dt == 1 ? dR : (A)0;
    g[5] += E.dt == 2 ? dR : (A)0;
    g[6] += E.dt == 3 ? dR : (A)0;
    g[7] += E.dt == 4 ? dR : (A)0;
    g[8] += E.pair ? -wc * (A)E.Tmma * (A)c.inv_s2sm : (A)0;
    const A we = wi * (A)c.eps;
    g[17] += wi * (A)E.io_raw;                              // eps
    g[9] += we * inv_f;                                     // L_TMA
    g[10] += -we * (A)E.ta_tb * (A)c.inv_btma * (A)c.inv_btma;
    g[23] += E.pair ? -we * (A)0.5 * (A)E.MB * (A)c.inv_dsm * (A)c.inv_dsm : (A)0;
    g[13] += E.comp ? -we * (A)E.Tde * (A)c.inv_link : (A)0;
    g[14] += E.comp ? -we * (A)E.Tde * (A)c.inv_eta : (A)0;
    g[15] += E.dt == 4 ? -we * (A)E.Dab * (A)c.inv_rdec * (A)c.inv_rdec : (A)0;
    g[16] += E.dt == 4 ? we * inv_f : (A)0;
}

}  // namespace wm
