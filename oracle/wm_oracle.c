/*
 * wm_oracle.c -- plain FP64 CPU reference for the CDNA wavefront-centric
 * execution-time model (Section IV-B of the paper, "AMD MI300A Model").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no header, helper or
 * table with the HIP implementation.
 *
 * Style: scalar double arithmetic, one descriptor at a time, in the order the
 * paper states the terms.  Built with -O2 -ffp-contract=off (no FMA
 * contraction, no fast-math).  OpenMP only splits the loop over descriptors;
 * every reduction is done in a fixed order so results do not depend on the
 * thread count.
 *
 * Readings adopted where the paper is silent or ambiguous (each is also
 * exercised by a test):
 *   - occupancy generalises the VGPR-limited wave count of Section IV-B to
 *     VGPR, wave-slot and LDS limits with allocation granules;
 *   - "1 - h_total" in Eq. (10) is the product of the per-level miss rates;
 *   - memory has two stages: bandwidth time bytes/S with S the hit-weighted
 *     bandwidth (the BW_effective sentence after Eq. (10), generalised to all
 *     levels), and latency time from Eq. (10) with N_loads = bytes per wave /
 *     bytes in flight per wave, serialised over workgroup rounds as in the
 *     N_ctas / (N_CU W_eff) term of Eq. (14) with W_eff = integer occupancy;
 *   - HK_MAX combines the stages with the max of Eq. (1) / Eq. (14);
 *     PAPER_ETA is Eq. (9) and Eq. (12) taken literally;
 *   - the overhead of Eq. (1) collects T_launch and the additive terms of
 *     Eq. (13), Eq. (14), the interference / multi-GPU / fusion sentences of
 *     Section IV-B and the per-sync term of Section IV-E;
 *   - the Infinity-Cache hit rate h_LLC(W) (Table "hlcc-piecewise") replaces
 *     the descriptor's LLC hit rate when a working set W > 0 is given, and the
 *     HBM bandwidth is blended by Eq. (16).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define N_THETA 24

/* parameter-vector slots */
enum {
    S_BW_L1 = 0, S_BW_L2 = 1, S_BW_LLC = 2, S_BW_HBM = 3,
    S_LAT_L1 = 4, S_LAT_L2 = 5, S_LAT_LLC = 6, S_LAT_HBM = 7,
    S_P0 = 8, /* 8..12: fp64, fp32, bf16/fp16, fp8, int8 */
    S_T_LAUNCH = 13, S_TAU_WG = 14, S_TAU_BAR = 15, S_TAU_INTERF = 16,
    S_TAU_GPU = 17, S_TAU_FUSION = 18, S_TAU_SYNC = 19,
    S_ALPHA = 20, S_BETA = 21, S_W0 = 22, S_BPEAK = 23
};

typedef struct {
    int32_t n_levels, n_cu, n_simd, wave, vgpr_simd, vgpr_gran, waves_simd,
            lds_cu, lds_gran, bytes_inflight_wave, mwp, cwp, combine, pad_;
    double f_clk, w_lo_mib, c_llc_mib;
    double theta[N_THETA];
} orc_params_t;

typedef struct {
    const float *F, *B, *r1, *r2, *r3, *K, *u, *W;
    const int32_t *vgpr, *lds, *gpack, *grid;
    int64_t n;
} orc_desc_t;

/* everything one evaluation computes, exposed for the pins */
typedef struct {
    int32_t valid, stage, eta_saturated, pad_;
    int64_t k, o, n_wf, n_r, n_eff;
    double h[3], s[4], S, Lam, bw_hbm_eff, blend_e;
    double T_c, T_b, T_lat, T_m, eta, T_ov, T;
} orc_trace_t;

/* ------------------------------------------------------------------ */
/* integer helpers                                                      */
/* ------------------------------------------------------------------ */
static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }

/*
 * Occupancy: resident workgroups per CU.  Section IV-B limits active
 * wavefronts by VGPRs (min(32, floor(65536 / VGPR_per_wf)) on MI300A, i.e.
 * 4 SIMDs x 256 VGPRs x 64 lanes); Table "arch-params" gives 32 wavefronts
 * per CU and 64 KB LDS per CU.  Generalised: a wave needs ceil(v/gran)*gran
 * VGPRs of its SIMD and one of its wave slots; a workgroup of g threads has
 * k = ceil(g / wave) waves and needs ceil(s/lds_gran)*lds_gran bytes of LDS.
 */
int64_t orc_occupancy(const orc_params_t *p, int64_t v, int64_t s, int64_t g, int64_t *k_out)
{
    int64_t k = ceil_div(g, p->wave);
    int64_t v_alloc = ceil_div(v, p->vgpr_gran) * p->vgpr_gran;
    int64_t waves_per_simd = 0;
    if (v_alloc <= p->vgpr_simd)
        waves_per_simd = imin(p->vgpr_simd / v_alloc, p->waves_simd);
    int64_t o_waves = (p->n_simd * waves_per_simd) / k;
    int64_t o = o_waves;
    if (s > 0) {
        int64_t s_alloc = ceil_div(s, p->lds_gran) * p->lds_gran;
        int64_t o_lds = p->lds_cu / s_alloc;
        o = imin(o, o_lds);
    }
    if (k_out) *k_out = k;
    return o;
}

/* Table "hlcc-piecewise": Infinity-Cache hit rate vs working set (MiB). */
double orc_h_llc(const orc_params_t *p, double W_bytes)
{
    double Wm = W_bytes / 1048576.0;
    double lo = p->w_lo_mib, C = p->c_llc_mib;
    if (Wm < lo) return 1.0;                                   /* resident   */
    if (Wm <= C) return pow(1.0 - (Wm - lo) / (C - lo), p->theta[S_ALPHA]); /* transition */
    return pow(C / Wm, p->theta[S_BETA]);                      /* streaming  */
}

/* Eq. (16): B_eff(W) = B_sus + (B_peak - B_sus) exp(-W / w0), off if w0 <= 0 */
double orc_bw_hbm_eff(const orc_params_t *p, double W_bytes)
{
    double bsus = p->theta[S_BW_HBM];
    double w0 = p->theta[S_W0];
    if (!(W_bytes > 0.0) || !(w0 > 0.0)) return bsus;
    return bsus + (p->theta[S_BPEAK] - bsus) * exp(-W_bytes / w0);
}

static int desc_valid(double F, double B, double r1, double r2, double r3, double K,
                      double u, double W, int64_t v, int64_t s, int64_t gpack, int64_t G)
{
    if (!(isfinite(F) && F >= 0.0)) return 0;
    if (!(isfinite(B) && B >= 0.0)) return 0;
    if (!(isfinite(K) && K >= 0.0)) return 0;
    if (!(isfinite(W) && W >= 0.0)) return 0;
    if (!(u > 0.0 && u <= 1.0)) return 0;
    if (!(r1 >= 0.0 && r1 <= 1.0)) return 0;
    if (!(r2 >= 0.0 && r2 <= 1.0)) return 0;
    if (!(r3 >= 0.0 && r3 <= 1.0)) return 0;
    if (v < 1 || s < 0 || G < 1) return 0;
    if (gpack < 0 || gpack >= ((int64_t)1 << 25)) return 0;
    int64_t g = gpack & 2047;
    int64_t dtype = (gpack >> 11) & 7;
    if (g < 1 || g > 1024 || dtype > 4) return 0;
    return 1;
}

/*
 * One descriptor.  Writes the trace and, if dT != NULL, the analytic
 * derivative dT/dtheta (24 entries, subgradient at the max/min switches:
 * first maximal stage; the saturated overlap branch when a*T_c >= T_m;
 * ties between bandwidth and latency go to bandwidth).
 */
void orc_eval(const orc_params_t *p, double F, double B, double r1, double r2, double r3,
              double K, double u, double W, int64_t v, int64_t s, int64_t gpack, int64_t G,
              orc_trace_t *tr, double *dT)
{
    const double *th = p->theta;
    memset(tr, 0, sizeof(*tr));
    if (dT) memset(dT, 0, sizeof(double) * N_THETA);

    if (!desc_valid(F, B, r1, r2, r3, K, u, W, v, s, gpack, G)) {
        tr->valid = 0;
        tr->T = NAN;
        tr->o = -1;
        return;
    }
    tr->valid = 1;
    int64_t g = gpack & 2047;
    int64_t dtype = (gpack >> 11) & 7;
    int64_t n_conc = ((gpack >> 14) & 7) + 1;
    int64_t n_dev = ((gpack >> 17) & 7) + 1;
    int64_t fused = (gpack >> 20) & 1;
    int64_t n_sync = (gpack >> 21) & 15;

    /* occupancy (Section IV-B, generalised) */
    int64_t k;
    int64_t o = orc_occupancy(p, v, s, g, &k);
    tr->k = k;
    tr->o = o;
    tr->n_wf = o * k;
    if (o == 0) {
        tr->T = INFINITY;
        return;
    }

    /* workgroup rounds: N_ctas / (N_CU W_eff) of Eq. (14), in whole rounds */
    int64_t n_r = ceil_div(G, (int64_t)p->n_cu * o);
    tr->n_r = n_r;

    /* hit rates per cache level; the LLC rate comes from h_LLC(W) if W > 0 */
    int L = p->n_levels;
    double h1 = r1, h2 = r2, h3 = r3;
    int wmode_llc = (L == 4 && W > 0.0);
    if (wmode_llc) h3 = orc_h_llc(p, W);
    tr->h[0] = h1;
    tr->h[1] = h2;
    tr->h[2] = (L == 4) ? h3 : 0.0;

    /* served fractions, Eq. (10): h_L1, (1-h_L1) h_L2, (1-h_L1)(1-h_L2) h_LLC,
       and the product of all miss rates for HBM */
    double s1, s2, s3 = 0.0, s_hbm;
    s1 = h1;
    s2 = (1.0 - h1) * h2;
    if (L == 4) {
        s3 = (1.0 - h1) * (1.0 - h2) * h3;
        s_hbm = (1.0 - h1) * (1.0 - h2) * (1.0 - h3);
    } else {
        s_hbm = (1.0 - h1) * (1.0 - h2);
    }
    tr->s[0] = s1;
    tr->s[1] = s2;
    tr->s[2] = s3;
    tr->s[3] = s_hbm;

    /* HBM bandwidth with the working-set blend of Eq. (16) */
    double e = 0.0;
    int wmode_bw = (W > 0.0 && th[S_W0] > 0.0);
    if (wmode_bw) e = exp(-W / th[S_W0]);
    double bw_hbm = orc_bw_hbm_eff(p, W);
    tr->blend_e = e;
    tr->bw_hbm_eff = bw_hbm;

    /* hit-weighted bandwidth (BW_effective of Section IV-B, all levels) and
       hit-weighted latency (bracket of Eq. (10)) */
    double S = s1 * th[S_BW_L1] + s2 * th[S_BW_L2] + s_hbm * bw_hbm;
    double Lam = s1 * th[S_LAT_L1] + s2 * th[S_LAT_L2] + s_hbm * th[S_LAT_HBM];
    if (L == 4) {
        S += s3 * th[S_BW_LLC];
        Lam += s3 * th[S_LAT_LLC];
    }
    tr->S = S;
    tr->Lam = Lam;

    /* stage times */
    double P = th[S_P0 + dtype];
    double T_c = F / (u * P);                              /* Eq. (11), Util = u */
    double T_b = B / S;                                    /* bytes / BW_effective */
    double n_loads = B / ((double)G * (double)k * (double)p->bytes_inflight_wave);
    double T_lat = (double)n_r * n_loads * Lam / p->f_clk; /* Eq. (10) x rounds */
    tr->T_c = T_c;
    tr->T_b = T_b;
    tr->T_lat = T_lat;

    /* overhead: launch, per-WG dispatch, per-round-step barrier, concurrency,
       devices, fusion, host syncs */
    double T_ov = th[S_T_LAUNCH]
                + th[S_TAU_WG] * (double)G
                + th[S_TAU_BAR] * (double)n_r * K
                + (double)(n_conc - 1) * th[S_TAU_INTERF]
                + (double)(n_dev - 1) * th[S_TAU_GPU]
                + (double)fused * th[S_TAU_FUSION]
                + (double)n_sync * th[S_TAU_SYNC];
    tr->T_ov = T_ov;

    /* weights of dT/dT_c, dT/dT_b, dT/dT_lat under the chosen combine */
    double wc = 0.0, wb = 0.0, wl = 0.0;
    if (p->combine == 0) {
        /* Eq. (1) / Eq. (14): max of the stages */
        double T_stage;
        if (T_c >= T_b && T_c >= T_lat) { T_stage = T_c; tr->stage = 0; wc = 1.0; }
        else if (T_b >= T_lat)          { T_stage = T_b; tr->stage = 1; wb = 1.0; }
        else                            { T_stage = T_lat; tr->stage = 2; wl = 1.0; }
        tr->T = T_ov + T_stage;
        tr->T_m = (T_b >= T_lat) ? T_b : T_lat;
    } else {
        /* Eq. (9) and Eq. (12) */
        int mem_is_b = (T_b >= T_lat);
        double T_m = mem_is_b ? T_b : T_lat;
        int64_t n_eff = o * k;
        if (p->mwp > 0) n_eff = imin(n_eff, p->mwp);
        if (p->cwp > 0) n_eff = imin(n_eff, p->cwp);
        double a = (double)(n_eff - 1);
        double eta, dTc, dTm;
        int sat;
        if (a == 0.0) {
            eta = 0.0; sat = 0;
            dTc = 1.0; dTm = 1.0;
        } else if (a * T_c >= T_m) {
            eta = 1.0; sat = 1;
            dTc = 0.5; dTm = 0.5;
        } else {
            eta = a * T_c / T_m; sat = 0;
            double den = (T_m + a * T_c) * (T_m + a * T_c);
            dTc = T_m * T_m * (1.0 - a) / den;
            dTm = (T_m * T_m + 2.0 * a * T_m * T_c + a * T_c * T_c) / den;
        }
        double num = T_m + T_c;
        double step = (num == 0.0) ? 0.0 : num / (1.0 + eta);
        tr->T = T_ov + step;
        tr->T_m = T_m;
        tr->eta = eta;
        tr->eta_saturated = sat;
        tr->n_eff = n_eff;
        tr->stage = mem_is_b ? 1 : 2;
        wc = dTc;
        if (mem_is_b) wb = dTm; else wl = dTm;
    }

    if (!dT) return;

    /* ---- analytic partial derivatives ---- */
    /* overhead */
    dT[S_T_LAUNCH] = 1.0;
    dT[S_TAU_WG] = (double)G;
    dT[S_TAU_BAR] = (double)n_r * K;
    dT[S_TAU_INTERF] = (double)(n_conc - 1);
    dT[S_TAU_GPU] = (double)(n_dev - 1);
    dT[S_TAU_FUSION] = (double)fused;
    dT[S_TAU_SYNC] = (double)n_sync;

    /* compute stage: d(F/(uP))/dP = -T_c / P */
    dT[S_P0 + dtype] += wc * (-T_c / P);

    /* bandwidth stage: dT_b/dX = -(B / S^2) dS/dX */
    if (wb != 0.0 && B > 0.0) {
        double c = -wb * T_b / S;
        dT[S_BW_L1] += c * s1;
        dT[S_BW_L2] += c * s2;
        if (L == 4) dT[S_BW_LLC] += c * s3;
        if (wmode_bw) {
            double w0 = th[S_W0];
            dT[S_BW_HBM] += c * s_hbm * (1.0 - e);
            dT[S_BPEAK] += c * s_hbm * e;
            dT[S_W0] += c * s_hbm * (th[S_BPEAK] - th[S_BW_HBM]) * e * W / (w0 * w0);
        } else {
            dT[S_BW_HBM] += c * s_hbm;
        }
    }
    /* latency stage: T_lat = q * Lam with q = n_r * n_loads / f_clk */
    double q = (double)n_r * n_loads / p->f_clk;
    if (wl != 0.0 && B > 0.0) {
        double c = wl * q;
        dT[S_LAT_L1] += c * s1;
        dT[S_LAT_L2] += c * s2;
        if (L == 4) dT[S_LAT_LLC] += c * s3;
        dT[S_LAT_HBM] += c * s_hbm;
    }
    /* h_LLC(W) exponents, through s3 and s_hbm */
    if (wmode_llc && B > 0.0 && (wb != 0.0 || wl != 0.0)) {
        double a3 = (1.0 - h1) * (1.0 - h2);
        double dS_dh = a3 * (th[S_BW_LLC] - bw_hbm);
        double dL_dh = a3 * (th[S_LAT_LLC] - th[S_LAT_HBM]);
        double dT_dh = wb * (-T_b / S) * dS_dh + wl * q * dL_dh;
        double Wm = W / 1048576.0;
        double lo = p->w_lo_mib, C = p->c_llc_mib;
        if (Wm >= lo && Wm <= C) {
            double base = 1.0 - (Wm - lo) / (C - lo);
            if (base > 0.0) dT[S_ALPHA] += dT_dh * h3 * log(base);
        } else if (Wm > C) {
            dT[S_BETA] += dT_dh * h3 * log(C / Wm);
        }
    }
}

/* ------------------------------------------------------------------ */
/* batched entry points                                                  */
/* ------------------------------------------------------------------ */
#define DESC_ARGS(d, i) (double)(d)->F[i], (double)(d)->B[i], (double)(d)->r1[i], \
    (double)(d)->r2[i], (double)(d)->r3[i], (double)(d)->K[i], (double)(d)->u[i], \
    (double)(d)->W[i], (int64_t)(d)->vgpr[i], (int64_t)(d)->lds[i], \
    (int64_t)(d)->gpack[i], (int64_t)(d)->grid[i]

void orc_predict(const orc_params_t *p, const orc_desc_t *d, double *T, int32_t *occ)
{
    int64_t n = d->n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        orc_trace_t tr;
        orc_eval(p, DESC_ARGS(d, i), &tr, NULL);
        T[i] = tr.T;
        if (occ) occ[i] = (int32_t)tr.o;
    }
}

void orc_trace(const orc_params_t *p, const orc_desc_t *d, orc_trace_t *out)
{
    int64_t n = d->n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) orc_eval(p, DESC_ARGS(d, i), &out[i], NULL);
}

/* per-descriptor Jacobian dT_i/dtheta_j, row-major [n][24] */
void orc_jacobian(const orc_params_t *p, const orc_desc_t *d, double *J)
{
    int64_t n = d->n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        orc_trace_t tr;
        orc_eval(p, DESC_ARGS(d, i), &tr, J + i * N_THETA);
    }
}

/* Naive roofline, max(FLOPs / P_peak, bytes / B_HBM) (Section V-A) */
void orc_roofline(const orc_params_t *p, const orc_desc_t *d, double *T)
{
    int64_t n = d->n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t gp = d->gpack[i];
        int64_t dtype = (gp >> 11) & 7;
        double F = d->F[i], B = d->B[i];
        if (!desc_valid(DESC_ARGS(d, i)) ) { T[i] = NAN; continue; }
        double tc = F / p->theta[S_P0 + dtype];
        double tb = B / p->theta[S_BW_HBM];
        T[i] = tc > tb ? tc : tb;
    }
}

/*
 * Weighted sum of per-descriptor Jacobian rows with a fixed reduction order:
 * rows are grouped into ORC_CHUNK-sized chunks summed serially, then the
 * chunk sums are added serially.
 * mode 0 (vector-Jacobian product): weight_i = dL/dT_i.
 * mode 1 (mean relative error): weight_i = sign(T_i - m_i) / m_i over the
 *        descriptors with finite T, finite m > 0; also sums |T-m|/m and the
 *        count; the final result is divided by the count.
 * out: [0] loss (mode 1), [1] count, [2..25] gradient.
 */
#define ORC_CHUNK 4096
void orc_weighted_grad(const orc_params_t *p, const orc_desc_t *d, const float *w_in,
                       int mode, double *out)
{
    int64_t n = d->n;
    int64_t nch = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    double *part = (double *)calloc((size_t)(nch > 0 ? nch : 1) * 26, sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; ++c) {
        double acc[26];
        memset(acc, 0, sizeof(acc));
        int64_t a = c * ORC_CHUNK, b = a + ORC_CHUNK < n ? a + ORC_CHUNK : n;
        for (int64_t i = a; i < b; ++i) {
            orc_trace_t tr;
            double J[N_THETA];
            orc_eval(p, DESC_ARGS(d, i), &tr, J);
            double wgt;
            if (mode == 0) {
                if (!isfinite(tr.T)) continue;
                wgt = (double)w_in[i];
            } else {
                double m = (double)w_in[i];
                if (!isfinite(tr.T) || !isfinite(m) || !(m > 0.0)) continue;
                double r = (tr.T - m) / m;
                acc[0] += fabs(r);
                acc[1] += 1.0;
                wgt = (tr.T > m) ? 1.0 / m : (tr.T < m ? -1.0 / m : 0.0);
            }
            for (int j = 0; j < N_THETA; ++j) acc[2 + j] += wgt * J[j];
        }
        memcpy(part + c * 26, acc, sizeof(acc));
    }
    memset(out, 0, 26 * sizeof(double));
    for (int64_t c = 0; c < nch; ++c)
        for (int j = 0; j < 26; ++j) out[j] += part[c * 26 + j];
    free(part);
    if (mode == 1 && out[1] > 0.0) {
        out[0] /= out[1];
        for (int j = 0; j < N_THETA; ++j) out[2 + j] /= out[1];
    }
}

/* ------------------------------------------------------------------ */
/* calibration: Adam on log(theta) over the free slots                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t steps, order;   /* order: bit 0 slots 0-3 non-increasing, bit 1 slots 4-7 non-decreasing */
    double lr, lr_final, beta1, beta2, eps;
    uint32_t free_mask, pad2_;
    double lo[N_THETA], hi[N_THETA];   /* box of fitted slot j; 0 = none */
} orc_calib_opts_t;

/*
 * Least-squares projection of y[0..n) onto non-decreasing sequences by pool
 * adjacent violators: values enter left to right as blocks; while a block's
 * mean is below the mean of the block before it, the two merge.  Every
 * element takes its block's mean.  (The calibration constraints, not a
 * passage of the paper: they keep fitted cache levels in their physical
 * order.)
 */
void orc_isotonic_inc(double *y, int n)
{
    double mean[N_THETA];
    int cnt[N_THETA], nb = 0;
    for (int i = 0; i < n; ++i) {
        mean[nb] = y[i];
        cnt[nb] = 1;
        ++nb;
        while (nb > 1 && mean[nb - 2] > mean[nb - 1]) {
            const int c = cnt[nb - 2] + cnt[nb - 1];
            mean[nb - 2] = (mean[nb - 2] * cnt[nb - 2] + mean[nb - 1] * cnt[nb - 1]) / c;
            cnt[nb - 2] = c;
            --nb;
        }
    }
    for (int b = 0, k = 0; b < nb; ++b)
        for (int c = 0; c < cnt[b]; ++c) y[k++] = mean[b];
}

/* The constraints of a calibration applied to log(theta) after an update:
 * the orderings (a non-increasing fit is the non-decreasing fit of the
 * negated values), then the boxes. */
static void orc_project(const orc_calib_opts_t *o, double *phi)
{
    if (o->order & 1) {
        double y[4];
        for (int k = 0; k < 4; ++k) y[k] = -phi[k];
        orc_isotonic_inc(y, 4);
        for (int k = 0; k < 4; ++k) phi[k] = -y[k];
    }
    if (o->order & 2) orc_isotonic_inc(phi + 4, 4);
    for (int j = 0; j < N_THETA; ++j) {
        if (!(o->free_mask >> j & 1u)) continue;
        if (o->lo[j] > 0.0 && phi[j] < log(o->lo[j])) phi[j] = log(o->lo[j]);
        if (o->hi[j] > 0.0 && phi[j] > log(o->hi[j])) phi[j] = log(o->hi[j]);
    }
}

/*
 * Returns 0 on success (p_out = theta after the last update) or 1 when the
 * loss or a gradient became non-finite, or an update left the positive
 * finite range; p_out is then the last theta whose loss was finite and the
 * remaining loss-history entries are NaN.
 */
int orc_calibrate(const orc_params_t *p0, const orc_desc_t *d, const float *m,
                  const orc_calib_opts_t *o, orc_params_t *p_out, double *loss_hist)
{
    orc_params_t p = *p0, last_ok = *p0;
    double phi[N_THETA], mom[N_THETA], vel[N_THETA], out[26];
    for (int j = 0; j < N_THETA; ++j) {
        phi[j] = (o->free_mask >> j & 1u) ? log(p.theta[j]) : 0.0;
        mom[j] = 0.0;
        vel[j] = 0.0;
    }
    for (int t = 1; t <= o->steps; ++t) {
        orc_weighted_grad(&p, d, m, 1, out);
        if (loss_hist) loss_hist[t - 1] = out[0];
        int finite = isfinite(out[0]);
        for (int j = 0; j < N_THETA; ++j) finite = finite && isfinite(out[2 + j]);
        int ok = finite;
        orc_params_t next = p;
        if (finite) {
            last_ok = p;
            double lr = o->lr;
            if (o->lr_final > 0.0 && o->steps > 1)
                lr = o->lr * pow(o->lr_final / o->lr, (double)(t - 1) / (double)(o->steps - 1));
            double b1t = pow(o->beta1, (double)t), b2t = pow(o->beta2, (double)t);
            for (int j = 0; j < N_THETA; ++j) {
                if (!(o->free_mask >> j & 1u)) continue;
                double gphi = p.theta[j] * out[2 + j];          /* d/dlog(theta) */
                mom[j] = o->beta1 * mom[j] + (1.0 - o->beta1) * gphi;
                vel[j] = o->beta2 * vel[j] + (1.0 - o->beta2) * gphi * gphi;
                double mh = mom[j] / (1.0 - b1t);
                double vh = vel[j] / (1.0 - b2t);
                phi[j] -= lr * mh / (sqrt(vh) + o->eps);
            }
            orc_project(o, phi);
            for (int j = 0; j < N_THETA; ++j) {
                if (!(o->free_mask >> j & 1u)) continue;
                next.theta[j] = exp(phi[j]);
                ok = ok && isfinite(next.theta[j]) && next.theta[j] > 0.0;
            }
        }
        if (!ok) {
            if (loss_hist)
                for (int k = t; k < o->steps; ++k) loss_hist[k] = NAN;
            *p_out = last_ok;
            return 1;
        }
        p = next;
    }
    *p_out = p;
    return 0;
}

/* ------------------------------------------------------------------ */
/* occupancy-driven tile selection (Section IV-B, adaptive tile         */
/* selection: evaluate every candidate tile, return the fastest)        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t valid, pad_;
    int64_t G, Ks, g, v, s;
    double F, B, U, r2;
} orc_tile_t;

/*
 * GEMM tile -> descriptor.  Candidate code: mt | nt << 2 | kd << 4 | (waves-1) << 6
 * with mt, nt in {32, 64, 128, 256} and kd in {16, 32, 64}.  A tile of
 * mt x nt outputs with K-depth kd runs as one workgroup of 64 * waves
 * threads; the grid covers the padded output, the K loop has ceil(K/kd)
 * steps, each loading an (mt + nt) x kd panel; accumulators live in VGPRs
 * (two per FP64 value), input panels are double-buffered in LDS.  A grid
 * of more than 2^31 - 1 workgroups, or a workgroup of more than 1024
 * threads, makes the tile infeasible.
 */
void orc_tile_derive(int64_t M, int64_t N, int64_t Kd, int64_t t, uint32_t code,
                     int64_t wave, orc_tile_t *out)
{
    static const int64_t MN[4] = {32, 64, 128, 256};
    static const int64_t KDV[3] = {16, 32, 64};
    static const int64_t ESZ[4] = {8, 4, 2, 1};
    static const int64_t EOUT[4] = {8, 4, 2, 2};
    memset(out, 0, sizeof(*out));
    int64_t kdc = (code >> 4) & 3;
    if ((code >> 9) != 0 || kdc == 3 || M < 1 || N < 1 || Kd < 1 || t < 0 || t > 3) {
        out->valid = 0;
        return;
    }
    int64_t mt = MN[code & 3], nt = MN[(code >> 2) & 3], kd = KDV[kdc];
    int64_t wpw = ((code >> 6) & 7) + 1;
    int64_t e = ESZ[t], eo = EOUT[t], acc = (t == 0) ? 2 : 1;
    int64_t gm = ceil_div(M, mt), gn = ceil_div(N, nt);
    int64_t G = gm * gn, Ks = ceil_div(Kd, kd), g = wave * wpw;
    /* a descriptor counts workgroups in 32 bits and a workgroup holds at
       most 1024 threads: larger grids or groups are not launchable */
    if (G > 0x7fffffffll || g > 1024) {
        out->valid = 0;
        return;
    }
    out->valid = 1;
    out->G = G;
    out->Ks = Ks;
    out->g = g;
    out->F = 2.0 * (double)(gm * mt) * (double)(gn * nt) * (double)(Ks * kd);
    /* bytes are real counts: products formed in double, so that no shape
       within the int32 limits overflows (exact below 2^53) */
    out->B = (double)G * (double)Ks * (double)(mt + nt) * (double)kd * (double)e +
             (double)M * (double)N * (double)eo;
    out->U = ((double)M * (double)Kd + (double)Kd * (double)N) * (double)e +
             (double)M * (double)N * (double)eo;
    double r2 = 1.0 - out->U / out->B;
    out->r2 = r2 > 0.0 ? r2 : 0.0;
    out->v = ceil_div(mt * nt * acc, g) + ceil_div((mt + nt) * kd * e, 4 * g) + 16;
    out->s = 2 * (mt + nt) * kd * e;
}

double orc_tile_cost(const orc_params_t *p, int64_t M, int64_t N, int64_t Kd, int64_t t,
                     uint32_t code)
{
    orc_tile_t td;
    orc_tile_derive(M, N, Kd, t, code, p->wave, &td);
    if (!td.valid) return NAN;
    orc_trace_t tr;
    int64_t gpack = td.g | (t << 11);
    orc_eval(p, td.F, td.B, 0.0, td.r2, 0.0, (double)td.Ks, 1.0, 0.0, td.v, td.s, gpack,
             td.G, &tr, NULL);
    return tr.T;
}

/* all candidate costs, flat over the CSR list */
void orc_tile_costs(const orc_params_t *p, int64_t n, const int32_t *M, const int32_t *N,
                    const int32_t *K, const int32_t *dt, const int32_t *off,
                    const uint32_t *code, double *cost)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = off[i]; j < off[i + 1]; ++j)
            cost[j] = orc_tile_cost(p, M[i], N[i], K[i], dt[i], code[j]);
}

/*
 * Argmin over each shape's candidate list: lowest finite cost, exact ties to
 * the lowest local index, -1 when nothing is feasible.  near_tie = 1 when the
 * runner-up is within 1e-6 relative of the winner.
 */
void orc_select_tile(const orc_params_t *p, int64_t n, const int32_t *M, const int32_t *N,
                     const int32_t *K, const int32_t *dt, const int32_t *off,
                     const uint32_t *code, int32_t *best, double *best_cost, uint8_t *near_tie)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int32_t bi = -1;
        double c1 = INFINITY, c2 = INFINITY;
        for (int64_t j = off[i]; j < off[i + 1]; ++j) {
            double c = orc_tile_cost(p, M[i], N[i], K[i], dt[i], code[j]);
            if (!isfinite(c)) continue;
            if (c < c1) { c2 = c1; c1 = c; bi = (int32_t)(j - off[i]); }
            else if (c < c2) { c2 = c; }
        }
        best[i] = bi;
        best_cost[i] = c1;
        near_tie[i] = (bi >= 0 && isfinite(c2) && (c2 - c1) <= 1e-6 * c1) ? 1 : 0;
    }
}

/* ------------------------------------------------------------------ */
/* workload segments (Sections IV-E, IV-F and the multi-segment model   */
/* of Section V-B): an application is a list of segments, each a kernel */
/* executed n_exec times                                                */
/* ------------------------------------------------------------------ */
typedef struct {
    const int32_t *app_off;   /* [n_apps + 1] CSR offsets into the segment rows */
    const float *n_exec;      /* executions of the segment                      */
    const int32_t *n_kern;    /* kernels launched per execution (>= 1)          */
    const int32_t *cls;       /* class 0 memory, 1 compute, 2 balanced, 3 stencil */
    const float *h2d, *d2h;   /* host-to-device / device-to-host bytes per execution */
    int64_t n_apps;
} orc_segs_t;

typedef struct {
    double kappa[4];          /* per-class scale of the kernel time              */
    double bw_h2d, bw_d2h;    /* effective transfer bandwidth per direction, B/s */
    double tau_memcpy;        /* fixed cost per transfer episode, s (Eq. (15))   */
} orc_segp_t;

#define ORC_NSEG 7            /* kappa[4], bw_h2d, bw_d2h, tau_memcpy */

static int seg_valid(double ne, int64_t nk, int64_t c, double h, double d)
{
    return isfinite(ne) && ne >= 0.0 && nk >= 1 && c >= 0 && c <= 3 &&
           isfinite(h) && h >= 0.0 && isfinite(d) && d >= 0.0;
}

/*
 * One segment: T_seg = n_exec * (kappa_cls * T_kernel          (kernel model)
 *                                + (n_kern - 1) * T_launch     (extra launches, Section IV-F)
 *                                + [h2d > 0] (h2d / B_h2d + tau_memcpy)   (Eq. (15))
 *                                + [d2h > 0] (d2h / B_d2h + tau_memcpy)).
 * Writes dT/dtheta (24) and dT/dsegparam (7) when the pointers are set.
 */
double orc_segment(const orc_params_t *p, const orc_segp_t *q, const orc_desc_t *d, const orc_segs_t *s,
                   int64_t i, double *dth, double *dsp)
{
    orc_trace_t tr;
    double J[N_THETA];
    orc_eval(p, DESC_ARGS(d, i), &tr, dth ? J : NULL);
    double ne = s->n_exec[i], h = s->h2d[i], dd = s->d2h[i];
    int64_t nk = s->n_kern[i], c = s->cls[i];
    if (dth) memset(dth, 0, sizeof(double) * N_THETA);
    if (dsp) memset(dsp, 0, sizeof(double) * ORC_NSEG);
    if (!seg_valid(ne, nk, c, h, dd)) return NAN;
    if (!tr.valid) return NAN;
    if (!isfinite(tr.T)) return INFINITY;
    double T = q->kappa[c] * tr.T + (double)(nk - 1) * p->theta[S_T_LAUNCH];
    if (h > 0.0) T += h / q->bw_h2d + q->tau_memcpy;
    if (dd > 0.0) T += dd / q->bw_d2h + q->tau_memcpy;
    if (dth) {
        for (int j = 0; j < N_THETA; ++j) dth[j] = ne * q->kappa[c] * J[j];
        dth[S_T_LAUNCH] += ne * (double)(nk - 1);
    }
    if (dsp) {
        dsp[c] = ne * tr.T;
        if (h > 0.0) { dsp[4] = -ne * h / (q->bw_h2d * q->bw_h2d); dsp[6] += ne; }
        if (dd > 0.0) { dsp[5] = -ne * dd / (q->bw_d2h * q->bw_d2h); dsp[6] += ne; }
    }
    return ne * T;
}

/* Application totals T_app[a] = sum of its segments' times (NaN if any
 * segment is invalid, else +inf if any is infeasible). */
void orc_predict_apps(const orc_params_t *p, const orc_segp_t *q, const orc_desc_t *d,
                      const orc_segs_t *s, double *T_app, double *T_seg)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < s->n_apps; ++a) {
        double tot = 0.0;
        for (int64_t i = s->app_off[a]; i < s->app_off[a + 1]; ++i) {
            double t = orc_segment(p, q, d, s, i, NULL, NULL);
            if (T_seg) T_seg[i] = t;
            tot += t;
        }
        T_app[a] = tot;
    }
}

/*
 * Mean relative error over applications with finite total and finite
 * measured m > 0, and its gradient: out[0] loss, out[1] count,
 * out[2..25] dL/dtheta, out[26..32] dL/dsegparam.  Fixed-order sums.
 */
void orc_apps_loss_grad(const orc_params_t *p, const orc_segp_t *q, const orc_desc_t *d,
                        const orc_segs_t *s, const double *measured, double *out)
{
    const int NO = 2 + N_THETA + ORC_NSEG;
    int64_t na = s->n_apps;
    double *part = (double *)calloc((size_t)(na > 0 ? na : 1) * NO, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < na; ++a) {
        double *row = part + a * NO;
        double tot = 0.0;
        for (int64_t i = s->app_off[a]; i < s->app_off[a + 1]; ++i)
            tot += orc_segment(p, q, d, s, i, NULL, NULL);
        double m = measured[a];
        if (!isfinite(tot) || !isfinite(m) || !(m > 0.0)) continue;
        row[0] = fabs((tot - m) / m);
        row[1] = 1.0;
        double w = tot > m ? 1.0 / m : (tot < m ? -1.0 / m : 0.0);
        double dth[N_THETA], dsp[ORC_NSEG];
        for (int64_t i = s->app_off[a]; i < s->app_off[a + 1]; ++i) {
            orc_segment(p, q, d, s, i, dth, dsp);
            for (int j = 0; j < N_THETA; ++j) row[2 + j] += w * dth[j];
            for (int j = 0; j < ORC_NSEG; ++j) row[2 + N_THETA + j] += w * dsp[j];
        }
    }
    memset(out, 0, sizeof(double) * NO);
    for (int64_t a = 0; a < na; ++a)
        for (int j = 0; j < NO; ++j) out[j] += part[a * NO + j];
    free(part);
    if (out[1] > 0.0) {
        out[0] /= out[1];
        for (int j = 2; j < NO; ++j) out[j] /= out[1];
    }
}

/* ------------------------------------------------------------------ */
/* per-group calibration multipliers (Section IV-D optional per-case    */
/* multipliers with train/holdout separation; Section V-B m_case)       */
/* ------------------------------------------------------------------ */
typedef struct { double x, w; int64_t i; } orc_xw_t;

static int cmp_xw(const void *a, const void *b)
{
    const orc_xw_t *p = (const orc_xw_t *)a, *q = (const orc_xw_t *)b;
    if (p->x < q->x) return -1;
    if (p->x > q->x) return 1;
    return p->i < q->i ? -1 : (p->i > q->i ? 1 : 0);
}

static int mult_row_ok(double T, double m)
{
    return isfinite(T) && T > 0.0 && isfinite(m) && m > 0.0;
}

/*
 * Group g owns rows [off[g], off[g+1]).  Its multiplier minimises the
 * training mean relative error sum_i |mult * T_i - m_i| / m_i over its
 * valid training rows (T_i, m_i finite and > 0, train_i != 0): writing
 * x_i = m_i / T_i and w_i = T_i / m_i the objective is sum_i w_i |mult - x_i|,
 * minimised by a weighted median of the x_i -- the smallest x_k (ascending
 * x, then row index) whose cumulative weight reaches half the total.
 * Groups without a valid training row keep mult = 1.  T_scaled[i] =
 * mult[g] * T_i for every row; stats: training loss sum, training count,
 * held-out loss sum, held-out count over valid rows.
 */
void orc_fit_multipliers(const double *T, const double *m, const int32_t *off, int64_t n_groups,
                         const uint8_t *train, double *mult, double *T_scaled, double *stats)
{
    stats[0] = stats[1] = stats[2] = stats[3] = 0.0;
    for (int64_t g = 0; g < n_groups; ++g) {
        int64_t a = off[g], b = off[g + 1];
        orc_xw_t *buf = (orc_xw_t *)malloc(sizeof(orc_xw_t) * (size_t)(b > a ? b - a : 1));
        int64_t k = 0;
        double W = 0.0;
        for (int64_t i = a; i < b; ++i) {
            if (!train[i] || !mult_row_ok(T[i], m[i])) continue;
            buf[k].x = m[i] / T[i];
            buf[k].w = T[i] / m[i];
            buf[k].i = i;
            ++k;
        }
        double mu = 1.0;
        if (k > 0) {
            qsort(buf, (size_t)k, sizeof(orc_xw_t), cmp_xw);
            for (int64_t j = 0; j < k; ++j) W += buf[j].w;
            double c = 0.0;
            for (int64_t j = 0; j < k; ++j) {
                c += buf[j].w;
                if (c >= 0.5 * W) { mu = buf[j].x; break; }
            }
        }
        free(buf);
        mult[g] = mu;
        for (int64_t i = a; i < b; ++i) {
            T_scaled[i] = mu * T[i];
            if (!mult_row_ok(T[i], m[i])) continue;
            double e = fabs(mu * T[i] - m[i]) / m[i];
            if (train[i]) { stats[0] += e; stats[1] += 1.0; }
            else { stats[2] += e; stats[3] += 1.0; }
        }
    }
}

/* ------------------------------------------------------------------ */
/* kernel-fusion planning (Section IV-B: a fused kernel is modelled with */
/* the combined flops and bytes plus tau_fusion)                         */
/* ------------------------------------------------------------------ */
typedef struct {
    double F, B, r1, r2, r3, K, u, W;
    int64_t v, s, gpack, G;
} orc_fdesc_t;

/*
 * The descriptor of rows a .. a+len-1 of one chain run as one kernel
 * (len = 1: the row itself).  edge[k] = bytes row k hands to row k+1 (written
 * by k, read by k+1), which a fused kernel keeps on chip:
 *   F = sum F_k;  B = max(sum B_k - 2 sum edges, 0);
 *   r_l = sum r_l,k B_k / sum B_k (0 when sum B_k = 0);
 *   K = sum K_k;  W = max(sum W_k - sum edges, 0);
 *   dtype of the first row with the largest F_k;  u such that the fused
 *   compute time F / (u P_dtype) equals the sum of the rows' F_k / (u_k
 *   P_dtype_k), capped at 1 (1 when F = 0);
 *   VGPRs, LDS, workgroup size, grid, concurrent kernels and devices: the
 *   largest;  host syncs: the sum (at most 15);  fused flag set.
 * Returns 0 if a row or an edge is invalid.
 */
int orc_fuse(const orc_params_t *p, const orc_desc_t *d, const float *edge, int64_t a,
             int64_t len, orc_fdesc_t *o)
{
    memset(o, 0, sizeof(*o));
    for (int64_t k = a; k < a + len; ++k) {
        if (!desc_valid(DESC_ARGS(d, k))) return 0;
        if (k < a + len - 1 && !(isfinite((double)edge[k]) && edge[k] >= 0.0f)) return 0;
    }
    if (len == 1) {
        o->F = d->F[a]; o->B = d->B[a]; o->r1 = d->r1[a]; o->r2 = d->r2[a]; o->r3 = d->r3[a];
        o->K = d->K[a]; o->u = d->u[a]; o->W = d->W[a];
        o->v = d->vgpr[a]; o->s = d->lds[a]; o->gpack = d->gpack[a]; o->G = d->grid[a];
        return 1;
    }
    double F = 0, Bs = 0, E = 0, r1 = 0, r2 = 0, r3 = 0, K = 0, Ws = 0, tc = 0, Fmax = -1.0;
    int64_t v = 0, s = 0, g = 0, G = 0, nc = 0, nd = 0, ns = 0, dt = 0;
    for (int64_t k = a; k < a + len; ++k) {
        const double Fk = d->F[k], Bk = d->B[k];
        const int64_t gp = d->gpack[k];
        const int64_t dtk = (gp >> 11) & 7;
        F += Fk;
        Bs += Bk;
        r1 += (double)d->r1[k] * Bk;
        r2 += (double)d->r2[k] * Bk;
        r3 += (double)d->r3[k] * Bk;
        K += d->K[k];
        Ws += d->W[k];
        if (Fk > 0.0) tc += Fk / ((double)d->u[k] * p->theta[8 + dtk]);
        if (Fk > Fmax) { Fmax = Fk; dt = dtk; }
        if (k < a + len - 1) E += edge[k];
        v = d->vgpr[k] > v ? d->vgpr[k] : v;
        s = d->lds[k] > s ? d->lds[k] : s;
        g = (gp & 2047) > g ? (gp & 2047) : g;
        G = d->grid[k] > G ? d->grid[k] : G;
        nc = ((gp >> 14) & 7) > nc ? ((gp >> 14) & 7) : nc;
        nd = ((gp >> 17) & 7) > nd ? ((gp >> 17) & 7) : nd;
        ns += (gp >> 21) & 15;
    }
    o->F = F;
    o->B = Bs - 2.0 * E > 0.0 ? Bs - 2.0 * E : 0.0;
    o->r1 = Bs > 0.0 ? r1 / Bs : 0.0;
    o->r2 = Bs > 0.0 ? r2 / Bs : 0.0;
    o->r3 = Bs > 0.0 ? r3 / Bs : 0.0;
    o->K = K;
    o->W = Ws - E > 0.0 ? Ws - E : 0.0;
    if (F > 0.0) {
        double u = F / (p->theta[8 + dt] * tc);
        o->u = u < 1.0 ? u : 1.0;
    } else {
        o->u = 1.0;
    }
    o->v = v; o->s = s; o->G = G;
    ns = ns < 15 ? ns : 15;
    o->gpack = g | (dt << 11) | (nc << 14) | (nd << 17) | ((int64_t)1 << 20) | (ns << 21);
    return 1;
}

/* Modelled time of rows a .. a+len-1 run as one kernel; NaN if invalid. */
double orc_fused_cost(const orc_params_t *p, const orc_desc_t *d, const float *edge, int64_t a,
                      int64_t len)
{
    orc_fdesc_t f;
    if (!orc_fuse(p, d, edge, a, len, &f)) return NAN;
    orc_trace_t tr;
    orc_eval(p, f.F, f.B, f.r1, f.r2, f.r3, f.K, f.u, f.W, f.v, f.s, f.gpack, f.G, &tr, NULL);
    return tr.T;
}

/*
 * Chain c owns rows [off[c], off[c+1]) in execution order.  A plan cuts the
 * chain into runs of 1 .. R consecutive rows, each run one kernel; its cost
 * is the sum of the runs' modelled times (NaN counts as +inf).  Dynamic
 * programming over the prefix: best[j] = min over run lengths L (1 .. R,
 * shortest first, strict improvement) of best[j - L] + cost(run of the L
 * rows ending at j).  total[c] = best over the whole chain (+inf if no plan
 * is finite), unfused[c] = the all-singles plan, start[i] = 1 where a run of
 * the chosen plan begins.
 */
void orc_plan_fusion(const orc_params_t *p, const orc_desc_t *d, const float *edge,
                     const int32_t *off, int64_t n_chains, int32_t R, double *total,
                     double *unfused, uint8_t *start)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < n_chains; ++c) {
        int64_t a = off[c], n = off[c + 1] - off[c];
        double *best = (double *)malloc(sizeof(double) * (size_t)(n + 1));
        int64_t *cut = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        best[0] = 0.0;
        double single = 0.0;
        for (int64_t j = 1; j <= n; ++j) {
            best[j] = INFINITY;
            cut[j] = 1;
            for (int64_t L = 1; L <= R && L <= j; ++L) {
                double t = orc_fused_cost(p, d, edge, a + j - L, L);
                if (!(t == t)) t = INFINITY;
                if (L == 1) single += t;
                double v = best[j - L] + t;
                if (v < best[j]) { best[j] = v; cut[j] = L; }
            }
        }
        total[c] = best[n];
        unfused[c] = single;
        for (int64_t i = a; i < a + n; ++i) start[i] = 0;
        int64_t j = n;
        while (j > 0) {
            start[a + j - cut[j]] = 1;
            j -= cut[j];
        }
        free(best);
        free(cut);
    }
}

/*
 * Vector-Jacobian product of the application totals: out[0..23] =
 * sum_a w_a dT_a/dtheta, out[24..30] = sum_a w_a dT_a/d(segment parameters),
 * over applications with finite T_a.  Fixed-order sums.
 */
void orc_apps_vjp(const orc_params_t *p, const orc_segp_t *q, const orc_desc_t *d,
                  const orc_segs_t *s, const double *w_app, double *out)
{
    const int NO = N_THETA + ORC_NSEG;
    int64_t na = s->n_apps;
    double *part = (double *)calloc((size_t)(na > 0 ? na : 1) * NO, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < na; ++a) {
        double *row = part + a * NO;
        double tot = 0.0;
        for (int64_t i = s->app_off[a]; i < s->app_off[a + 1]; ++i)
            tot += orc_segment(p, q, d, s, i, NULL, NULL);
        if (!isfinite(tot)) continue;
        const double w = w_app[a];
        double dth[N_THETA], dsp[ORC_NSEG];
        for (int64_t i = s->app_off[a]; i < s->app_off[a + 1]; ++i) {
            orc_segment(p, q, d, s, i, dth, dsp);
            for (int j = 0; j < N_THETA; ++j) row[j] += w * dth[j];
            for (int j = 0; j < ORC_NSEG; ++j) row[N_THETA + j] += w * dsp[j];
        }
    }
    memset(out, 0, sizeof(double) * NO);
    for (int64_t a = 0; a < na; ++a)
        for (int j = 0; j < NO; ++j) out[j] += part[a * NO + j];
    free(part);
}

/* Thread count of the OpenMP loops (the CPU-baseline measurement times the
 * oracle on one core and on all cores); returns the count in effect. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
