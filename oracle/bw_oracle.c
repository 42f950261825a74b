/*
 * bw_oracle.c -- plain FP64 CPU reference for the Blackwell stage-centric
 * execution-time model (Section IV-A of the paper, "NVIDIA Blackwell Model":
 * Eq. (2) TMEM per-tile time, Eq. (3) per-CTA compute, Eq. (4) TMA multicast,
 * Eq. (5) decompression and the sub-byte unpack / mbarrier terms, Eq. (6)
 * 2-SM CTA pairs, Eq. (7) I/O overlap, Eq. (8) K-step time, and the kernel
 * total of the workflow paragraph of Section IV-D).
 *
 * TEST INFRASTRUCTURE ONLY: nothing in the product library links, includes
 * or calls this file; it shares no header, helper or table with the HIP
 * implementation.  Scalar double arithmetic, one descriptor at a time, in
 * the order the paper states the terms; built with -ffp-contract=off.
 *
 * One descriptor is one tile kernel: tile bM x bN x bK, Kt K-steps per tile,
 * G CTAs, data type, 2-SM pair mode, TMEM strategy (B: the A tile also goes
 * through TMEM), multicast participants P_A / P_B, barriers per K-step,
 * compressed operands with ratio CR, output element bytes.
 *
 * Readings (the paper leaves them open; each is pinned by a test):
 *   - rates are per SM (TMEM, TMA, tensor throughput, link, unpack, store,
 *     DSMEM); latencies are in cycles at f_clk;
 *   - accumulators are 4 bytes per element (8 for FP64); a CTA needs
 *     bM bN x that in TMEM; CTAs resident per SM = min(max_cta, floor(TMEM /
 *     accumulator bytes)), 0 (+inf time) when the accumulator exceeds TMEM;
 *   - Eq. (2) per K-step: accumulator read (plus the A tile under strategy
 *     B) at the TMEM read rate, L_mma, accumulator write at the write rate;
 *   - Eq. (3): 2 bM bN bK / (R_TC[dtype] S_mode) + T_TMEM + T_mgmt, with
 *     S_mode = S_2SM for pairs, 1 otherwise, and the TMEM management
 *     (L_alloc + L_dealloc) amortised over the Kt steps (Eq. (8) text);
 *   - Eq. (4): one TMA latency per K-step plus the A and B tile bytes, each
 *     divided by its multicast participants, at B_TMA (the two loads are
 *     summed: issued back to back by one producer);
 *   - Eq. (6): a pair loads 2 M_A + M_B for two CTAs, i.e. M_A + M_B / 2
 *     per CTA, plus the DSMEM exchange of the shared B half (M_B / 2 at
 *     BW_shared), and one L_commit per K-step;
 *   - Eq. (5): compressed operands go through the decompression engine at
 *     CR BW_link eta_DE (uncompressed bytes); FP4 operands add the sub-byte
 *     unpack (bytes / R_decomp + L_decomp_setup);
 *   - Eq. (7) with the exposed fraction eps = 1 - alpha as the parameter
 *     (positive, so calibration in log space keeps it meaningful);
 *   - Eq. (8) as printed: T_step = max(T_compute, T_io^eff) + T_sync +
 *     O_misc, where T_io^eff already contains T_sync (the sync is paid on
 *     the I/O path and again per step);
 *   - kernel: T = T_launch + n_r (Kt T_step + T_store) with n_r =
 *     ceil(G / (N_SM c)) rounds and the C-tile writeback T_store = bM bN
 *     ob / B_gmem + L_store_setup once per tile.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BW_NTHETA 24

enum {
    B_TMEM_R = 0, B_TMEM_W = 1, B_L_MMA = 2,
    B_RTC0 = 3, /* 3..7: fp64, tf32, fp16/bf16, fp8, fp4 tensor flop/s per SM */
    B_S2SM = 8, B_L_TMA = 9, B_B_TMA = 10, B_L_MBAR = 11, B_L_COMMIT = 12,
    B_BW_LINK = 13, B_ETA_DE = 14, B_R_DECOMP = 15, B_L_DSETUP = 16, B_EPS = 17,
    B_B_GMEM = 18, B_L_STORE = 19, B_L_TMGMT = 20, B_O_MISC = 21, B_T_LAUNCH = 22,
    B_BW_DSM = 23
};

typedef struct {
    int32_t n_sm, max_cta;
    int64_t tmem_bytes;
    double f_clk;
    double theta[BW_NTHETA];
} bw_params_t;

typedef struct {
    const int32_t *bM, *bN, *bK, *G, *flags;
    const float *Kt, *CR, *ob;
    int64_t n;
} bw_desc_t;

typedef struct {
    int32_t valid, compute_bound, c, pad_;
    int64_t n_r;
    double MA, MB, D_acc, T_tmem, T_mgmt, T_compute, T_tma, T_decomp, T_dsm, T_sync, T_io, T_step,
        T_store, T;
} bw_trace_t;

static const double elem_bytes[5] = {8.0, 4.0, 2.0, 1.0, 0.5};

/*
 * flags: [0,3) dtype (0 fp64, 1 tf32, 2 fp16/bf16, 3 fp8, 4 fp4), [3] 2-SM
 * pair, [4] TMEM strategy B, [5,9) P_A - 1, [9,13) P_B - 1, [13,16) barriers
 * per K-step, [16] compressed; other bits zero.
 */
void bw_eval(const bw_params_t *p, int64_t bM, int64_t bN, int64_t bK, int64_t G, int64_t flags,
             double Kt, double CR, double ob, bw_trace_t *tr, double *dT)
{
    const double *th = p->theta;
    const double f = p->f_clk;
    memset(tr, 0, sizeof(*tr));
    if (dT) memset(dT, 0, sizeof(double) * BW_NTHETA);
    tr->T = NAN;
    const int64_t dt = flags & 7;
    const int pair = (int)((flags >> 3) & 1), stratB = (int)((flags >> 4) & 1);
    const int64_t PA = ((flags >> 5) & 15) + 1, PB = ((flags >> 9) & 15) + 1;
    const int64_t nbar = (flags >> 13) & 7;
    const int comp = (int)((flags >> 16) & 1);
    if (bM < 1 || bN < 1 || bK < 1 || G < 1 || flags < 0 || (flags >> 17) != 0 || dt > 4) return;
    if (!(isfinite(Kt) && Kt >= 1.0) || !(isfinite(CR) && CR >= 1.0) || !(isfinite(ob) && ob > 0.0))
        return;
    tr->valid = 1;

    /* TMEM residency and rounds */
    const double acc_b = dt == 0 ? 8.0 : 4.0;
    tr->D_acc = (double)bM * (double)bN * acc_b;
    int64_t c = (int64_t)floor((double)p->tmem_bytes / tr->D_acc);
    if (c > p->max_cta) c = p->max_cta;
    tr->c = (int32_t)c;
    if (c < 1) { tr->T = INFINITY; return; }
    tr->n_r = (G + (int64_t)p->n_sm * c - 1) / ((int64_t)p->n_sm * c);

    const double e = elem_bytes[dt];
    tr->MA = (double)bM * (double)bK * e;
    tr->MB = (double)bN * (double)bK * e;

    /* Eq. (2), Eq. (3) */
    const double D_read = tr->D_acc + (stratB ? tr->MA : 0.0);
    tr->T_tmem = D_read / th[B_TMEM_R] + th[B_L_MMA] / f + tr->D_acc / th[B_TMEM_W];
    tr->T_mgmt = th[B_L_TMGMT] / f / Kt;
    const double S_mode = pair ? th[B_S2SM] : 1.0;
    const double fl = 2.0 * (double)bM * (double)bN * (double)bK;
    const double T_mma = fl / (th[B_RTC0 + dt] * S_mode);
    tr->T_compute = T_mma + tr->T_tmem + tr->T_mgmt;

    /* Eq. (4), Eq. (6) */
    const double ta = tr->MA / (double)PA;
    const double tb = (pair ? 0.5 * tr->MB : tr->MB) / (double)PB;
    tr->T_tma = th[B_L_TMA] / f + (ta + tb) / th[B_B_TMA];
    tr->T_dsm = pair ? 0.5 * tr->MB / th[B_BW_DSM] : 0.0;

    /* Eq. (5): decompression engine, sub-byte unpack */
    const double Dab = tr->MA + tr->MB;
    double T_de = 0.0, T_up = 0.0;
    if (comp) T_de = Dab / (CR * th[B_BW_LINK] * th[B_ETA_DE]);
    if (dt == 4) T_up = Dab / th[B_R_DECOMP] + th[B_L_DSETUP] / f;
    tr->T_decomp = T_de + T_up;

    /* mbarrier / commit sync per K-step */
    tr->T_sync = (double)nbar * th[B_L_MBAR] / f + (pair ? th[B_L_COMMIT] / f : 0.0);

    /* Eq. (7), Eq. (8) */
    const double io_raw = tr->T_tma + tr->T_decomp + tr->T_dsm;
    tr->T_io = th[B_EPS] * io_raw + tr->T_sync;
    tr->compute_bound = tr->T_compute >= tr->T_io;
    const double Tm = tr->compute_bound ? tr->T_compute : tr->T_io;
    tr->T_step = Tm + tr->T_sync + th[B_O_MISC];
    tr->T_store = (double)bM * (double)bN * ob / th[B_B_GMEM] + th[B_L_STORE] / f;
    const double nr = (double)tr->n_r;
    tr->T = th[B_T_LAUNCH] + nr * (Kt * tr->T_step + tr->T_store);

    if (!dT) return;
    /* dT/dtheta: the first maximal stage (compute on ties) is active */
    const double cs = nr * Kt;                 /* weight of T_step */
    dT[B_T_LAUNCH] = 1.0;
    dT[B_O_MISC] = cs;
    dT[B_B_GMEM] = -nr * (double)bM * (double)bN * ob / (th[B_B_GMEM] * th[B_B_GMEM]);
    dT[B_L_STORE] = nr / f;
    /* T_sync appears in T_step directly and, when I/O is the maximum, inside T_io */
    const double ws = cs * (tr->compute_bound ? 1.0 : 2.0);
    dT[B_L_MBAR] = ws * (double)nbar / f;
    if (pair) dT[B_L_COMMIT] = ws / f;
    if (tr->compute_bound) {
        const double w = cs;
        dT[B_TMEM_R] = -w * D_read / (th[B_TMEM_R] * th[B_TMEM_R]);
        dT[B_TMEM_W] = -w * tr->D_acc / (th[B_TMEM_W] * th[B_TMEM_W]);
        dT[B_L_MMA] = w / f;
        dT[B_L_TMGMT] = w / f / Kt;
        dT[B_RTC0 + dt] = -w * T_mma / th[B_RTC0 + dt];
        if (pair) dT[B_S2SM] = -w * T_mma / th[B_S2SM];
    } else {
        const double w = cs * th[B_EPS];
        dT[B_EPS] = cs * io_raw;
        dT[B_L_TMA] = w / f;
        dT[B_B_TMA] = -w * (ta + tb) / (th[B_B_TMA] * th[B_B_TMA]);
        if (pair) dT[B_BW_DSM] = -w * 0.5 * tr->MB / (th[B_BW_DSM] * th[B_BW_DSM]);
        if (comp) {
            dT[B_BW_LINK] = -w * T_de / th[B_BW_LINK];
            dT[B_ETA_DE] = -w * T_de / th[B_ETA_DE];
        }
        if (dt == 4) {
            dT[B_R_DECOMP] = -w * Dab / (th[B_R_DECOMP] * th[B_R_DECOMP]);
            dT[B_L_DSETUP] = w / f;
        }
    }
}

#define BW_ARGS(d, i) (int64_t)(d)->bM[i], (int64_t)(d)->bN[i], (int64_t)(d)->bK[i], \
    (int64_t)(d)->G[i], (int64_t)(d)->flags[i], (double)(d)->Kt[i], (double)(d)->CR[i], \
    (double)(d)->ob[i]

void bw_predict(const bw_params_t *p, const bw_desc_t *d, double *T, int32_t *cta)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < d->n; ++i) {
        bw_trace_t tr;
        bw_eval(p, BW_ARGS(d, i), &tr, NULL);
        T[i] = tr.T;
        if (cta) cta[i] = tr.valid ? tr.c : -1;
    }
}

void bw_trace(const bw_params_t *p, const bw_desc_t *d, bw_trace_t *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < d->n; ++i) bw_eval(p, BW_ARGS(d, i), &out[i], NULL);
}

void bw_jacobian(const bw_params_t *p, const bw_desc_t *d, double *J)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < d->n; ++i) {
        bw_trace_t tr;
        bw_eval(p, BW_ARGS(d, i), &tr, J + i * BW_NTHETA);
    }
}

/*
 * mode 0: out[2..25] = sum_i w_i dT_i/dtheta over descriptors with finite T;
 * mode 1: mean relative error against measured w_i (finite, > 0) and its
 * gradient: out[0] loss, out[1] count, out[2..25] gradient.  Partial sums
 * over fixed chunks of 4096 descriptors, added in chunk order.
 */
void bw_weighted_grad(const bw_params_t *p, const bw_desc_t *d, const float *w_in, int mode,
                      double *out)
{
    const int64_t n = d->n, CH = 4096;
    const int64_t nch = (n + CH - 1) / CH;
    double *part = (double *)calloc((size_t)(nch > 0 ? nch : 1) * 26, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nch; ++c) {
        double *row = part + c * 26;
        double J[BW_NTHETA];
        for (int64_t i = c * CH; i < n && i < (c + 1) * CH; ++i) {
            bw_trace_t tr;
            bw_eval(p, BW_ARGS(d, i), &tr, J);
            if (!isfinite(tr.T)) continue;
            double wt;
            if (mode == 1) {
                const double m = w_in[i];
                if (!(isfinite(m) && m > 0.0)) continue;
                row[0] += fabs(tr.T - m) / m;
                row[1] += 1.0;
                wt = tr.T > m ? 1.0 / m : (tr.T < m ? -1.0 / m : 0.0);
            } else {
                wt = w_in[i];
            }
            for (int j = 0; j < BW_NTHETA; ++j) row[2 + j] += wt * J[j];
        }
    }
    memset(out, 0, sizeof(double) * 26);
    for (int64_t c = 0; c < nch; ++c)
        for (int j = 0; j < 26; ++j) out[j] += part[c * 26 + j];
    free(part);
    if (mode == 1 && out[1] > 0.0) {
        out[0] /= out[1];
        for (int j = 2; j < 26; ++j) out[j] /= out[1];
    }
}

/*
 * Calibration (Section IV-D), as for the CDNA model: Adam on phi = log theta
 * for the slots in free_mask, learning rate decayed geometrically from lr to
 * lr_final over the steps, FP64 moments; hist[t] = loss before step t.
 * Returns 1 if the loss or a gradient slot was not finite or a fitted theta
 * left (0, inf): theta_out is then the last theta with a finite loss and the
 * remaining history entries are NaN.
 */
int bw_calibrate(const bw_params_t *p0, const bw_desc_t *d, const float *m, int32_t steps,
                 double lr0, double lr_final, double b1, double b2, double eps, uint32_t mask,
                 bw_params_t *p_out, double *hist)
{
    bw_params_t p = *p0, last_ok = *p0;
    double phi[BW_NTHETA], mom[BW_NTHETA], vel[BW_NTHETA], out[26];
    for (int j = 0; j < BW_NTHETA; ++j) {
        phi[j] = (mask >> j & 1u) ? log(p.theta[j]) : 0.0;
        mom[j] = 0.0;
        vel[j] = 0.0;
    }
    for (int t = 1; t <= steps; ++t) {
        bw_weighted_grad(&p, d, m, 1, out);
        if (hist) hist[t - 1] = out[0];
        int finite = isfinite(out[0]);
        for (int j = 0; j < BW_NTHETA; ++j) finite = finite && isfinite(out[2 + j]);
        int ok = finite;
        bw_params_t next = p;
        if (finite) {
            last_ok = p;
            double lr = lr0;
            if (lr_final > 0.0 && steps > 1)
                lr = lr0 * pow(lr_final / lr0, (double)(t - 1) / (double)(steps - 1));
            const double b1t = pow(b1, (double)t), b2t = pow(b2, (double)t);
            for (int j = 0; j < BW_NTHETA; ++j) {
                if (!(mask >> j & 1u)) continue;
                const double g = p.theta[j] * out[2 + j];
                mom[j] = b1 * mom[j] + (1.0 - b1) * g;
                vel[j] = b2 * vel[j] + (1.0 - b2) * g * g;
                phi[j] -= lr * (mom[j] / (1.0 - b1t)) / (sqrt(vel[j] / (1.0 - b2t)) + eps);
                next.theta[j] = exp(phi[j]);
                ok = ok && isfinite(next.theta[j]) && next.theta[j] > 0.0;
            }
        }
        if (!ok) {
            if (hist)
                for (int k = t; k < steps; ++k) hist[k] = NAN;
            *p_out = last_ok;
            return 1;
        }
        p = next;
    }
    *p_out = p;
    return 0;
}
