/*
 * wm_microbench.h -- C ABI of libwmbench.so: microbenchmarks that measure the
 * hardware parameters of the wavefront-centric model on the GPU they run on,
 * and validation kernels with known flops and bytes.
 *
 * The paper derives its parameters from microbenchmarks (Section IV-D; the
 * MI300A list: bandwidth and latency of each cache level and HBM, matrix
 * throughput by data type, the h_LLC(W) working-set sweep; Table
 * "parameters": launch, interference, fusion and transfer constants) and
 * scores the model on measured kernel times (Section V-A).  These calls are
 * the measuring side of that workflow on gfx950.
 *
 * Conventions: array arguments are DEVICE memory owned by the caller
 * (16-byte aligned where noted); `stream` is a hipStream_t as void*; every
 * call synchronises `stream` before returning (it reports host results).
 * Times are medians of `launches` event-timed launches after one warm-up.
 * Status: 0 ok, -1 invalid argument (checked before any HIP call),
 * -3 HIP error (code from wmb_last_hip_error()).
 */
#ifndef WM_MICROBENCH_H
#define WM_MICROBENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WMB_OK 0
#define WMB_EINVAL (-1)
#define WMB_EHIP (-3)

/* data types of the throughput benchmark (the model's dtype order) */
#define WMB_PEAK_FP64 0   /* v_mfma_f64_16x16x4f64 */
#define WMB_PEAK_FP32 1   /* vector FMA (no packed FP32) */
#define WMB_PEAK_BF16 2   /* v_mfma_f32_32x32x16_bf16 */
#define WMB_PEAK_FP8 3    /* v_mfma_scale_f32_32x32x64_f8f6f4, fp8 e4m3 */
#define WMB_PEAK_INT8 4   /* v_mfma_i32_32x32x32_i8 */

/* validation kernels */
#define WMB_VAL_COPY 0             /* b = a, n floats (16-B vectors) */
#define WMB_VAL_TRIAD 1            /* c = a + 1.5 b, n floats */
#define WMB_VAL_FMA 2              /* b = (iters dependent FMAs of a), n floats */
#define WMB_VAL_STENCIL 3          /* 5-point stencil, n x n floats */
#define WMB_VAL_TRANSPOSE_NAIVE 4  /* n x n transpose, strided writes */
#define WMB_VAL_TRANSPOSE_LDS 5    /* n x n transpose through a 32 x 33 LDS tile */
#define WMB_VAL_REDUCE 6           /* per-block sums of n floats (<= 4096 blocks) */
#define WMB_VAL_GEMM8 7            /* FP32 GEMM n x n, 8 x 8 LDS tiles, one output per thread */
#define WMB_VAL_GEMM16 8           /* same, 16 x 16 */
#define WMB_VAL_GEMM32 9           /* same, 32 x 32 */
#define WMB_VAL_GEMM_MFMA 10       /* BF16 C = A B^T on matrix cores, 64 x 64 tiles, n % 64 == 0 */
#define WMB_VAL_BIAS 11            /* c[r][col] += a[col], n x n floats, n % 64 == 0 */
#define WMB_VAL_GEMM_MFMA_BIAS 12  /* GEMM_MFMA with the bias added in its epilogue: b holds
                                      B^T (bf16) followed by the n float bias values */

int32_t wmb_last_hip_error(void);

/* Read bandwidth: `blocks` blocks of 256 threads sum float4s of buf[bytes]
 * `passes` times with ordinary loads: shared = 0, each block its grid-stride
 * partition (bytes read per launch = bytes * passes); shared = 1, every block
 * the whole buffer (bytes * passes * blocks).  bytes a positive multiple of
 * 16, buf 16-byte aligned; sink: 1 float.  seconds: median per launch. */
int32_t wmb_read_bw(const void *buf, int64_t bytes, int32_t passes, int32_t blocks, int32_t shared,
                    float *sink, int32_t launches, void *stream, double *seconds);

/* Dependent-load latency: one lane follows i = next[i & (n_nodes - 1)] from
 * i = 0 for `steps` steps (n_nodes a power of two <= 2^32; any contents stay
 * in bounds), timed on the device wall clock.  An untimed pass of
 * warm_steps (>= 0) steps from i = 0 runs first, so a timed pass of at most
 * warm_steps steps revisits lines the warm pass brought into the caches;
 * warm_steps = 0 times a cold pass.  sink: 1 uint32; ticks: 1 int64 (device
 * scratch).  ns_per_step: host. */
int32_t wmb_chase(const uint32_t *next, int64_t n_nodes, int64_t steps, int64_t warm_steps, uint32_t *sink,
                  int64_t *ticks, void *stream, double *ns_per_step);

/* Shader clock: `blocks` workgroups of one wave each run `spins` dependent
 * FMAs; block 0 reads the shader-cycle counter and the constant-rate wall
 * clock around its chain.  hz (host) = cycles / seconds of that chain, on the
 * second of two launches.  blocks 1 gives the clock of a lightly loaded
 * part, several per CU the clock under load.  sink: 1 float (never
 * written); ticks: 2 int64 (device scratch). */
int32_t wmb_clock(int32_t blocks, int32_t spins, float *sink, int64_t *ticks, void *stream,
                  double *hz);

/* Throughput of data type `kind` (WMB_PEAK_*): `blocks` blocks of 4 waves,
 * `iters` iterations of independent instruction chains per wave.  flops:
 * operations per launch (host); seconds: median time per launch.
 * sink: 256 floats. */
int32_t wmb_peak(int32_t kind, int32_t iters, int32_t blocks, float *sink, int32_t launches,
                 void *stream, double *seconds, double *flops);

/* Launch, workgroup-dispatch and barrier costs: `blocks` workgroups of
 * `block` threads (multiple of 64, <= 1024), each thread passing
 * `barriers` workgroup barriers; sink: 1 int32 (never written). */
int32_t wmb_empty(int32_t blocks, int32_t block, int32_t barriers, int32_t *sink, int32_t launches,
                  void *stream, double *seconds);

/* Cost of one host synchronisation (Section IV-E, tau_sync): `reps` empty
 * kernels each followed by hipStreamSynchronize against `reps` launched back
 * to back and synchronised once; per_sync (host) = the difference per
 * kernel, host wall clock.  sink: 1 int32 (never written). */
int32_t wmb_sync(int32_t reps, int32_t *sink, void *stream, double *per_sync);

/* Resources of validation kernel `kind` as compiled: VGPRs per thread, static
 * LDS bytes per workgroup, threads per workgroup (host outputs). */
int32_t wmb_val_attr(int32_t kind, int32_t *vgprs, int32_t *lds_bytes, int32_t *block);

/* Bytes validation kernel `kind` needs at size n in buffer `which`
 * (0 = a, 1 = b, 2 = c); 0 if the buffer is unused, -1 for a bad kind or n. */
int64_t wmb_val_bytes(int32_t kind, int64_t n, int32_t which);

/* Time validation kernel `kind` at size n (element count for the 1-D kernels,
 * a multiple of 4; matrix order for the 2-D ones, <= 65536): buffers a, b, c
 * with their sizes in bytes, at least wmb_val_bytes(); iters = FMA count of
 * WMB_VAL_FMA.  seconds: median per launch; grid: workgroups launched. */
int32_t wmb_val_run(int32_t kind, const void *a, int64_t a_bytes, const void *b, int64_t b_bytes,
                    void *c, int64_t c_bytes, int64_t n, int32_t iters, int32_t launches,
                    void *stream, double *seconds, int64_t *grid);

#ifdef __cplusplus
}
#endif

#endif /* WM_MICROBENCH_H */
