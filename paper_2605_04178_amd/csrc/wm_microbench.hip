// wm_microbench.hip -- libwmbench.so: the microbenchmarks that measure the
// model's hardware parameters on the GPU it runs on (Section IV-D: bandwidth
// and latency per memory level, matrix and vector throughput per data type,
// working-set sweep for h_LLC(W); launch, workgroup-dispatch and barrier
// costs; Table "parameters"), and a set of validation kernels with known
// flops and bytes whose measured times the calibrated model is scored on
// (Section V-A).  Public interface: include/wm_microbench.h.
//
// Every kernel here reads and writes only inside the buffers the caller
// passes with their sizes; the pointer chase masks every index with
// n_nodes - 1 (n_nodes a power of two), so any contents of the chain array
// stay in bounds.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <functional>
#include <vector>

#include "../../include/wm_microbench.h"

namespace {

thread_local int32_t g_last_hip = 0;

int32_t fail(hipError_t e)
{
    g_last_hip = (int32_t)e;
    return WMB_EHIP;
}

#define WMB_HIP(call)                                 \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return fail(e_);        \
    } while (0)

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef int i16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// microbenchmarks
// ---------------------------------------------------------------------------

// Read bandwidth: each thread sums float4s, `passes` times, with ordinary
// (cached) loads.  SHARED = false: grid-stride partition of the buffer (a
// block rereads its own partition, so a partition that fits a cache level is
// served from it after the first pass); SHARED = true: every block reads the
// whole buffer (per-CU caches see all of it).
template <bool SHARED>
__global__ __launch_bounds__(256) void k_mb_read(const f4* __restrict__ buf, int64_t n4,
                                                 int32_t passes, float* __restrict__ sink)
{
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const int64_t stride = SHARED ? (int64_t)blockDim.x : (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = SHARED ? (int64_t)threadIdx.x : (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int32_t p = 0; p < passes; ++p)
        for (int64_t i = i0; i < n4; i += stride) acc += buf[i];
    const float s = acc.x + acc.y + acc.z + acc.w;
    if (s == -1.0f) sink[0] = s;  // keeps the loads; the buffers hold non-negative values
}

// Dependent-load latency: one lane follows next[] for `steps` steps.
__global__ __launch_bounds__(64) void k_mb_chase(const uint32_t* __restrict__ next, uint32_t mask,
                                                 int64_t steps, uint32_t* __restrict__ sink,
                                                 int64_t* __restrict__ ticks)
{
    if (threadIdx.x != 0) return;
    uint32_t i = 0;
    const int64_t t0 = wall_clock64();
    for (int64_t s = 0; s < steps; ++s) i = next[i & mask];
    const int64_t t1 = wall_clock64();
    sink[0] = i;
    ticks[0] = t1 - t0;
}

// Shader clock: every thread runs a chain of `spins` dependent FMAs; the
// first lane of block 0 reads the shader-cycle counter (clock64) and the
// constant-rate wall clock (wall_clock64) before and after its chain.
__global__ __launch_bounds__(64) void k_mb_clock(int32_t spins, float seed, float* __restrict__ sink,
                                                 int64_t* __restrict__ ticks)
{
    const int64_t c0 = clock64(), w0 = wall_clock64();
    float x = seed + (float)threadIdx.x + (float)(c0 & 1);
    for (int32_t i = 0; i < spins; ++i) x = __builtin_fmaf(x, 0.9999999f, 1e-7f);
    // the chain's result enters the second reading, which therefore follows it
    const int64_t c1 = clock64() + (x == -1.0f ? 1 : 0);
    const int64_t w1 = wall_clock64();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ticks[0] = c1 - c0;
        ticks[1] = w1 - w0;
    }
    if (x == -1.0f) sink[0] = x;  // keeps the chain; it never reaches -1
}

// Throughput per data type: independent accumulator chains per wave.
template <int KIND>
__global__ __launch_bounds__(256) void k_mb_peak(int32_t iters, float seed, float* __restrict__ sink)
{
    float out = 0.0f;
    if constexpr (KIND == WMB_PEAK_FP64) {
        d4v c[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) c[j] = d4v{0, 0, 0, 0};
        const double a = seed + threadIdx.x, b = seed * 0.5;
        for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 8; ++j) c[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[j], 0, 0, 0);
        }
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) t += c[j][j & 3];
        out = (float)t;
    } else if constexpr (KIND == WMB_PEAK_FP32) {
        float x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = seed + (float)(threadIdx.x + j);
        const float m = 0.999f, c = seed * 1e-3f;
        for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = __builtin_fmaf(x[j], m, c);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) out += x[j];
    } else if constexpr (KIND == WMB_PEAK_BF16) {
        f16v c0 = {}, c1 = {}, c2 = {}, c3 = {};
        bf8v a;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = (__bf16)(seed + (float)j);
        for (int32_t i = 0; i < iters; ++i) {
            c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, c1, 0, 0, 0);
            c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, c2, 0, 0, 0);
            c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, c3, 0, 0, 0);
        }
        out = c0[0] + c1[1] + c2[2] + c3[3];
    } else if constexpr (KIND == WMB_PEAK_FP8) {
        f16v c0 = {}, c1 = {};
        i8v a;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = 0x38383838 + j;
        for (int32_t i = 0; i < iters; ++i) {
            c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, a, c0, 0, 0, 0, 127, 0, 127);
            c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, a, c1, 0, 0, 0, 127, 0, 127);
        }
        out = c0[0] + c1[1] + seed;
    } else {  // WMB_PEAK_INT8
        i16v c0 = {}, c1 = {}, c2 = {}, c3 = {};
        i4v a;
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = 0x01010101 * (j + 1);
        for (int32_t i = 0; i < iters; ++i) {
            c0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, c1, 0, 0, 0);
            c2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, c2, 0, 0, 0);
            c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, c3, 0, 0, 0);
        }
        out = (float)(c0[0] + c1[1] + c2[2] + c3[3]) + seed;
    }
    if (out == -12345.0f) sink[threadIdx.x] = out;
}

// Flops one wave issues per loop iteration of k_mb_peak<KIND>.
double peak_flops_per_wave_iter(int kind)
{
    switch (kind) {
    case WMB_PEAK_FP64: return 8.0 * 2.0 * 16 * 16 * 4;       // 8 x v_mfma_f64_16x16x4
    case WMB_PEAK_FP32: return 8.0 * 2.0 * 64;                // 8 FMAs per lane
    case WMB_PEAK_BF16: return 4.0 * 2.0 * 32 * 32 * 16;      // 4 x 32x32x16
    case WMB_PEAK_FP8: return 2.0 * 2.0 * 32 * 32 * 64;       // 2 x 32x32x64
    default: return 4.0 * 2.0 * 32 * 32 * 32;                 // 4 x i8 32x32x32
    }
}

// Launch / dispatch / barrier costs: every thread passes `barriers` barriers.
__global__ void k_mb_empty(int32_t barriers, int32_t* __restrict__ sink)
{
    for (int32_t i = 0; i < barriers; ++i) __syncthreads();
    if (barriers < 0) sink[0] = 1;
}

// ---------------------------------------------------------------------------
// validation kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_val_copy(const f4* __restrict__ a, f4* __restrict__ b,
                                                  int64_t n4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_val_triad(const f4* __restrict__ a, const f4* __restrict__ b,
                                                   f4* __restrict__ c, float s, int64_t n4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) c[i] = a[i] + s * b[i];
}

// `iters` dependent FMAs per element: flops / byte = iters / 4.
__global__ __launch_bounds__(256) void k_val_fma(const f4* __restrict__ a, f4* __restrict__ b,
                                                 int32_t iters, int64_t n4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4) return;
    f4 x = a[i];
    const float m = 0.9999f, c = 1e-4f;
    for (int32_t k = 0; k < iters; ++k) {
        x.x = __builtin_fmaf(x.x, m, c);
        x.y = __builtin_fmaf(x.y, m, c);
        x.z = __builtin_fmaf(x.z, m, c);
        x.w = __builtin_fmaf(x.w, m, c);
    }
    b[i] = x;
}

// Five-point stencil on an nx x ny grid (interior points).
__global__ __launch_bounds__(256) void k_val_stencil(const float* __restrict__ in, float* __restrict__ out,
                                                     int32_t nx, int32_t ny)
{
    const int32_t x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int32_t y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x < 1 || y < 1 || x >= nx - 1 || y >= ny - 1) return;
    const int64_t i = (int64_t)y * nx + x;
    out[i] = 0.2f * (in[i] + in[i - 1] + in[i + 1] + in[i - nx] + in[i + nx]);
}

// Transpose of an n x n matrix: naive (coalesced reads, strided writes) and
// through a padded 32 x 32 LDS tile.
__global__ __launch_bounds__(256) void k_val_transpose_naive(const float* __restrict__ in,
                                                             float* __restrict__ out, int32_t n)
{
    const int32_t x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int32_t y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x < n && y < n) out[(int64_t)x * n + y] = in[(int64_t)y * n + x];
}

__global__ __launch_bounds__(256) void k_val_transpose_lds(const float* __restrict__ in,
                                                           float* __restrict__ out, int32_t n)
{
    __shared__ float tile[32][33];
    const int32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int32_t x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    for (int32_t r = ty; r < 32; r += 8) {
        const int32_t x = x0 + tx, y = y0 + r;
        if (x < n && y < n) tile[r][tx] = in[(int64_t)y * n + x];
    }
    __syncthreads();
    for (int32_t r = ty; r < 32; r += 8) {
        const int32_t x = y0 + tx, y = x0 + r;
        if (x < n && y < n) out[(int64_t)y * n + x] = tile[tx][r];
    }
}

// Block sums of n floats (one partial per block).
__global__ __launch_bounds__(256) void k_val_reduce(const f4* __restrict__ a, int64_t n4,
                                                    float* __restrict__ part)
{
    __shared__ float red[4];
    float s = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const f4 v = a[i];
        s += (v.x + v.y) + (v.z + v.w);
    }
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// FP32 GEMM C = A B (n x n, row-major) with T x T workgroup tiles staged in
// LDS, one output per thread: the classic occupancy / tile-size study.
template <int T>
__global__ __launch_bounds__(T * T) void k_val_gemm_tile(const float* __restrict__ A,
                                                        const float* __restrict__ B,
                                                        float* __restrict__ C, int32_t n)
{
    __shared__ float As[T][T + 1], Bs[T][T + 1];
    const int32_t tx = threadIdx.x % T, ty = threadIdx.x / T;
    const int32_t row = blockIdx.y * T + ty, col = blockIdx.x * T + tx;
    float acc = 0.0f;
    for (int32_t k0 = 0; k0 < n; k0 += T) {
        As[ty][tx] = (row < n && k0 + tx < n) ? A[(int64_t)row * n + k0 + tx] : 0.0f;
        Bs[ty][tx] = (k0 + ty < n && col < n) ? B[(int64_t)(k0 + ty) * n + col] : 0.0f;
        __syncthreads();
#pragma unroll
        for (int32_t k = 0; k < T; ++k) acc = __builtin_fmaf(As[ty][k], Bs[k][tx], acc);
        __syncthreads();
    }
    if (row < n && col < n) C[(int64_t)row * n + col] = acc;
}

// BF16 GEMM C = A B^T (A: n x n row-major, Bt: n x n row-major holding B
// transposed, C fp32) on matrix cores: a 256-thread block owns a 64 x 64
// tile, each wave one 32 x 32 quarter, v_mfma_f32_32x32x16_bf16 over K in
// steps of 16; operands are read straight from global memory (each lane
// loads 8 consecutive bf16 = 16 bytes of one row).  n must be a multiple of 64.
// BIAS: the epilogue adds bias[column] (the fused GEMM + bias of the fusion
// microbenchmark).
template <bool BIAS>
__global__ __launch_bounds__(256) void k_val_gemm_mfma(const __bf16* __restrict__ A,
                                                       const __bf16* __restrict__ Bt,
                                                       const float* __restrict__ bias,
                                                       float* __restrict__ C, int32_t n)
{
    const int32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t r0 = blockIdx.y * 64 + (w >> 1) * 32, c0 = blockIdx.x * 64 + (w & 1) * 32;
    // operand layout: lane l supplies row (l % 32), k-slice (l / 32) * 8 .. + 8
    const int32_t rr = lane & 31, kk = (lane >> 5) * 8;
    const __bf16* pa = A + (int64_t)(r0 + rr) * n + kk;
    const __bf16* pb = Bt + (int64_t)(c0 + rr) * n + kk;
    f16v acc = {};
    for (int32_t k = 0; k < n; k += 16) {
        const bf8v a = *reinterpret_cast<const bf8v*>(pa + k);
        const bf8v b = *reinterpret_cast<const bf8v*>(pb + k);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    // result layout: lane l holds column (l % 32), rows 8 (j / 4) + 4 (l / 32) + (j % 4)
    const float bc = BIAS ? bias[c0 + rr] : 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int32_t r = r0 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        C[(int64_t)r * n + c0 + rr] = BIAS ? acc[j] + bc : acc[j];
    }
}

// C[r][c] += bias[c] over an n x n float matrix (n % 4 == 0), one float4
// per thread: the unfused second kernel of the fusion microbenchmark.
__global__ __launch_bounds__(256) void k_val_bias(const float* __restrict__ bias, f4* __restrict__ C,
                                                  int32_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n4 = (int64_t)n * n / 4;
    if (i >= n4) return;
    const int32_t c = (int32_t)((i * 4) % n);
    const f4 b = *reinterpret_cast<const f4*>(bias + c);
    C[i] += b;
}

const void* val_kernel(int32_t kind)
{
    switch (kind) {
    case WMB_VAL_COPY: return reinterpret_cast<const void*>(&k_val_copy);
    case WMB_VAL_TRIAD: return reinterpret_cast<const void*>(&k_val_triad);
    case WMB_VAL_FMA: return reinterpret_cast<const void*>(&k_val_fma);
    case WMB_VAL_STENCIL: return reinterpret_cast<const void*>(&k_val_stencil);
    case WMB_VAL_TRANSPOSE_NAIVE: return reinterpret_cast<const void*>(&k_val_transpose_naive);
    case WMB_VAL_TRANSPOSE_LDS: return reinterpret_cast<const void*>(&k_val_transpose_lds);
    case WMB_VAL_REDUCE: return reinterpret_cast<const void*>(&k_val_reduce);
    case WMB_VAL_GEMM8: return reinterpret_cast<const void*>(&k_val_gemm_tile<8>);
    case WMB_VAL_GEMM16: return reinterpret_cast<const void*>(&k_val_gemm_tile<16>);
    case WMB_VAL_GEMM32: return reinterpret_cast<const void*>(&k_val_gemm_tile<32>);
    case WMB_VAL_GEMM_MFMA: return reinterpret_cast<const void*>(&k_val_gemm_mfma<false>);
    case WMB_VAL_BIAS: return reinterpret_cast<const void*>(&k_val_bias);
    case WMB_VAL_GEMM_MFMA_BIAS: return reinterpret_cast<const void*>(&k_val_gemm_mfma<true>);
    default: return nullptr;
    }
}

// median of `launches` event-timed runs of `run` (after one warm-up), seconds
template <typename F>
int32_t median_time(hipStream_t s, int32_t launches, F run, double* seconds)
{
    hipEvent_t a = nullptr, b = nullptr;
    WMB_HIP(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(e);
    }
    std::vector<float> t;
    e = run();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (int32_t r = 0; r < launches && e == hipSuccess; ++r) {
        e = hipEventRecord(a, s);
        if (e == hipSuccess) e = run();
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(e);
    std::sort(t.begin(), t.end());
    *seconds = 1e-3 * (double)t[t.size() / 2];
    return WMB_OK;
}

bool blk_ok(int32_t b) { return b >= 64 && b <= 1024 && b % 64 == 0; }

}  // namespace

extern "C" {

int32_t wmb_last_hip_error(void) { return g_last_hip; }

int32_t wmb_read_bw(const void* buf, int64_t bytes, int32_t passes, int32_t blocks, int32_t shared,
                    float* sink, int32_t launches, void* stream, double* seconds)
{
    if (!buf || !sink || !seconds || bytes < 16 || (bytes & 15) || passes < 1 || blocks < 1 ||
        launches < 1 || ((uintptr_t)buf & 15))
        return WMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n4 = bytes / 16;
    return median_time(s, launches, [&]() {
        if (shared) k_mb_read<true><<<blocks, 256, 0, s>>>((const f4*)buf, n4, passes, sink);
        else k_mb_read<false><<<blocks, 256, 0, s>>>((const f4*)buf, n4, passes, sink);
        return hipGetLastError();
    }, seconds);
}

int32_t wmb_chase(const uint32_t* next, int64_t n_nodes, int64_t steps, int64_t warm_steps, uint32_t* sink,
                  int64_t* ticks, void* stream, double* ns_per_step)
{
    if (!next || !sink || !ticks || !ns_per_step || n_nodes < 1 || (n_nodes & (n_nodes - 1)) ||
        n_nodes > (1ll << 32) || steps < 1 || warm_steps < 0)
        return WMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, khz = 0;
    WMB_HIP(hipGetDevice(&dev));
    WMB_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return WMB_EHIP;
    const uint32_t mask = (uint32_t)(n_nodes - 1);
    // an untimed pass of warm_steps steps from node 0 (the timed pass then
    // revisits the same nodes first), then the timed pass from node 0
    if (warm_steps > 0) {
        k_mb_chase<<<1, 64, 0, s>>>(next, mask, warm_steps, sink, ticks);
        WMB_HIP(hipGetLastError());
    }
    k_mb_chase<<<1, 64, 0, s>>>(next, mask, steps, sink, ticks);
    WMB_HIP(hipGetLastError());
    int64_t t = 0;
    WMB_HIP(hipMemcpyAsync(&t, ticks, sizeof(t), hipMemcpyDeviceToHost, s));
    WMB_HIP(hipStreamSynchronize(s));
    *ns_per_step = (double)t * 1e6 / (double)khz / (double)steps;
    return WMB_OK;
}

int32_t wmb_clock(int32_t blocks, int32_t spins, float* sink, int64_t* ticks, void* stream, double* hz)
{
    if (blocks < 1 || blocks > (1 << 20) || spins < 1 || !sink || !ticks || !hz) return WMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, khz = 0;
    WMB_HIP(hipGetDevice(&dev));
    WMB_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return WMB_EHIP;
    // a warm-up launch (the clock ramps under load), then the measured one
    k_mb_clock<<<blocks, 64, 0, s>>>(spins, 1.0f, sink, ticks);
    WMB_HIP(hipGetLastError());
    k_mb_clock<<<blocks, 64, 0, s>>>(spins, 1.0f, sink, ticks);
    WMB_HIP(hipGetLastError());
    int64_t t[2] = {0, 0};
    WMB_HIP(hipMemcpyAsync(t, ticks, sizeof(t), hipMemcpyDeviceToHost, s));
    WMB_HIP(hipStreamSynchronize(s));
    if (t[1] <= 0) return WMB_EHIP;
    *hz = (double)t[0] * (double)khz * 1e3 / (double)t[1];
    return WMB_OK;
}

int32_t wmb_peak(int32_t kind, int32_t iters, int32_t blocks, float* sink, int32_t launches,
                 void* stream, double* seconds, double* flops)
{
    if (kind < 0 || kind > 4 || iters < 1 || blocks < 1 || !sink || launches < 1 || !seconds || !flops)
        return WMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    auto run = [&]() -> hipError_t {
        switch (kind) {
        case WMB_PEAK_FP64: k_mb_peak<WMB_PEAK_FP64><<<blocks, 256, 0, s>>>(iters, 1.0f, sink); break;
        case WMB_PEAK_FP32: k_mb_peak<WMB_PEAK_FP32><<<blocks, 256, 0, s>>>(iters, 1.0f, sink); break;
        case WMB_PEAK_BF16: k_mb_peak<WMB_PEAK_BF16><<<blocks, 256, 0, s>>>(iters, 1.0f, sink); break;
        case WMB_PEAK_FP8: k_mb_peak<WMB_PEAK_FP8><<<blocks, 256, 0, s>>>(iters, 1.0f, sink); break;
        default: k_mb_peak<WMB_PEAK_INT8><<<blocks, 256, 0, s>>>(iters, 1.0f, sink); break;
        }
        return hipGetLastError();
    };
    *flops = peak_flops_per_wave_iter(kind) * (double)iters * 4.0 * (double)blocks;
    return median_time(s, launches, run, seconds);
}

int32_t wmb_empty(int32_t blocks, int32_t block, int32_t barriers, int32_t* sink, int32_t launches,
                  void* stream, double* seconds)
{
    if (blocks < 1 || !blk_ok(block) || barriers < 0 || !sink || launches < 1 || !seconds)
        return WMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    return median_time(s, launches, [&]() {
        k_mb_empty<<<blocks, block, 0, s>>>(barriers, sink);
        return hipGetLastError();
    }, seconds);
}

int32_t wmb_sync(int32_t reps, int32_t* sink, void* stream, double* per_sync)
{
    if (reps < 1 || !sink || !per_sync) return WMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    using clk = std::chrono::steady_clock;
    k_mb_empty<<<1, 64, 0, s>>>(0, sink);
    WMB_HIP(hipGetLastError());
    WMB_HIP(hipStreamSynchronize(s));
    const auto t0 = clk::now();
    for (int32_t r = 0; r < reps; ++r) {
        k_mb_empty<<<1, 64, 0, s>>>(0, sink);
        WMB_HIP(hipGetLastError());
        WMB_HIP(hipStreamSynchronize(s));
    }
    const auto t1 = clk::now();
    for (int32_t r = 0; r < reps; ++r) {
        k_mb_empty<<<1, 64, 0, s>>>(0, sink);
        WMB_HIP(hipGetLastError());
    }
    WMB_HIP(hipStreamSynchronize(s));
    const auto t2 = clk::now();
    const double with_sync = std::chrono::duration<double>(t1 - t0).count();
    const double without = std::chrono::duration<double>(t2 - t1).count();
    *per_sync = (with_sync - without) / (double)reps;
    return WMB_OK;
}

int32_t wmb_val_attr(int32_t kind, int32_t* vgprs, int32_t* lds_bytes, int32_t* block)
{
    const void* k = val_kernel(kind);
    if (!k || !vgprs || !lds_bytes || !block) return WMB_EINVAL;
    hipFuncAttributes a;
    WMB_HIP(hipFuncGetAttributes(&a, k));
    *vgprs = a.numRegs;
    *lds_bytes = (int32_t)a.sharedSizeBytes;
    switch (kind) {
    case WMB_VAL_GEMM8: *block = 64; break;
    case WMB_VAL_GEMM16: *block = 256; break;
    case WMB_VAL_GEMM32: *block = 1024; break;
    default: *block = 256; break;
    }
    return WMB_OK;
}

int64_t wmb_val_bytes(int32_t kind, int64_t n, int32_t which)
{
    if (!val_kernel(kind) || n < 1 || which < 0 || which > 2) return -1;
    if (kind == WMB_VAL_BIAS || kind == WMB_VAL_GEMM_MFMA_BIAS) {
        if (n > 65536 || n % 64) return -1;
        const int64_t el = n * n;
        if (kind == WMB_VAL_BIAS) return which == 0 ? n * 4 : (which == 1 ? 0 : el * 4);
        return which == 0 ? el * 2 : (which == 1 ? el * 2 + n * 4 : el * 4);
    }
    const bool two_d = kind == WMB_VAL_STENCIL || kind == WMB_VAL_TRANSPOSE_NAIVE ||
                       kind == WMB_VAL_TRANSPOSE_LDS || kind >= WMB_VAL_GEMM8;
    if (two_d) {
        if (n > 65536 || (kind == WMB_VAL_GEMM_MFMA && n % 64)) return -1;
        const int64_t el = n * n;
        const bool has_b = kind >= WMB_VAL_GEMM8;
        if (which == 1) return has_b ? el * (kind == WMB_VAL_GEMM_MFMA ? 2 : 4) : 0;
        if (which == 0) return el * (kind == WMB_VAL_GEMM_MFMA ? 2 : 4);
        return el * 4;
    }
    if ((n & 3) || n / 4 / 256 >= 0x7fffffffll) return -1;
    if (kind == WMB_VAL_REDUCE) return which == 0 ? n * 4 : (which == 2 ? 4096 * 4 : 0);
    if (which == 1) return kind == WMB_VAL_TRIAD ? n * 4 : 0;
    return n * 4;
}

int32_t wmb_val_run(int32_t kind, const void* a, int64_t a_bytes, const void* b, int64_t b_bytes,
                    void* c, int64_t c_bytes, int64_t n, int32_t iters, int32_t launches,
                    void* stream, double* seconds, int64_t* grid)
{
    if (!val_kernel(kind) || n < 1 || launches < 1 || !seconds || !grid) return WMB_EINVAL;
    const int64_t na = wmb_val_bytes(kind, n, 0), nb = wmb_val_bytes(kind, n, 1),
                  nc = wmb_val_bytes(kind, n, 2);
    if (na < 0 || !a || !c || a_bytes < na || c_bytes < nc || (nb > 0 && (!b || b_bytes < nb)))
        return WMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::function<hipError_t()> run;
    const int64_t n4 = n / 4;
    const int32_t m = (int32_t)(n < 65536 ? n : 65536);
    switch (kind) {
    case WMB_VAL_COPY:
    case WMB_VAL_TRIAD:
    case WMB_VAL_FMA: {
        if (kind == WMB_VAL_FMA && iters < 0) return WMB_EINVAL;
        const int64_t g = (n4 + 255) / 256;
        *grid = g;
        run = [=]() {
            if (kind == WMB_VAL_COPY) k_val_copy<<<g, 256, 0, s>>>((const f4*)a, (f4*)c, n4);
            else if (kind == WMB_VAL_TRIAD)
                k_val_triad<<<g, 256, 0, s>>>((const f4*)a, (const f4*)b, (f4*)c, 1.5f, n4);
            else k_val_fma<<<g, 256, 0, s>>>((const f4*)a, (f4*)c, iters, n4);
            return hipGetLastError();
        };
        break;
    }
    case WMB_VAL_REDUCE: {
        const int64_t g = std::min<int64_t>((n4 + 255) / 256, 4096);
        *grid = g;
        run = [=]() {
            k_val_reduce<<<g, 256, 0, s>>>((const f4*)a, n4, (float*)c);
            return hipGetLastError();
        };
        break;
    }
    case WMB_VAL_STENCIL:
    case WMB_VAL_TRANSPOSE_NAIVE: {
        const dim3 g((m + 63) / 64, (m + 3) / 4);
        *grid = (int64_t)g.x * g.y;
        run = [=]() {
            if (kind == WMB_VAL_STENCIL) k_val_stencil<<<g, 256, 0, s>>>((const float*)a, (float*)c, m, m);
            else k_val_transpose_naive<<<g, 256, 0, s>>>((const float*)a, (float*)c, m);
            return hipGetLastError();
        };
        break;
    }
    case WMB_VAL_TRANSPOSE_LDS: {
        const dim3 g((m + 31) / 32, (m + 31) / 32);
        *grid = (int64_t)g.x * g.y;
        run = [=]() {
            k_val_transpose_lds<<<g, 256, 0, s>>>((const float*)a, (float*)c, m);
            return hipGetLastError();
        };
        break;
    }
    case WMB_VAL_GEMM8:
    case WMB_VAL_GEMM16:
    case WMB_VAL_GEMM32: {
        const int t = kind == WMB_VAL_GEMM8 ? 8 : (kind == WMB_VAL_GEMM16 ? 16 : 32);
        const dim3 g((m + t - 1) / t, (m + t - 1) / t);
        *grid = (int64_t)g.x * g.y;
        run = [=]() {
            if (t == 8) k_val_gemm_tile<8><<<g, 64, 0, s>>>((const float*)a, (const float*)b, (float*)c, m);
            else if (t == 16) k_val_gemm_tile<16><<<g, 256, 0, s>>>((const float*)a, (const float*)b, (float*)c, m);
            else k_val_gemm_tile<32><<<g, 1024, 0, s>>>((const float*)a, (const float*)b, (float*)c, m);
            return hipGetLastError();
        };
        break;
    }
    case WMB_VAL_GEMM_MFMA: {
        if (((uintptr_t)a & 15) || ((uintptr_t)b & 15)) return WMB_EINVAL;
        const dim3 g(m / 64, m / 64);
        *grid = (int64_t)g.x * g.y;
        run = [=]() {
            k_val_gemm_mfma<false><<<g, 256, 0, s>>>((const __bf16*)a, (const __bf16*)b, nullptr, (float*)c, m);
            return hipGetLastError();
        };
        break;
    }
    case WMB_VAL_GEMM_MFMA_BIAS: {
        if (((uintptr_t)a & 15) || ((uintptr_t)b & 15)) return WMB_EINVAL;
        const dim3 g(m / 64, m / 64);
        *grid = (int64_t)g.x * g.y;
        // the bias vector follows Bt in buffer b
        const float* bias = (const float*)((const char*)b + (int64_t)m * m * 2);
        run = [=]() {
            k_val_gemm_mfma<true><<<g, 256, 0, s>>>((const __bf16*)a, (const __bf16*)b, bias, (float*)c, m);
            return hipGetLastError();
        };
        break;
    }
    case WMB_VAL_BIAS: {
        if (((uintptr_t)a & 15) || ((uintptr_t)c & 15)) return WMB_EINVAL;
        const int64_t g = ((int64_t)m * m / 4 + 255) / 256;
        *grid = g;
        run = [=]() {
            k_val_bias<<<g, 256, 0, s>>>((const float*)a, (f4*)c, m);
            return hipGetLastError();
        };
        break;
    }
    default:
        return WMB_EINVAL;
    }
    return median_time(s, launches, run, seconds);
}

}  // extern "C"
