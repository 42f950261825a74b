// wm_tile.hip -- gfx950 kernel of occupancy-driven tile selection (Section
// IV-B, adaptive tile selection): every candidate GEMM tile of a shape becomes
// a kernel descriptor whose predicted time is its cost, and the cheapest wins.
//
// Layout: shapes are structure-of-arrays, candidate codes one flat uint32
// array with CSR offsets per shape.  Persistent waves take batches of eight
// consecutive shapes and lay their candidate lists end to end over the lanes
// (float32 costs kept in registers); the float64 re-evaluations of the
// near-minimum window queue up in LDS across batches and run on all lanes.
#include "wm_device.hpp"

namespace wm {

// GEMM tile -> descriptor.  Tile sizes are powers of two, so the grid, the
// K steps and the panel sizes are shifts of 32-bit integers (every padded
// extent is below 2^32).  Flops and bytes are real quantities formed in R
// from those exact integers: in double they are exact while below 2^53 and
// never overflow; in float they carry a few ulps, which the float64 window
// of the selection absorbs.
template <typename R>
__device__ inline bool derive_tile(int32_t M, int32_t N, int32_t Kd, int32_t t, uint32_t code,
                                   int wave_shift, Desc<R>& x)
{
#pragma clang fp contract(off)
    const uint32_t kdc = (code >> 4) & 3u;
    if ((code >> 9) != 0u || kdc == 3u || M < 1 || N < 1 || Kd < 1 || t < 0 || t > 3) return false;
    const uint32_t lmt = 5u + (code & 3u), lnt = 5u + ((code >> 2) & 3u), lkd = 4u + kdc;
    const uint32_t wpw = ((code >> 6) & 7u) + 1u;
    const uint32_t le = 3u - (uint32_t)t;          // element bytes 8, 4, 2, 1
    const uint32_t eo = t == 3 ? 2u : (1u << le);  // fp8 writes 16-bit results
    const uint32_t acc = t == 0 ? 2u : 1u;
    const uint32_t gm = ((uint32_t)M + (1u << lmt) - 1u) >> lmt;
    const uint32_t gn = ((uint32_t)N + (1u << lnt) - 1u) >> lnt;
    const uint32_t Ks = ((uint32_t)Kd + (1u << lkd) - 1u) >> lkd;
    const uint64_t G = (uint64_t)gm * gn;
    const uint32_t g = wpw << wave_shift;
    if (G > 0x7fffffffull || g > 1024u) return false;
    const uint32_t pan = ((1u << lmt) + (1u << lnt)) << (lkd + le);   // (mt + nt) kd e <= 2^18
    const R fM = (R)(uint32_t)M, fN = (R)(uint32_t)N, fK = (R)(uint32_t)Kd;
    const R Bi = (R)(uint32_t)G * (R)Ks * (R)pan + fM * fN * (R)eo;
    const R Ui = (fM * fK + fK * fN) * (R)(1u << le) + fM * fN * (R)eo;
    x.F = (R)2 * (R)(gm << lmt) * (R)(gn << lnt) * (R)(Ks << lkd);
    x.B = Bi;
    const R r2 = (R)1 - Ui * Ar<R>::rcp(Bi);
    x.r2 = r2 > (R)0 ? r2 : (R)0;
    x.r1 = (R)0;
    x.r3 = (R)0;
    x.K = (R)Ks;
    x.u = (R)1;
    x.W = (R)0;
    // VGPRs: accumulators and the panel share per thread (numerators below
    // 2^19, divisors at most 4096: udiv21 is exact)
    x.v = (int32_t)(udiv21((acc << (lmt + lnt)) + g - 1u, g) + udiv21(pan + 4u * g - 1u, 4u * g) + 16u);
    x.s = (int32_t)(2u * pan);
    x.gp = (int32_t)g | (t << 11);
    x.G = (int32_t)G;
    return true;
}

template <typename R> __device__ inline const Const<R>& cst(const Set& S);
template <> __device__ inline const Const<float>& cst<float>(const Set& S) { return S.cf; }
template <> __device__ inline const Const<double>& cst<double>(const Set& S) { return S.cd; }

// cost of one candidate; invalid codes and infeasible tiles cost +inf
template <typename R>
__device__ inline R tile_cost(const Set& S, int32_t M, int32_t N, int32_t K, int32_t t, uint32_t code)
{
    const R inf = (R)__builtin_huge_val();
    Desc<R> x;
    if (!derive_tile<R>(M, N, K, t, code, S.st.wave_shift, x)) return inf;
    Eval<R> E;
    evaluate<R, false, true>(S.st, cst<R>(S), x, E);
    return E.T == E.T ? E.T : inf;
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, m, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Orders this wave's LDS stores before its later LDS loads from other lanes
// (the LDS executes one wave's operations in issue order; the fences keep
// the compiler from moving accesses across this point).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// float64 minimum, its lowest local index and the second-smallest value of
// a multiset, accumulated in candidate order (exact ties keep the first)
struct Best2 {
    double c1, c2;
    int32_t j1;
    __device__ inline void add(double cd, int32_t jl)
    {
        if (cd < c1 || (cd == c1 && jl < j1)) {
            c2 = c1;
            c1 = cd;
            j1 = jl;
        } else if (cd < c2) {
            c2 = cd;
        }
    }
};

__device__ inline void write_best(const Best2& r, int64_t i, int32_t* best, double* best_cost,
                                  uint8_t* near_tie)
{
    const double dinf = __builtin_huge_val();
    const bool fin = r.c1 < dinf;
    best[i] = fin ? r.j1 : -1;
    best_cost[i] = r.c1;
    near_tie[i] = (fin && r.c2 < dinf && (r.c2 - r.c1) <= 1e-6 * r.c1) ? 1 : 0;
}

constexpr int kTileQueue = 128;   // queued float64 window candidates per wave
constexpr int kTileSlots = 64;    // shapes per queue (one lane each at the end)
constexpr int kTileBatch = 8;     // consecutive shapes whose candidates share wavefronts
constexpr int kTileSpan = 768;    // candidates a batch may hold (12 rounds of 64)

// A batch shape as the lanes of its candidates read it: extents, dtype,
// first batch position P, code index minus batch position D, window
// threshold and rank among the batch's shapes with a finite minimum.
struct alignas(16) TileShape {
    int32_t M, N, K, t;
    int32_t P, D;
    float thr;
    int32_t rank;
};

// Per-wave LDS: the current batch's shapes and float32 costs, and the queue
// of float64 window re-evaluations, shared across batches.  Queue entries
// are appended in (slot, local index) order.
struct TileQueue {
    TileShape bs[kTileBatch];
    float cost32[kTileSpan];
    uint8_t slot32[kTileSpan];       // batch shape of each candidate
    int64_t shape[kTileSlots];
    uint32_t key[kTileQueue];        // slot << 24 | local candidate index
    uint32_t cand[kTileQueue];       // index into the candidate-code array
    double cost[kTileQueue];
    unsigned long long bmin[kTileBatch];   // packed float32 minimum per batch shape
};

__device__ inline uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// first entry in [0, qn) whose slot is >= sl
__device__ inline int first_entry(const TileQueue& q, int qn, uint32_t sl)
{
    int lo = 0, hi = qn;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((q.key[mid] >> 24) < sl) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Evaluates every queued candidate in float64 with all lanes (their codes
// are read here, one load per lane), then one lane per shape scans that
// shape's entries (ascending candidate index) and writes its result.
// Wave-uniform ns, qn.
__device__ inline void flush_tiles(TileQueue& q, int ns, int qn, const Set& S, const ShapePtrs& sh,
                                   const uint32_t* __restrict__ code, int lane, int32_t* best,
                                   double* best_cost, uint8_t* near_tie)
{
    wave_lds_sync();
    for (int e = lane; e < qn; e += 64) {
        const int sl = (int)(q.key[e] >> 24);
        // the shape's fields come back from global memory (cached): keeping
        // them in LDS would cost a wave's sixth slot per SIMD
        const int64_t i = q.shape[sl];
        q.cost[e] = tile_cost<double>(S, sh.M[i], sh.N[i], sh.K[i], sh.dtype[i], code[q.cand[e]]);
    }
    wave_lds_sync();
    if (lane < ns) {
        const int e1 = first_entry(q, qn, (uint32_t)lane + 1u);
        Best2 r{__builtin_huge_val(), __builtin_huge_val(), 0x7fffffff};
        for (int e = first_entry(q, qn, (uint32_t)lane); e < e1; ++e)
            r.add(q.cost[e], (int32_t)(q.key[e] & 0xffffffu));
        write_best(r, q.shape[lane], best, best_cost, near_tie);
    }
    wave_lds_sync();   // the queue is refilled next
}

struct TileCtx {
    ShapePtrs sh;
    const int32_t* off;
    const uint32_t* code;
    int64_t n_cand;
    int32_t* best;
    double* best_cost;
    uint8_t* near_tie;
};

__device__ inline void clamp_list(int64_t n_cand, int64_t& a, int64_t& b)
{
    // offsets are caller data: clamp them into the candidate array
    a = a < 0 ? 0 : (a > n_cand ? n_cand : a);
    b = b < a ? a : (b > n_cand ? n_cand : b);
}

// One shape on the whole wave, without the queue: float32 minimum over its
// list, then the float64 window evaluated lane-parallel and reduced across
// the wave.  For batches too long for LDS or with too large a window.
__device__ inline void direct_shape(const TileCtx& C, const Set& S, int64_t i, int lane)
{
    const double dinf = __builtin_huge_val();
    const float finf = __builtin_huge_valf();
    const int32_t M = C.sh.M[i], N = C.sh.N[i], K = C.sh.K[i], t = C.sh.dtype[i];
    int64_t a = C.off[i], b = C.off[i + 1];
    clamp_list(C.n_cand, a, b);
    uint64_t key = ~0ull;
    for (int64_t j = a + lane; j < b; j += 64) {
        const float c = tile_cost<float>(S, M, N, K, t, C.code[j]);
        const uint64_t k = ((uint64_t)__float_as_uint(c) << 32) | (uint32_t)(j - a);
        key = k < key ? k : key;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o = shfl_xor_u64(key, m);
        key = o < key ? o : key;
    }
    const float c32 = __uint_as_float((uint32_t)(key >> 32));
    Best2 r{dinf, dinf, 0x7fffffff};
    if (key != ~0ull && c32 < finf) {
        const float thr = c32 * (1.0f + kTileWindow);
        for (int64_t j = a + lane; j < b; j += 64) {
            if (!(tile_cost<float>(S, M, N, K, t, C.code[j]) <= thr)) continue;
            r.add(tile_cost<double>(S, M, N, K, t, C.code[j]), (int32_t)(j - a));
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const double oc1 = __shfl_xor(r.c1, m, 64);
        const double oc2 = __shfl_xor(r.c2, m, 64);
        const int32_t oj1 = __shfl_xor(r.j1, m, 64);
        if (oc1 < r.c1 || (oc1 == r.c1 && oj1 < r.j1)) {
            r.c2 = r.c1 < oc2 ? r.c1 : oc2;
            r.c1 = oc1;
            r.j1 = oj1;
        } else {
            r.c2 = oc1 < r.c2 ? oc1 : r.c2;
        }
    }
    if (lane == 0) write_best(r, i, C.best, C.best_cost, C.near_tie);
}

// Persistent waves over batches of kTileBatch consecutive shapes whose
// candidate lists are laid end to end over the lanes, so that short lists
// leave no lane idle.  Pass 1 writes each candidate's float32 cost to LDS
// and takes each shape's minimum with a packed (cost bits, local index) key.
// Every candidate within kTileWindow of its shape's minimum is queued for a
// float64 re-evaluation by a second pass that counts as it appends (a queue
// that overflows is evaluated and the window appended again); the queue
// fills across batches and runs on all lanes at once.  The result per shape is the smallest float64 cost (the
// lowest index winning exact ties) and the second-smallest, for the
// near-tie flag.  A batch of more than kTileSpan candidates, or whose window
// would not fit an empty queue, goes shape by shape without the queue.
// The batch's shapes sit in LDS as 32-byte records that a candidate's lane
// reads by its slot (two 16-byte reads where cross-lane shuffles took seven).
// The LDS of a wave (6720 bytes) leaves room for 24 waves per CU, so the
// kernel asks for 6 waves per SIMD (at most 80 VGPRs).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_select_tile(ShapePtrs sh, const int32_t* __restrict__ off,
                                                      const uint32_t* __restrict__ code, int64_t n,
                                                      int64_t n_cand,
                                                      Set S, int32_t* __restrict__ best,
                                                      double* __restrict__ best_cost,
                                                      uint8_t* __restrict__ near_tie)
{
    constexpr int SB = kTileBatch;
    __shared__ TileQueue queues[BLOCK / 64];
    const int lane = threadIdx.x & 63;
    TileQueue& q = queues[threadIdx.x >> 6];
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * BLOCK + threadIdx.x) >> 6));
    const int64_t nwaves = (int64_t)((gridDim.x * BLOCK) >> 6);
    const TileCtx C{sh, off, code, n_cand, best, best_cost, near_tie};
    const float finf = __builtin_huge_valf();
    const int64_t nb = (n + SB - 1) / SB;
    int ns = 0, qn = 0;
    for (int64_t bt = wave;; bt += nwaves) {
        const bool done = bt >= nb;
        const int64_t s0 = bt * SB;
        // lane k < SB holds shape s0 + k
        const int64_t si = s0 + lane;
        const bool has = !done && lane < SB && si < n;
        int32_t M = 0, N = 0, K = 0, t = 0;
        int64_t a = 0, b = 0;
        if (has) {
            M = sh.M[si];
            N = sh.N[si];
            K = sh.K[si];
            t = sh.dtype[si];
            a = off[si];
            b = off[si + 1];
            clamp_list(n_cand, a, b);
        }
        // list lengths, saturated (a batch past kTileSpan goes shape by shape)
        const int32_t len = (int32_t)(b - a < kTileSpan + 1 ? b - a : kTileSpan + 1);
        int32_t inc = len;   // inclusive prefix over lanes 0..SB-1
#pragma unroll
        for (int d = 1; d < SB; d <<= 1) {
            const int32_t o = __shfl_up(inc, d, 64);
            inc += lane >= d ? o : 0;
        }
        const int32_t T = __builtin_amdgcn_readlane(inc, SB - 1);
        const int32_t P = inc - len;   // first batch position of lane's shape
        const bool queued = !done && T <= kTileSpan;
        float thr = -finf;
        bool fin = false;
        int32_t rank = 0;   // among the batch's shapes with a finite minimum
        if (queued) {
            int32_t Pk[SB];
#pragma unroll
            for (int k = 0; k < SB; ++k) Pk[k] = __builtin_amdgcn_readlane(P, k);
            wave_lds_sync();   // the previous batch's lanes are done reading bs
            if (lane < SB) {
                q.bmin[lane] = ~0ull;
                // a <= n_cand < 2^31 and P < kTileSpan, so D fits 32 bits
                q.bs[lane] = TileShape{M, N, K, t, P, (int32_t)(a - P), 0.0f, 0};
            }
            wave_lds_sync();
            // pass 1: float32 costs to LDS and the per-shape minimum
            for (int32_t v = lane; v < T; v += 64) {
                int32_t sl = 0;
#pragma unroll
                for (int k = 1; k < SB; ++k) sl += v >= Pk[k] ? 1 : 0;
                const TileShape z = q.bs[sl];
                const int32_t jl = v - z.P;
                const float c = tile_cost<float>(S, z.M, z.N, z.K, z.t, code[(int64_t)v + z.D]);
                q.cost32[v] = c;
                q.slot32[v] = (uint8_t)sl;
                __hip_atomic_fetch_min(&q.bmin[sl],
                                       ((unsigned long long)__float_as_uint(c) << 32) | (uint32_t)jl,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
            wave_lds_sync();
            // per shape: the window threshold, or the empty result
            if (has) {
                const unsigned long long key = q.bmin[lane];
                const float c32 = __uint_as_float((uint32_t)(key >> 32));
                fin = key != ~0ull && c32 < finf;
                if (fin) {
                    thr = c32 * (1.0f + kTileWindow);
                } else {
                    best[si] = -1;
                    best_cost[si] = __builtin_huge_val();
                    near_tie[si] = 0;
                }
            }
            rank = (int32_t)lanes_below(__ballot(fin));
            if (lane < SB) {
                q.bs[lane].thr = thr;
                q.bs[lane].rank = rank;
            }
        }
        const int nf = __popcll(__ballot(fin));
        // The one flush site.  Attempt 0 flushes at the end, or when the
        // batch's shapes would not find queue slots; then the batch's window
        // is appended after entry qn (shapes taking slots from ns in batch
        // order), entries past the queue's end counted but not written.  If
        // the queue overflowed, attempt 1 evaluates what it held and appends
        // the window again to the empty queue.
        bool flush = done ? ns > 0 : (queued && ns + nf > kTileSlots);
        int cnt = 0;
        for (int attempt = 0; attempt < 2; ++attempt) {
            if (flush) {
                flush_tiles(q, ns, qn, S, sh, code, lane, best, best_cost, near_tie);
                ns = 0;
                qn = 0;
            }
            if (done || !queued) break;
            if (fin) q.shape[ns + rank] = si;
            wave_lds_sync();   // the shapes' thresholds and ranks
            cnt = 0;
            for (int32_t v = lane; v < ((T + 63) & ~63); v += 64) {
                // every lane takes part in the ballot
                const int sl = v < T ? (int)q.slot32[v] : 0;
                const TileShape z = q.bs[sl];
                const bool w = v < T && q.cost32[v] <= z.thr;
                const uint64_t m = __ballot(w);
                const int e = qn + cnt + (int)lanes_below(m);
                if (w && e < kTileQueue) {
                    const int32_t jl = v - z.P;
                    q.key[e] = ((uint32_t)(ns + z.rank) << 24) | (uint32_t)jl;
                    q.cand[e] = (uint32_t)(v + z.D);
                }
                cnt += __popcll(m);
            }
            flush = qn + cnt > kTileQueue && qn > 0;
            if (!flush) break;
        }
        if (done) break;
        if (!queued || cnt > kTileQueue) {
            // too many candidates for LDS, or a window longer than the whole
            // queue: shape by shape
            for (int k = 0; k < SB && s0 + k < n; ++k) direct_shape(C, S, s0 + k, lane);
            continue;
        }
        qn += cnt;
        ns += nf;
    }
}

template <int BLOCK>
static void select_t(const ShapePtrs& sh, const int32_t* off, const uint32_t* code, int64_t n,
                     int64_t n_cand, const Set& S, int32_t* best, double* best_cost,
                     uint8_t* near_tie, int grid_mult, hipStream_t stream)
{
    const int64_t waves_per_block = BLOCK / 64;
    const int64_t batches = (n + kTileBatch - 1) / kTileBatch;
    const int64_t want = (batches + waves_per_block - 1) / waves_per_block;
    int64_t b = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_select_tile<BLOCK>), BLOCK) *
                (grid_mult < 1 ? 1 : grid_mult);
    b = b < want ? b : want;
    k_select_tile<BLOCK><<<(int)(b < 1 ? 1 : b), BLOCK, 0, stream>>>(sh, off, code, n, n_cand, S, best,
                                                                     best_cost, near_tie);
}

// Every candidate's float32 cost (the selection's first pass): a wave per
// shape, its lanes over the shape's list; grid-stride over shapes.
__global__ __launch_bounds__(256) void k_tile_costs(ShapePtrs sh, const int32_t* __restrict__ off,
                                                     const uint32_t* __restrict__ code, int64_t n,
                                                     int64_t n_cand, Set S, float* __restrict__ cost)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n; i += nw) {
        int64_t a = off[i], b = off[i + 1];
        clamp_list(n_cand, a, b);
        const int32_t M = sh.M[i], N = sh.N[i], K = sh.K[i], t = sh.dtype[i];
        for (int64_t j = a + lane; j < b; j += 64) cost[j] = tile_cost<float>(S, M, N, K, t, code[j]);
    }
}

hipError_t launch_tile_costs(const ShapePtrs& sh, const int32_t* off, const uint32_t* code, int64_t n,
                             int64_t n_cand, const Set& S, float* cost, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 3) / 4;
    const int64_t cap = (int64_t)resident_blocks(reinterpret_cast<const void*>(&k_tile_costs), 256) * 4;
    const int64_t b = want < cap ? want : cap;
    k_tile_costs<<<(int)(b < 1 ? 1 : b), 256, 0, stream>>>(sh, off, code, n, n_cand, S, cost);
    return hipGetLastError();
}

hipError_t launch_select_tile(const ShapePtrs& sh, const int32_t* off, const uint32_t* code,
                              int64_t n, int64_t n_cand, const Set& S, int32_t* best,
                              double* best_cost, uint8_t* near_tie, const LaunchCfg& c,
                              hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    switch (c.block) {
    case 64: select_t<64>(sh, off, code, n, n_cand, S, best, best_cost, near_tie, c.grid_mult, stream); break;
    case 128: select_t<128>(sh, off, code, n, n_cand, S, best, best_cost, near_tie, c.grid_mult, stream); break;
    case 256: select_t<256>(sh, off, code, n, n_cand, S, best, best_cost, near_tie, c.grid_mult, stream); break;
    case 512: select_t<512>(sh, off, code, n, n_cand, S, best, best_cost, near_tie, c.grid_mult, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wm
