// Stable LSD radix sort of 64-bit keys (8-bit digits) and the top-k ranking built on it.
//
// Each wavefront owns a tile of kTile consecutive keys.  Per pass: (1) every tile counts its
// digits, (2) one block turns the digit-major count table into exclusive offsets, (3) every
// tile scatters its keys in index order; a key's rank among equal digits of its 64-key round
// comes from eight ballots, so the scatter is stable without atomics.
#include "common.h"

namespace ligate {

constexpr int kItems = 16;               // keys per lane per tile
constexpr int kTile = kWave * kItems;    // keys per wavefront tile
constexpr int kSortWaves = 4;            // wavefronts per block
constexpr int kScanThreads = 1024;

static inline int64_t n_tiles(int64_t n) { return (n + kTile - 1) / kTile; }
static inline size_t al(size_t v) { return (v + 255) & ~size_t(255); }

size_t radix_sort_ws_bytes(int64_t n) {
    return al(sizeof(uint64_t) * (size_t)n) + al(sizeof(uint32_t) * 256 * (size_t)n_tiles(n));
}

__global__ __launch_bounds__(kWave *kSortWaves) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                               int shift, uint32_t *__restrict__ hist,
                                                               int64_t ntiles) {
    __shared__ uint32_t cnt[kSortWaves][256];
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t tile = (int64_t)blockIdx.x * kSortWaves + w;
    if (tile >= ntiles) return;
    for (int d = lane; d < 256; d += kWave) cnt[w][d] = 0u;
    wave_sync();
    const int64_t base = tile * kTile;
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = base + r * kWave + lane;
        if (idx < n) atomicAdd(&cnt[w][(keys[idx] >> shift) & 255u], 1u);
    }
    wave_sync();
    for (int d = lane; d < 256; d += kWave) hist[(int64_t)d * ntiles + tile] = cnt[w][d];
}

// Exclusive prefix sum over `total` counters, in place, by one block.
__global__ __launch_bounds__(kScanThreads) void k_rs_scan(uint32_t *__restrict__ a, int64_t total) {
    __shared__ uint32_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t seg = (total + kScanThreads - 1) / kScanThreads;
    const int64_t lo = t * seg, hi = min(total, lo + seg);
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += a[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {  // Hillis-Steele inclusive scan
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t ? part[t - 1] : 0u;
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kWave *kSortWaves) void k_rs_scatter(const uint64_t *__restrict__ in,
                                                                  uint64_t *__restrict__ out, int64_t n, int shift,
                                                                  const uint32_t *__restrict__ offs, int64_t ntiles) {
    __shared__ uint32_t run[kSortWaves][256];
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t tile = (int64_t)blockIdx.x * kSortWaves + w;
    if (tile >= ntiles) return;
    for (int d = lane; d < 256; d += kWave) run[w][d] = offs[(int64_t)d * ntiles + tile];
    wave_sync();
    const int64_t base = tile * kTile;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = base + r * kWave + lane;
        const bool valid = idx < n;
        const uint64_t key = valid ? in[idx] : 0ull;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(valid && bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t pos = run[w][d] + (uint32_t)__popcll(peers & below);
        if (valid) out[pos] = key;
        wave_sync();
        const bool leader = valid && (63 - __clzll((long long)peers)) == lane;
        if (leader) run[w][d] += (uint32_t)__popcll(peers);
        wave_sync();
    }
}

int radix_sort_u64(uint64_t *d_keys, int64_t n, int lo_bit, int hi_bit, void *d_ws, hipStream_t stream) {
    if (n <= 1) return DOCK_OK;
    LIGATE_REQUIRE(lo_bit % 16 == 0 && hi_bit % 16 == 0 && lo_bit < hi_bit && hi_bit <= 64, DOCK_ERR_INVALID_ARG,
                   "radix sort bit range");
    const int64_t nt = n_tiles(n);
    uint64_t *alt = (uint64_t *)d_ws;
    uint32_t *hist = (uint32_t *)((char *)d_ws + al(sizeof(uint64_t) * (size_t)n));
    const unsigned blocks = (unsigned)((nt + kSortWaves - 1) / kSortWaves);
    uint64_t *src = d_keys, *dst = alt;
    for (int shift = lo_bit; shift < hi_bit; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(blocks), dim3(kWave * kSortWaves), 0, stream, src, n, shift, hist, nt);
        hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(kScanThreads), 0, stream, hist, 256 * nt);
        hipLaunchKernelGGL(k_rs_scatter, dim3(blocks), dim3(kWave * kSortWaves), 0, stream, src, dst, n, shift, hist,
                           nt);
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    // an even number of passes leaves the result in d_keys
    return check_launch("radix sort");
}

// ---------------------------------------------------------------------------------------------
// Top-k
// ---------------------------------------------------------------------------------------------

__global__ void k_topk_keys(const float *__restrict__ s, const int32_t *__restrict__ ids, int64_t n,
                            uint64_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t id = ids ? (uint32_t)ids[i] : (uint32_t)i;
    keys[i] = ((uint64_t)float_to_ordered(s[i]) << 32) | id;
}

__global__ void k_topk_out(const uint64_t *__restrict__ keys, int32_t k, float *__restrict__ os,
                           int32_t *__restrict__ oi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const uint64_t key = keys[i];
    os[i] = ordered_to_float((uint32_t)(key >> 32));
    oi[i] = (int32_t)(uint32_t)key;
}

}  // namespace ligate

using namespace ligate;

extern "C" int dock_topk(const float *d_scores, const int32_t *d_ids, int64_t n, int32_t k, float *d_out_scores,
                         int32_t *d_out_ids, void *d_ws, size_t *ws_bytes, void *stream) {
    LIGATE_ABI_RANGE();
    LIGATE_REQUIRE(n >= 1 && n < (1ll << 31), DOCK_ERR_INVALID_ARG, "n must be in [1, 2^31)");
    LIGATE_REQUIRE(k >= 1 && k <= n, DOCK_ERR_INVALID_ARG, "k must be in [1, n]");
    LIGATE_REQUIRE(ws_bytes != nullptr, DOCK_ERR_INVALID_ARG, "ws_bytes is NULL");
    const size_t need = al(sizeof(uint64_t) * (size_t)n) + radix_sort_ws_bytes(n);
    if (d_ws == nullptr) {
        *ws_bytes = need;
        return DOCK_OK;
    }
    LIGATE_REQUIRE(*ws_bytes >= need, DOCK_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", *ws_bytes, need);
    LIGATE_REQUIRE(d_scores && d_out_scores && d_out_ids, DOCK_ERR_INVALID_ARG, "NULL array");
    hipStream_t st = (hipStream_t)stream;
    uint64_t *keys = (uint64_t *)d_ws;
    void *rws = (char *)d_ws + al(sizeof(uint64_t) * (size_t)n);
    hipLaunchKernelGGL(k_topk_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d_scores, d_ids, n, keys);
    // ids 0..n-1 are already in index order, so a stable sort of the score half suffices
    int rc = radix_sort_u64(keys, n, d_ids ? 0 : 32, 64, rws, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_topk_out, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, st, keys, k, d_out_scores,
                       d_out_ids);
    return check_launch("dock_topk");
}

namespace ligate {

__global__ void k_merge_pockets(const float *__restrict__ scores, int n_pockets, int64_t n, float *best,
                                int32_t *pocket) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float b = INFINITY;
    int bp = -1;
    for (int p = 0; p < n_pockets; ++p) {
        float v = scores[(int64_t)p * n + i];
        v = v != v ? INFINITY : v;
        if (v < b) {
            b = v;
            bp = p;
        }
    }
    best[i] = b;
    pocket[i] = bp;
}

}  // namespace ligate

extern "C" int dock_merge_pockets(const float *d_scores, int32_t n_pockets, int64_t n, float *d_best,
                                  int32_t *d_pocket, void *stream) {
    LIGATE_ABI_RANGE();
    LIGATE_REQUIRE(n_pockets >= 1 && n_pockets <= 1024, DOCK_ERR_INVALID_ARG, "n_pockets must be in [1, 1024]");
    LIGATE_REQUIRE(n >= 1 && n < (1ll << 31), DOCK_ERR_INVALID_ARG, "n must be in [1, 2^31)");
    LIGATE_REQUIRE(d_scores && d_best && d_pocket, DOCK_ERR_INVALID_ARG, "NULL array");
    hipLaunchKernelGGL(ligate::k_merge_pockets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       d_scores, n_pockets, n, d_best, d_pocket);
    return ligate::check_launch("dock_merge_pockets");
}
