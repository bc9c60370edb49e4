// scan.hip -- device-wide exclusive prefix sum over int64 (three phases:
// tile sums, scan of tile sums, tile scan with carried offset).
#include "internal.h"

namespace fsm {
namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* excl) {
    __shared__ int64_t wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(v, lane);
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int64_t before = 0, total = 0;
#pragma unroll
    for (int i = 0; i < SCAN_THREADS / 64; ++i) {
        if (i < wv) before += wsum[i];
        total += wsum[i];
    }
    *excl = before + inc - v;
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_tile_sums(const int64_t* in, int64_t n,
                                                            int64_t* sums) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        if (i < n) s += in[i];
    }
    int64_t excl;
    int64_t total = block_excl_scan(s, &excl);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_tile_scan(const int64_t* in, int64_t* out,
                                                            int64_t n, const int64_t* offs) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    int64_t excl;
    block_excl_scan(s, &excl);
    int64_t run = excl + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

}  // namespace

int64_t scan_exclusive(const int64_t* in, int64_t* out, int64_t n) {
    if (n <= 0) return 0;
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles > (1ll << 31) - 1) fail(FSM_EOVERFLOW, "scan of %lld items too large", (long long)n);
    if (tiles == 1) {
        DBuf<int64_t> total(1);
        k_tile_sums<<<1, SCAN_THREADS, 0, stream()>>>(in, n, total.p);
        FSM_LAUNCH_CHECK();
        int64_t t = scalar_to_host(total.p);
        k_tile_scan<<<1, SCAN_THREADS, 0, stream()>>>(in, out, n, nullptr);
        FSM_LAUNCH_CHECK();
        return t;
    }
    DBuf<int64_t> sums((size_t)tiles);
    k_tile_sums<<<(unsigned)tiles, SCAN_THREADS, 0, stream()>>>(in, n, sums.p);
    FSM_LAUNCH_CHECK();
    DBuf<int64_t> offs((size_t)tiles);
    int64_t total = scan_exclusive(sums.p, offs.p, tiles);
    k_tile_scan<<<(unsigned)tiles, SCAN_THREADS, 0, stream()>>>(in, out, n, offs.p);
    FSM_LAUNCH_CHECK();
    return total;
}

}  // namespace fsm
