// graph.hip -- graph ingest: edge list -> simple undirected CSR with rows
// sorted by neighbour id, and dense label ranks (the labelled graph
// G = (V, E, L) of Section 2.1; vertex labels only, no self-loops, no
// repeated edges).
#include <climits>
#include <cstring>

#include "internal.h"

namespace fsm {
namespace {

constexpr int T = 256;
constexpr int SMALL_ROW = 4096;    // rows up to this length sort in LDS

__global__ void k_mark_labels(const int32_t* lab, int64_t n, int64_t* flag) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        flag[lab[v]] = 1;   // benign race: every writer stores 1
}

__global__ void k_rank_labels(const int32_t* lab, int64_t n, const int64_t* rank, int32_t* out,
                              unsigned long long* count) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int32_t r = (int32_t)rank[lab[v]];
        out[v] = r;
        atomicAdd(&count[r], 1ull);
    }
}

__global__ void k_label_values(const int64_t* flag, const int64_t* rank, int64_t maxlab,
                               int32_t* values) {
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < maxlab;
         l += (int64_t)gridDim.x * blockDim.x)
        if (flag[l]) values[rank[l]] = (int32_t)l;
}

__global__ void k_degree(const int32_t* src, const int32_t* dst, int64_t m,
                         unsigned long long* deg, unsigned long long* loops) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = src[e], b = dst[e];
        if (a == b) { atomicAdd(loops, 1ull); continue; }
        atomicAdd(&deg[a], 1ull);
        atomicAdd(&deg[b], 1ull);
    }
}

__global__ void k_scatter(const int32_t* src, const int32_t* dst, int64_t m,
                          unsigned long long* cursor, int32_t* col) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = src[e], b = dst[e];
        if (a == b) continue;
        col[atomicAdd(&cursor[a], 1ull)] = b;
        col[atomicAdd(&cursor[b], 1ull)] = a;
    }
}

// Ascending bitonic sort of keys[0..P) (P a power of two) by one block.
__device__ void bitonic_block(int32_t* keys, int P) {
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                int ixj = i ^ j;
                if (ixj > i) {
                    int32_t a = keys[i], b = keys[ixj];
                    bool up = (i & k) == 0;
                    if ((a > b) == up) { keys[i] = b; keys[ixj] = a; }
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// One block per row; rows longer than SMALL_ROW go through `tmp`, which has
// room for 2*len entries at offset 2*off[row] (>= next power of two).
__global__ __launch_bounds__(T) void k_sort_rows(const int64_t* off, int64_t n, int32_t* col,
                                                 int32_t* tmp) {
    __shared__ int32_t s[SMALL_ROW];
    for (int64_t v = blockIdx.x; v < n; v += gridDim.x) {
        const int64_t b = off[v];
        const int len = (int)(off[v + 1] - b);
        if (len <= 1) continue;
        const int P = next_pow2(len);
        int32_t* keys = (len <= SMALL_ROW) ? s : tmp + 2 * b;
        for (int i = threadIdx.x; i < P; i += blockDim.x) keys[i] = i < len ? col[b + i] : INT_MAX;
        __syncthreads();
        bitonic_block(keys, P);
        for (int i = threadIdx.x; i < len; i += blockDim.x) col[b + i] = keys[i];
        __syncthreads();
    }
}

// keep[e] = 1 for the first copy of each neighbour in a row
__global__ void k_first_copy(const int64_t* off, int64_t n, const int32_t* col, int64_t* keep) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t e = off[v]; e < off[v + 1]; ++e)
            keep[e] = (e == off[v] || col[e] != col[e - 1]) ? 1 : 0;
    }
}

// pos is the exclusive scan of keep over all raw entries, so the kept
// entries before row v number pos[off[v]] (or all of them past the end)
__global__ void k_compact(const int64_t* off, int64_t n, const int32_t* col, const int64_t* pos,
                          const int64_t* keep, int64_t raw, int64_t total, int32_t* row,
                          int32_t* out) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = off[v];
        row[v] = (int32_t)(b < raw ? pos[b] : total);
        if (v == n) continue;
        for (int64_t i = b; i < off[v + 1]; ++i)
            if (keep[i]) out[pos[i]] = col[i];
    }
}

}  // namespace

void build_graph(fsm_graph* g, int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                 const int32_t* labels) {
    hipStream_t st = stream();
    int32_t maxlab = 0;
    for (int64_t v = 0; v < n; ++v) maxlab = labels[v] > maxlab ? labels[v] : maxlab;
    g->n = n;

    // labels -> dense ranks
    DBuf<int32_t> dlab((size_t)n);
    to_device(dlab.p, labels, (size_t)n);
    const int64_t nl = (int64_t)maxlab + 1;
    DBuf<int64_t> flag((size_t)nl), rank((size_t)nl);
    flag.zero();
    k_mark_labels<<<grid_for(n, T), T, 0, st>>>(dlab.p, n, flag.p);
    FSM_LAUNCH_CHECK();
    int64_t L = scan_exclusive(flag.p, rank.p, nl);
    g->num_labels = (int32_t)L;
    g->lab.alloc((size_t)n);
    DBuf<unsigned long long> lcount((size_t)L);
    lcount.zero();
    k_rank_labels<<<grid_for(n, T), T, 0, st>>>(dlab.p, n, rank.p, g->lab.p, lcount.p);
    FSM_LAUNCH_CHECK();
    DBuf<int32_t> lval((size_t)L);
    k_label_values<<<grid_for(nl, T), T, 0, st>>>(flag.p, rank.p, nl, lval.p);
    FSM_LAUNCH_CHECK();
    to_host(g->label_value, lval.p, (size_t)L);
    std::vector<unsigned long long> lc;
    to_host(lc, lcount.p, (size_t)L);
    g->label_count.assign(lc.begin(), lc.end());

    // degrees, offsets, scatter
    DBuf<int32_t> dsrc((size_t)(m > 0 ? m : 1)), ddst((size_t)(m > 0 ? m : 1));
    to_device(dsrc.p, src, (size_t)m);
    to_device(ddst.p, dst, (size_t)m);
    DBuf<unsigned long long> deg((size_t)n + 1), loops(1);
    deg.zero();
    loops.zero();
    if (m > 0) {
        k_degree<<<grid_for(m, T), T, 0, st>>>(dsrc.p, ddst.p, m, deg.p, loops.p);
        FSM_LAUNCH_CHECK();
    }
    DBuf<int64_t> off((size_t)n + 1);
    int64_t raw = scan_exclusive(reinterpret_cast<int64_t*>(deg.p), off.p, n + 1);
    g->dropped_loops = (int64_t)scalar_to_host(loops.p);
    if (raw > (int64_t)INT32_MAX)
        fail(FSM_EUNSUPPORTED, "graph has %lld directed entries; at most 2^31-1 supported",
             (long long)raw);
    DBuf<int32_t> col((size_t)raw);
    if (raw > 0) {
        FSM_HIP(hipMemcpyAsync(deg.p, off.p, sizeof(int64_t) * (size_t)(n + 1),
                               hipMemcpyDeviceToDevice, st));
        k_scatter<<<grid_for(m, T), T, 0, st>>>(dsrc.p, ddst.p, m, deg.p, col.p);
        FSM_LAUNCH_CHECK();
        DBuf<int32_t> tmp((size_t)(2 * raw));
        k_sort_rows<<<grid_for(n, 1, 1u << 16), T, 0, st>>>(off.p, n, col.p, tmp.p);
        FSM_LAUNCH_CHECK();
    }

    // drop repeated neighbours
    DBuf<int64_t> keep((size_t)raw), pos((size_t)raw);
    int64_t total = 0;
    if (raw > 0) {
        k_first_copy<<<grid_for(n, T), T, 0, st>>>(off.p, n, col.p, keep.p);
        FSM_LAUNCH_CHECK();
        total = scan_exclusive(keep.p, pos.p, raw);
    }
    g->row.alloc((size_t)n + 1);
    g->col.alloc((size_t)(total > 0 ? total : 1));
    if (raw > 0) {
        k_compact<<<grid_for(n + 1, T), T, 0, st>>>(off.p, n, col.p, pos.p, keep.p, raw, total,
                                                    g->row.p, g->col.p);
        FSM_LAUNCH_CHECK();
    } else {
        g->row.zero();
    }
    FSM_HIP(hipStreamSynchronize(st));
    g->nnz = total;
    g->dropped_dups = (raw - total) / 2;
}

}  // namespace fsm
