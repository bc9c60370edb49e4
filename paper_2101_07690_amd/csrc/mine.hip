// mine.hip -- the level-by-level two-vertex-exploration miner.
//
// Levels (Section 3 workflow):
//   size 2  labelled edges over frequent labels            (Step 2)
//   size 3  wedges and triangles over frequent edges       (Steps 1-2)
//   size n  join of size-(n-2) embeddings of frequent patterns with size-3
//           pieces on one common vertex (Section 4.1, Theorem 1), over CSR
//           adjacency restricted to frequent labelled edges  (Step 3)
// Every produced subgraph gets a quick pattern (QP, Section 4.4); a QP table
// maps it to a canonical pattern and to the automorphism orbit of each of its
// positions; MNI domains (Section 2.2) are bitmaps per (pattern, orbit);
// patterns below t are dropped and, when a later join needs them, the
// embeddings of frequent patterns are compacted by count / scan / fill
// (Step 4).
//
// Recording a subgraph (any level), with no canonical form in the loop:
//   QP key  -> open-addressing table slot s (insert by CAS; the inserting
//              lane also stores the QP's ordered labels and adjacency)
//   bits    -> for each position p: set bit rank(v_p) in the bitmap of
//              (QP slot s, position p); rank(v) numbers the vertices of v's
//              label (a position only ever holds vertices of its label);
//              read first, atomicOr only when unset
// After the pass, one thread per QP computes its canonical form (Section
// 4.4: one isomorphism computation per quick-pattern group), the QP's
// position bitmaps are OR-ed into the bitmaps of (pattern, orbit of the
// position), and the MNI support is the smallest orbit popcount.  The QP
// value word then holds VALID | FREQ | 3-bit orbit slot per position.
#include <algorithm>
#include <array>
#include <map>
#include <memory>
#include <atomic>
#include <deque>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "common.h"
#include "internal.h"
#include "model.h"

// FSM_TRACE=1 in the environment: one line per domain pass and join level on
// stderr (progress of long calls).
static bool fsm_trace() {
    static const bool on = [] {
        const char* e = std::getenv("FSM_TRACE");
        return e && *e && *e != '0';
    }();
    return on;
}

namespace fsm {
namespace {

constexpr int TPB = 256;
constexpr uint64_t VALID = 1ull << 63;
constexpr uint64_t FREQ = 1ull << 62;
constexpr uint64_t REGION_MASK = (1ull << 41) - 1;
constexpr int JOIN_CHUNK = 4;   // work items fetched per queue access
// buckets of one vertex's neighbour table: the join addresses a bucket by a
// 32-bit byte offset from the table's base
constexpr int64_t NB_MAX = 1ll << 29;

enum : uint32_t { OVF_QP = 1, OVF_CODE = 2, ERR_MISSING = 8, ERR_FILL = 16, ERR_BATCH = 32,
                  ERR_GRAPH = 64 };
enum { MODE_DOMAIN = 0, MODE_COUNT = 1, MODE_FILL = 2 };
enum { PIECE_KC = 0, PIECE_KL = 1, PIECE_TR = 2 };   // k-centre wedge, k-leaf wedge, triangle

struct QPTab {
    uint64_t* kv;      // 2 words per slot: key, value
    uint64_t mask;     // capacity - 1
    uint64_t* adj;     // packed adjacency of the QP's ordered subgraph
    uint64_t* lab;     // packed labels of the QP's ordered subgraph
    int32_t* pat;      // pattern-table slot
    unsigned* count;   // occupied slots
};

struct CodeTab {
    uint64_t* kv;      // 2 words per slot: canonical code, bitmap region + 1
    uint64_t mask;
    uint64_t* info;    // VALID | 3-bit orbit representative per canonical position
    int64_t* sup;      // MNI support after the reduction
    unsigned* count;
};

struct Pool {
    uint32_t* words;           // table slot s owns bitmaps s*n .. s*n+n-1
    const int32_t* lrank;      // rank of each vertex among its label's vertices
    uint32_t W;                // words per bitmap in this pass
    int32_t rbase;             // this pass covers ranks rbase .. rbase + 32 W - 1
    const int32_t* porb = nullptr;   // set: (slot s, position p) owns bitmap porb[s*n+p]
                                     // (its pattern's orbit; -1: none)
    unsigned long long* qcnt = nullptr;   // set: subgraphs recorded per QP slot
};

struct Rec {
    QPTab q;
    CodeTab c;
    Pool pool;
    uint32_t* flags;
    int n;             // subgraph size of this level
    unsigned* item_qps = nullptr;   // join levels, when recording: new QPs per work item
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ int64_t wave_excl(int64_t v, int lane) {
    int64_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    return inc - v;
}

// Inserting tables hold at most half their slots: past that load (or after
// PROBE_LIMIT probes) an insert gives up and raises the overflow flag, and
// the host reruns the pass with a larger table.  Lookups are never cut short.
constexpr uint64_t PROBE_LIMIT = 4096;

__device__ __forceinline__ bool over_load(const unsigned* count, uint64_t mask) {
    const unsigned c = __hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (uint64_t)c * 2 > mask;
}

// Find `key`; insert it when `insert` (CAS on an empty slot).  Returns the
// slot, or -1 when absent (lookup) or the insert gave up (flag raised).
__device__ int64_t ht_probe(uint64_t* kv, uint64_t mask, uint64_t key, bool insert,
                            unsigned* count, uint32_t* flags, uint32_t bit) {
    uint64_t h = mix64(key) & mask;
    const uint64_t limit = insert ? (mask < PROBE_LIMIT ? mask : PROBE_LIMIT) : mask;
    for (uint64_t i = 0; i <= limit; ++i) {
        uint64_t cur = kv[2 * h];
        if (cur == key) return (int64_t)h;
        if (cur == EMPTY_KEY) {
            if (!insert) return -1;
            if (over_load(count, mask)) break;
            unsigned long long prev =
                atomicCAS((unsigned long long*)&kv[2 * h], (unsigned long long)EMPTY_KEY,
                          (unsigned long long)key);
            if (prev == EMPTY_KEY) {
                unsigned c = atomicAdd(count, 1u);
                if ((uint64_t)c * 2 > mask) atomicOr(flags, bit);   // keep load <= 1/2
                return (int64_t)h;
            }
            if (prev == key) return (int64_t)h;
        }
        h = (h + 1) & mask;
    }
    atomicOr(flags, bit);
    return -1;
}

// QP slot of `key`, inserting it when new; the inserting lane stores the
// ordered subgraph (labels L, adjacency A) for the canonical pass.
__device__ __forceinline__ int64_t qp_slot(const Rec& R, uint64_t key, uint64_t L, uint64_t A) {
    uint64_t h = mix64(key) & R.q.mask;
    const uint64_t limit = R.q.mask < PROBE_LIMIT ? R.q.mask : PROBE_LIMIT;
    for (uint64_t i = 0; i <= limit; ++i) {
        const uint64_t cur = R.q.kv[2 * h];
        if (cur == key) return (int64_t)h;
        if (cur == EMPTY_KEY) {
            if (over_load(R.q.count, R.q.mask)) break;
            const unsigned long long prev =
                atomicCAS((unsigned long long*)&R.q.kv[2 * h], (unsigned long long)EMPTY_KEY,
                          (unsigned long long)key);
            if (prev == EMPTY_KEY) {
                R.q.adj[h] = A;
                R.q.lab[h] = L;
                // join keys: parent slot << 35 | position << 32 | ...
                if (R.item_qps)
                    atomicAdd(&R.item_qps[(key >> 35) * (uint64_t)(R.n - 2) + ((key >> 32) & 7u)], 1u);
                const unsigned c = atomicAdd(R.q.count, 1u);
                if ((uint64_t)c * 2 > R.q.mask) atomicOr(R.flags, OVF_QP);
                return (int64_t)h;
            }
            if (prev == key) return (int64_t)h;
        }
        h = (h + 1) & R.q.mask;
    }
    atomicOr(R.flags, OVF_QP);
    return -1;
}

// Size 5: the parent's own triple {k, b1, b2} is connected and leaves the
// connected piece {k, u, w} when k is shared, so it is a valid split of the
// child; the accepted split is the lexicographically smallest, hence a child
// can only be kept when sorted(k, u, w) < sorted(parent) (exact filter).
__device__ __forceinline__ void sort3(int32_t a, int32_t b, int32_t c, int32_t& x, int32_t& y,
                                      int32_t& z) {
    x = min(a, min(b, c));
    z = max(a, max(b, c));
    y = a ^ b ^ c ^ x ^ z;
}

__device__ __forceinline__ bool lex_less3(int32_t a0, int32_t a1, int32_t a2, int32_t b0,
                                          int32_t b1, int32_t b2) {
    return a0 < b0 || (a0 == b0 && (a1 < b1 || (a1 == b1 && a2 < b2)));
}

// bit r of the bitmap at `bm`: read first, atomicOr only when unset
// Device buffers live in global memory; reading them through pointers of
// that address space lets the compiler use global (not flat) loads and
// atomics, which do not hold up the LDS reads of the same wave.
#define FSM_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ FSM_GLOBAL T* gmem(T* p) {
    return (FSM_GLOBAL T*)p;
}

// Read-only for the whole kernel: a wave-uniform address loads through the
// scalar unit into SGPRs.
#define FSM_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const FSM_CONST T* cmem(const T* p) {
    return (const FSM_CONST T*)p;
}

__device__ __forceinline__ void set_bit(uint32_t* bm, int32_t r) {
    FSM_GLOBAL uint32_t* w = gmem(bm) + (r >> 5);
    const uint32_t bit = 1u << (r & 31);
    if (!(*w & bit)) __hip_atomic_fetch_or(w, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Domain passes cover the ranks in slices: rank r is set when it falls in
// [rbase, rbase + 32 W).
__device__ __forceinline__ void set_bit_in(uint32_t* bm, int32_t r, int32_t rbase, uint32_t W) {
    const uint32_t x = (uint32_t)(r - rbase);
    if (x < 32u * W) set_bit(bm, (int32_t)x);
}

// Bitmap of (QP slot s, position p) in this pass's pool, or null.
__device__ __forceinline__ uint32_t* bitmap_at(const Pool& P, uint64_t s, int n, int p) {
    if (P.porb) {
        const int32_t x = P.porb[s * n + p];
        return x < 0 ? nullptr : P.words + (uint64_t)x * P.W;
    }
    return P.words + (s * n + p) * P.W;
}

// Domain pass: record one subgraph; returns its QP slot (or -1).
template <int N>
__device__ __forceinline__ int64_t record(const Rec& R, uint64_t key, uint64_t L, uint64_t A,
                                          const int32_t (&v)[N]) {
    const int64_t s = qp_slot(R, key, L, A);
    if (s < 0) return -1;
    if (R.pool.qcnt) atomicAdd(&R.pool.qcnt[s], 1ull);
#pragma unroll
    for (int p = 0; p < N; ++p)
        if (uint32_t* bm = bitmap_at(R.pool, (uint64_t)s, N, p))
            set_bit_in(bm, R.pool.lrank[v[p]], R.pool.rbase, R.pool.W);
    return s;
}

// Count / fill passes: QP slot of a subgraph of a frequent pattern, else -1.
__device__ __forceinline__ int64_t frequent_slot(const Rec& R, uint64_t key) {
    int64_t s = ht_probe(R.q.kv, R.q.mask, key, false, nullptr, R.flags, ERR_MISSING);
    if (s < 0) {
        atomicOr(R.flags, ERR_MISSING);
        return -1;
    }
    return (R.q.kv[2 * s + 1] & FREQ) ? s : -1;
}

// Adjacency test through per-vertex neighbour tables: vertex b owns a
// two-choice cuckoo table of its G_f neighbours, nb(b) = pow2 >= 2 deg(b)
// one-slot buckets (load <= 1/2) at tab[off[b] .. off[b+1]), empty slots
// -1.  A neighbour x sits in bucket h1(x) or h2(x), so a test reads two
// 4-byte words and makes two compares -- no probe loop, the same work on
// every lane -- and a wave testing one vertex b for many x stays within
// b's table.
struct NbrHash {
    const uint32_t* off;   // n + 1, in buckets
    const int32_t* tab;
};

__host__ __device__ __forceinline__ uint32_t nbr_hash(int32_t x) {
    uint32_t h = (uint32_t)x * 0x9E3779B1u;
    return h ^ (h >> 15);
}

__host__ __device__ __forceinline__ uint32_t nbr_hash2(int32_t x) {
    uint32_t h = ((uint32_t)x ^ 0x5bd1e995u) * 0x85EBCA77u;
    return h ^ (h >> 13);
}

// b's table holds x (nb = its bucket count, o its first bucket)
__device__ __forceinline__ bool nbr_has(const int32_t* tab, uint32_t o, uint32_t nb, int32_t x) {
    const FSM_GLOBAL int32_t* t = gmem(tab) + o;
    return t[nbr_hash(x) & (nb - 1)] == x || t[nbr_hash2(x) & (nb - 1)] == x;
}

__device__ __forceinline__ bool has_edge(const NbrHash& H, int32_t b, int32_t x) {
    const uint32_t o = gmem(H.off)[b], nb = gmem(H.off)[b + 1] - o;
    return nb != 0 && nbr_has(H.tab, o, nb, x);
}

// Vertex-induced mode: graph edges between frequent-label vertices whose
// labelled edge is infrequent (not in G_f), in tables of the same layout
// (off null when there are none).  Such an edge inside a vertex set makes
// its induced pattern infrequent, so the set is never a subgraph to keep.
__device__ __forceinline__ bool blocked(const NbrHash& X, int32_t b, int32_t x) {
    return X.off != nullptr && has_edge(X, b, x);
}

// wave index, kept in a scalar register so wave-uniform work stays scalar
__device__ __forceinline__ int wave_id_global() {
    return __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (TPB / 64) + (threadIdx.x >> 6)));
}

// ------------------------------------------------------------- setup kernels

__global__ void k_init_table(uint64_t* kv, uint64_t slots) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < slots;
         s += (uint64_t)gridDim.x * blockDim.x) {
        kv[2 * s] = EMPTY_KEY;
        kv[2 * s + 1] = 0;
    }
}

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// rank of each vertex among the vertices of its graph with its frequent
// label (any order)
__global__ void k_label_rank(const int32_t* vf, const int32_t* vg, int F, int64_t n,
                             unsigned* cnt, int32_t* rank) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int l = vf[v];
        rank[v] = l >= 0 ? (int32_t)atomicAdd(&cnt[(size_t)vg[v] * F + l], 1u) : 0;
    }
}

__global__ void k_vinfo(const int32_t* vf, const int32_t* rank, int64_t n, uint32_t* vinfo) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        vinfo[v] = vf[v] >= 0 ? ((uint32_t)vf[v] << 26 | (uint32_t)rank[v]) : 0xffffffffu;
}

__global__ void k_vertex_flabel(const int32_t* lab, const int32_t* vg, int NL, int64_t n,
                                const int32_t* fmap, int32_t* vf) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        vf[v] = fmap[(size_t)vg[v] * NL + lab[v]];
}

// frequent-edge subgraph G_f: keep (v, w) when both labels are frequent and
// the labelled edge is frequent (want = 1), or infrequent (want = 0: the
// edges a vertex-induced subgraph must not contain)
__global__ void k_gf_count(const int32_t* row, const int32_t* col, const int32_t* vf,
                           const int32_t* vg, int64_t n, const uint8_t* freq2, int F, int want,
                           int64_t* cnt) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = 0;
        int a = vf[v];
        const uint8_t* f2 = freq2 + (size_t)vg[v] * F * F;
        if (a >= 0)
            for (int32_t e = row[v]; e < row[v + 1]; ++e) {
                int b = vf[col[e]];
                if (b >= 0 && (f2[a * F + b] != 0) == (want != 0)) ++c;
            }
        cnt[v] = c;
    }
}

__global__ void k_gf_fill(const int32_t* row, const int32_t* col, const int32_t* vf,
                          const int32_t* vg, int64_t n, const uint8_t* freq2, int F, int want,
                          const int64_t* off, int64_t total, int32_t* frow, int32_t* fcol) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (v == n) { frow[n] = (int32_t)total; continue; }
        int64_t o = off[v];
        frow[v] = (int32_t)o;
        int a = vf[v];
        if (a < 0) continue;
        const uint8_t* f2 = freq2 + (size_t)vg[v] * F * F;
        for (int32_t e = row[v]; e < row[v + 1]; ++e) {
            int32_t w = col[e];
            int b = vf[w];
            if (b >= 0 && (f2[a * F + b] != 0) == (want != 0)) fcol[o++] = w;
        }
    }
}

// Buckets of each vertex's neighbour table: the smallest power of two >=
// 2 deg (one slot each), times 2^grow[v] after failed builds; 0 for an
// isolated vertex.
__global__ void k_nbr_sizes(const int32_t* row, int64_t n, const uint8_t* grow, int64_t* nb,
                            unsigned* big) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = row[v + 1] - row[v];
        int64_t c = 0;
        if (d > 0) {
            c = 1;
            while (c < 2 * d) c <<= 1;
            c <<= grow[v];
        }
        if (c > NB_MAX) atomicOr(big, 1u);
        nb[v] = c;
    }
}

// One thread per vertex: cuckoo insertion of its neighbours (a displaced
// key moves to its other bucket); a vertex whose chain exceeds the bound is
// marked in `failed` and rebuilt with twice the buckets.
constexpr int CUCKOO_STEPS = 512;

__global__ void k_nbr_fill(const int32_t* row, const int32_t* col, int64_t n, const int64_t* off,
                           int64_t total, uint32_t* off32, int32_t* tab, uint8_t* failed,
                           unsigned* nfailed) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (v == n) { off32[n] = (uint32_t)total; continue; }
        const int64_t o = off[v];
        off32[v] = (uint32_t)o;
        const uint32_t nb = (uint32_t)((v + 1 < n ? off[v + 1] : total) - o);
        int32_t* t = tab + o;
        for (uint32_t b = 0; b < nb; ++b) t[b] = -1;
        bool ok = true;
        for (int32_t e = row[v]; e < row[v + 1] && ok; ++e) {
            int32_t x = col[e];
            uint32_t b = nbr_hash(x) & (nb - 1);   // the bucket x is tried in first
            for (int step = 0;; ++step) {
                if (t[b] < 0) { t[b] = x; break; }
                const uint32_t h1 = nbr_hash(x) & (nb - 1), h2 = nbr_hash2(x) & (nb - 1);
                const uint32_t alt = h1 == b ? h2 : h1;
                if (t[alt] < 0) { t[alt] = x; break; }
                if (step >= CUCKOO_STEPS) { ok = false; break; }
                // x takes the slot of bucket alt; the key it displaces moves
                // on to its own other bucket
                const int32_t y = t[alt];
                t[alt] = x;
                x = y;
                const uint32_t y1 = nbr_hash(x) & (nb - 1), y2 = nbr_hash2(x) & (nb - 1);
                b = y1 == alt ? y2 : y1;
            }
        }
        if (!ok) {
            failed[v] = 1;
            atomicAdd(nfailed, 1u);
        }
    }
}

__global__ void k_grow_failed(const uint8_t* failed, int64_t n, uint8_t* grow) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        if (failed[v]) grow[v] += 1;
}

// pieces rooted at k: centre pairs C(d,2) plus one slot per (u in N(k),
// w in N(u)) for k-leaf wedges; leafoff = per-row prefix of neighbour degrees
__global__ void k_pieces(const int32_t* row, const int32_t* col, int64_t n, int64_t* npieces,
                         int32_t* leafoff) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = row[k + 1] - row[k];
        int64_t s = 0;
        for (int32_t e = row[k]; e < row[k + 1]; ++e) {
            leafoff[e] = (int32_t)s;
            int32_t u = col[e];
            s += row[u + 1] - row[u];
        }
        npieces[k] = d * (d - 1) / 2 + s;
    }
}

// --------------------------------------------------------------- level 2

struct L2Args {
    const int32_t* row;
    const int32_t* col;
    const int32_t* vf;
    const int32_t* vg;       // graph of each vertex (a batch is one disjoint union)
    int64_t n;
    Rec R;
    unsigned long long* emitted;
    int64_t* counts;
    const int64_t* offsets;
    int32_t* out;
    int64_t out_rows;
};

// One wave per vertex u; lanes over neighbours w > u with a frequent label.
// Stored order (u, w), u < w; QP = the ordered label pair.
template <int MODE>
__global__ __launch_bounds__(TPB) void k_level2(L2Args a) {
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (TPB / 64);
    unsigned long long emit = 0;
    for (int64_t u = wave_id_global(); u < a.n; u += nwaves) {
        const int lu = a.vf[u];
        if (lu < 0) continue;
        const uint64_t gid = (uint64_t)a.vg[u];
        const int32_t rb = a.row[u], re = a.row[u + 1];
        int64_t base = (MODE == MODE_FILL) ? a.offsets[u] : 0, total = 0;
        for (int32_t e0 = rb; e0 < re; e0 += 64) {
            const int32_t e = e0 + lane;
            int32_t w = -1;
            int lw = -1;
            if (e < re) {
                w = a.col[e];
                lw = w > u ? a.vf[w] : -1;
            }
            int64_t s = -1;
            if (lw >= 0) {
                uint64_t key = gid << 12 | (uint64_t)lu << 6 | (uint64_t)lw;
                if (MODE == MODE_DOMAIN) {
                    int32_t v[2] = {(int32_t)u, w};
                    uint64_t L = (uint64_t)lu | (uint64_t)lw << 6 | gid << 48;
                    record<2>(a.R, key, L, add_edge(0, 0, 1), v);
                    ++emit;
                } else {
                    s = frequent_slot(a.R, key);
                }
            }
            if (MODE != MODE_DOMAIN) {
                int64_t c = s >= 0 ? 1 : 0;
                int64_t ex = wave_excl(c, lane);
                if (MODE == MODE_FILL && c) {
                    int64_t r = base + total + ex;
                    if (r < a.out_rows) {
                        int32_t* o = a.out + r * 3;
                        o[0] = (int32_t)u; o[1] = w; o[2] = (int32_t)s;
                    } else {
                        atomicOr(a.R.flags, ERR_FILL);
                    }
                }
                total += wave_sum(c);
            }
        }
        if (MODE == MODE_COUNT && lane == 0) a.counts[u] = total;
    }
    if (MODE == MODE_DOMAIN) {
        int64_t t = wave_sum((int64_t)emit);
        if (lane == 0 && t) atomicAdd(a.emitted, (unsigned long long)t);
    }
}

// --------------------------------------------------------------- level 3

// ------------------------------------------------------------- sampling
//
// Subgraph sampling (Section 5).  Every member of a sampled group gets a
// counter-based hash: the splitmix64 finalizer chained over (seed ^ tag, a,
// b).  Rate sampling keeps a member when its hash is below rate * 2^64;
// fixed-size sampling keeps the members whose hash is at most the group's
// threshold, the cap-th smallest hash of the group (~0 when the group has at
// most cap members), i.e. a uniform sample of exactly min(size, cap).
//   rate, joining vertex k  tag n << 56,                 a = k, b = {u, w}
//   ST piece of type t      tag n << 56 | (t + 1) << 48, a = k, b = {u, w}
//                           (k-centre wedge, triangle) or u << 32 | w
//                           (k-leaf wedge k-u-w)
//   ST edge of a size-n join  tag n << 56 | 4 << 48,     a = k, b = other end
//                           (two-vertex n = 4; every single-vertex join)
//   matching                tag 3 << 56 | (s + 1) << 48, a = credited vertex
//                           (wedge centre, s = 0; smallest triangle vertex,
//                           s = 1), b = the other two
// where {u, w} = min << 32 | max.

struct Sampling {
    uint64_t seed = 0;
    const uint64_t* mthr = nullptr;   // matching: per credited vertex
    const uint64_t* kthr = nullptr;   // a join's key groups: per joining vertex
    const uint64_t* ethr = nullptr;   // size-4 join: edge groups per joining vertex
};

__device__ __forceinline__ uint64_t unit_hash(uint64_t seed, uint64_t tag, int32_t a, uint64_t b) {
    uint64_t h = mix64(seed ^ tag);
    h = mix64(h ^ (uint64_t)(uint32_t)a);
    return mix64(h ^ b);
}

__device__ __forceinline__ uint64_t pair_key(int32_t x, int32_t y) {
    return (uint64_t)(uint32_t)min(x, y) << 32 | (uint32_t)max(x, y);
}

// Rate-sampling hash of the size-3 piece {k, u, w} joined at level n.
__device__ __forceinline__ uint64_t sample_hash(uint64_t seed, int n, int32_t k, int32_t u,
                                                int32_t w) {
    return unit_hash(seed, (uint64_t)n << 56, k, pair_key(u, w));
}

__device__ __forceinline__ uint64_t piece_hash(uint64_t seed, int n, int t, int32_t k, int32_t u,
                                               int32_t w) {
    const uint64_t b = t == PIECE_KL ? ((uint64_t)(uint32_t)u << 32 | (uint32_t)w) : pair_key(u, w);
    return unit_hash(seed, (uint64_t)n << 56 | (uint64_t)(t + 1) << 48, k, b);
}

__device__ __forceinline__ uint64_t edge_hash(uint64_t seed, int n, int32_t k, int32_t o) {
    return unit_hash(seed, (uint64_t)n << 56 | 4ull << 48, k, (uint64_t)(uint32_t)o);
}

__device__ __forceinline__ uint64_t match_hash(uint64_t seed, int s, int32_t c, int32_t x,
                                               int32_t y) {
    return unit_hash(seed, 3ull << 56 | (uint64_t)(s + 1) << 48, c, pair_key(x, y));
}

// The size-3 subgraphs a neighbour pair u < w of centre c stands for in
// matching: the wedge (c; u, w), and the triangle when c < u and u ~ w
// (credited to its smallest vertex).  Vertex-induced: the wedge only when
// u !~ w, nothing when u, w are joined by an edge outside G_f.
__device__ __forceinline__ void level3_units(const NbrHash& nh, const NbrHash& xh, int induced,
                                             int32_t c, int32_t u, int32_t w, bool& wedge,
                                             bool& tri) {
    const bool uw = (induced || c < u) && has_edge(nh, u, w);
    tri = c < u && uw;
    wedge = !(induced && (uw || blocked(xh, u, w)));
}

// Piece types (bit PIECE_*) that survive matching sampling: each is the
// matched size-3 subgraph it stands for -- the wedge centred at k (k-centre),
// at u (k-leaf k-u-w), the triangle credited to its smallest vertex.
__device__ __forceinline__ uint32_t matched_types(const Sampling& s, uint32_t types, int32_t k,
                                                  int32_t u, int32_t w) {
    if (!s.mthr || !types) return types;
    if (((types >> PIECE_KC) & 1u) && match_hash(s.seed, 0, k, u, w) > s.mthr[k])
        types &= ~(1u << PIECE_KC);
    if (((types >> PIECE_KL) & 1u) && match_hash(s.seed, 0, u, k, w) > s.mthr[u])
        types &= ~(1u << PIECE_KL);
    if ((types >> PIECE_TR) & 1u) {
        const int32_t c = min(k, min(u, w));
        const int32_t x = c == k ? u : k, y = c == w ? u : w;
        if (match_hash(s.seed, 1, c, x, y) > s.mthr[c]) types &= ~(1u << PIECE_TR);
    }
    return types;
}

// Piece types kept by k's key group at the size-n join under ST sampling.
__device__ __forceinline__ uint32_t st_types(const Sampling& s, int n, uint32_t types, int32_t k,
                                             int32_t u, int32_t w) {
    if (!s.kthr || !types) return types;
    const uint64_t thr = s.kthr[k];
#pragma unroll
    for (int t = 0; t < 3; ++t)
        if (((types >> t) & 1u) && piece_hash(s.seed, n, t, k, u, w) > thr) types &= ~(1u << t);
    return types;
}

struct L3Args {
    const int32_t* row;    // G_f
    const int32_t* col;
    const int32_t* vf;
    const int32_t* vg;
    int64_t n;
    NbrHash nh;
    Rec R;
    unsigned long long* emitted;
    int64_t* counts;
    const int64_t* offsets;
    int32_t* out;
    int64_t out_rows;
    int induced = 0;       // vertex-induced: a wedge only when u !~ w
    NbrHash xh{nullptr, nullptr};   // vertex-induced: edges outside G_f
    Sampling smp{};        // matching sampling (mthr) when set
};

__device__ __forceinline__ void decode_pair(int64_t r, int32_t* a, int32_t* b) {
    // pairs (a<b) listed by b, then a: index = b(b-1)/2 + a
    int64_t bb = (int64_t)((1.0f + sqrtf(1.0f + 8.0f * (float)r)) * 0.5f);
    while (bb * (bb - 1) / 2 > r) --bb;
    while ((bb + 1) * bb / 2 <= r) ++bb;
    *b = (int32_t)bb;
    *a = (int32_t)(r - bb * (bb - 1) / 2);
}

// Piece q of joining vertex k (rk = row[k], dk = deg(k), ncen = C(dk,2)):
// the k-centre pairs {u < w} of N(k) first, then the k-leaf paths k-u-w
// (w in N(u)); returns true for a k-centre piece.
__device__ __forceinline__ bool piece_at(const int32_t* row, const int32_t* col,
                                         const int32_t* leafoff, int32_t rk, int32_t dk,
                                         int64_t ncen, int64_t q, int32_t& u, int32_t& w) {
    if (q < ncen) {
        int32_t ia, ib;
        decode_pair(q, &ia, &ib);
        u = col[rk + ia];
        w = col[rk + ib];
        return true;
    }
    const int32_t rr = (int32_t)(q - ncen);
    int32_t lo = 0, hi = dk - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (leafoff[rk + mid] <= rr) lo = mid; else hi = mid - 1;
    }
    u = col[rk + lo];
    w = col[row[u] + (rr - leafoff[rk + lo])];
    return false;
}

// Size-5 piece lists: every vertex's pieces as key (min(u,w) << 32 |
// max(u,w)) and code (bit 0: k-leaf, bit 1: u is the larger id), at
// poff[k] + q; one wavefront per vertex.  Sorted by key afterwards.
__global__ void k_piece_fill(const int32_t* row, const int32_t* col, const int32_t* leafoff,
                             const int64_t* npieces, const int64_t* poff, int64_t n,
                             uint64_t* key, uint8_t* code) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t k = wave_id_global(); k < n; k += nw) {
        const int32_t rk = row[k], dk = row[k + 1] - rk;
        const int64_t ncen = (int64_t)dk * (dk - 1) / 2, Q = npieces[k];
        for (int64_t q = lane; q < Q; q += 64) {
            int32_t u, w;
            const bool centre = piece_at(row, col, leafoff, rk, dk, ncen, q, u, w);
            const int32_t lo = min(u, w), hi = max(u, w);
            key[poff[k] + q] = (uint64_t)(uint32_t)lo << 32 | (uint32_t)hi;
            code[poff[k] + q] = (uint8_t)((centre ? 0u : 1u) | (u > w ? 2u : 0u));
        }
    }
}

// One wave per centre c; lanes over neighbour pairs u < w.  Each pair is a
// wedge (c; u, w) stored (c, u, w); when c < u and u ~ w it is also the
// triangle stored (c, u, w) (each triangle once, at its smallest vertex).
// Vertex-induced mode drops the wedges whose ends are adjacent.  Matching
// sampling keeps the subgraphs credited to c whose hash is at most c's
// threshold.  QP = (type, labels in stored order).
template <int MODE>
__global__ __launch_bounds__(TPB) void k_level3(L3Args a) {
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (TPB / 64);
    unsigned long long emit = 0;
    for (int64_t c = wave_id_global(); c < a.n; c += nwaves) {
        const int32_t rb = a.row[c];
        const int64_t d = a.row[c + 1] - rb;
        const int64_t npairs = d * (d - 1) / 2;
        if (npairs == 0) {
            if (MODE == MODE_COUNT && lane == 0) a.counts[c] = 0;
            continue;
        }
        const int lc = a.vf[c];
        const uint64_t gid = (uint64_t)a.vg[c];
        int64_t base = (MODE == MODE_FILL) ? a.offsets[c] : 0, total = 0;
        for (int64_t r0 = 0; r0 < npairs; r0 += 64) {
            const int64_t r = r0 + lane;
            int32_t u = -1, w = -1;
            bool tri = false, wedge = false;
            int lu = 0, lw = 0;
            if (r < npairs) {
                int32_t ia, ib;
                decode_pair(r, &ia, &ib);
                u = a.col[rb + ia];
                w = a.col[rb + ib];
                lu = a.vf[u];
                lw = a.vf[w];
                level3_units(a.nh, a.xh, a.induced, (int32_t)c, u, w, wedge, tri);
                if (a.smp.mthr) {   // matching sampling: c's kept subgraphs
                    const uint64_t thr = a.smp.mthr[c];
                    if (wedge && match_hash(a.smp.seed, 0, (int32_t)c, u, w) > thr) wedge = false;
                    if (tri && match_hash(a.smp.seed, 1, (int32_t)c, u, w) > thr) tri = false;
                }
            }
            const uint64_t L = (uint64_t)lc | (uint64_t)lu << 6 | (uint64_t)lw << 12 | gid << 48;
            const uint64_t kw = gid << 19 | (uint64_t)lc << 12 | (uint64_t)lu << 6 | (uint64_t)lw;
            const uint64_t kt = (1ull << 18) | kw;
            const uint64_t Aw = add_edge(add_edge(0, 0, 1), 0, 2);
            const int32_t v[3] = {(int32_t)c, u, w};
            if (MODE == MODE_DOMAIN) {
                if (u >= 0) {
                    if (wedge) {
                        record<3>(a.R, kw, L, Aw, v);
                        ++emit;
                    }
                    if (tri) {
                        record<3>(a.R, kt, L, add_edge(Aw, 1, 2), v);
                        ++emit;
                    }
                }
            } else {
                int64_t sw = -1, stt = -1;
                if (u >= 0) {
                    if (wedge) sw = frequent_slot(a.R, kw);
                    if (tri) stt = frequent_slot(a.R, kt);
                }
                int64_t cnum = (sw >= 0 ? 1 : 0) + (stt >= 0 ? 1 : 0);
                int64_t ex = wave_excl(cnum, lane);
                if (MODE == MODE_FILL && cnum) {
                    int64_t r2 = base + total + ex;
                    if (r2 + cnum <= a.out_rows) {
                        int32_t* o = a.out + r2 * 4;
                        if (sw >= 0) {
                            o[0] = (int32_t)c; o[1] = u; o[2] = w; o[3] = (int32_t)sw;
                            o += 4;
                        }
                        if (stt >= 0) {
                            o[0] = (int32_t)c; o[1] = u; o[2] = w; o[3] = (int32_t)stt;
                        }
                    } else {
                        atomicOr(a.R.flags, ERR_FILL);
                    }
                }
                total += wave_sum(cnum);
            }
        }
        if (MODE == MODE_COUNT && lane == 0) a.counts[c] = total;
    }
    if (MODE == MODE_DOMAIN) {
        int64_t t = wave_sum((int64_t)emit);
        if (lane == 0 && t) atomicAdd(a.emitted, (unsigned long long)t);
    }
}

// ----------------------------------------------------------------- join

struct JoinArgs {
    const int32_t* row;      // G_f
    const int32_t* col;
    const int32_t* vf;
    const int64_t* npieces;
    const int32_t* leafoff;
    NbrHash nh;
    const int32_t* vg;
    const uint8_t* f3;       // per graph [2][F][F][F]: 0 wedge (centre first), 1 triangle
    int F;
    const int32_t* par;      // parents, rows of (M vertices, QP slot)
    const uint64_t* padj;    // parent level: packed adjacency per QP slot
    Rec R;
    unsigned long long* work_ctr;
    int64_t nwork;
    unsigned long long* emitted;
    unsigned long long* cands;
    unsigned long long* bytes;
    int prune;
    int sampled;
    uint64_t seed;
    uint64_t sample_thr;     // keep a piece when its hash is below this
    const uint64_t* item_thr;   // or, when set, below the threshold of its work item
    int induced;             // vertex-induced: the pieces' own edges are induced, C = E_c
    NbrHash xh;              // vertex-induced: edges outside G_f
    Sampling smp;            // matching and ST sampling thresholds
    int64_t* counts;
    const int64_t* offsets;
    int32_t* out;
    int64_t out_rows;
};

__device__ __forceinline__ bool f3_at(const uint8_t* f3, int F, int t, int a, int b, int c) {
    return gmem(f3)[((t * F + a) * F + b) * F + c] != 0;
}

// Size-3 subgraphs (bit PIECE_*) that the piece slot (k; u, w) holds among
// the stored ones: frequent size-3 patterns (f3), matched (Section 3), and
// in vertex-induced mode induced subgraphs of the input graph.  A k-centre
// slot holds the wedge u-k-w and, when u ~ w, the triangle; a k-leaf slot
// the wedge k-u-w.  `bytes` counts the adjacency probes.
template <class Count>
__device__ __forceinline__ uint32_t piece_types(const uint8_t* f3, int F, const NbrHash& nh,
                                                const NbrHash& xh, int induced, bool centre,
                                                int32_t k, int32_t u, int32_t w, int lk, int lu,
                                                int lw, Count& bytes) {
    uint32_t types = 0;
    if (centre) {
        const bool fw = f3_at(f3, F, 0, lk, lu, lw);
        const bool ft = f3_at(f3, F, 1, lk, lu, lw);
        bool uw = false;
        if (ft || (induced && fw)) {
            bytes += 8;
            uw = has_edge(nh, u, w);
        }
        if (fw && !(induced && (uw || blocked(xh, u, w)))) types |= 1u << PIECE_KC;
        if (ft && uw) types |= 1u << PIECE_TR;
    } else if (f3_at(f3, F, 0, lu, lk, lw)) {
        // vertex-induced: k !~ w (else it is the triangle)
        if (!induced || (!has_edge(nh, k, w) && !blocked(xh, k, w))) types |= 1u << PIECE_KL;
    }
    return types;
}

// All children of one (parent, position, piece-vertex pair) candidate.
// PHASE 0: domain pass (record) or count pass (count); PHASE 1: fill pass,
// writing rows from `dst`.  Returns the number of children accepted.
template <int N, int MODE, int PHASE>
__device__ int children(const JoinArgs& a, const uint8_t* f3, const int32_t (&cv)[N], int i,
                       uint32_t types, uint32_t ec, uint64_t PA, uint64_t L, uint64_t ob,
                       int32_t pslot, int lu, int lw, int32_t* dst) {
    constexpr int M = N - 2;
    const uint32_t Tstar = (1u << i) | (1u << M) | (1u << (M + 1));
    const uint32_t kbit = 1u << i;
    int got = 0;
    const int lk = lab_at(L, i);
    for (int t = 0; t < 3; ++t) {
        if (!((types >> t) & 1u)) continue;
        uint64_t A0 = add_edge(PA, i, M);
        if (t == PIECE_KC) A0 = add_edge(A0, i, M + 1);
        else if (t == PIECE_KL) A0 = add_edge(A0, M, M + 1);
        else A0 = add_edge(add_edge(A0, i, M + 1), M, M + 1);
        const uint64_t kbase = (uint64_t)pslot << 35 | (uint64_t)i << 32 | (uint64_t)t << 30 |
                               (uint64_t)lu << 24 | (uint64_t)lw << 18;
        uint32_t sub = ec;
        for (;;) {
            uint64_t A = A0;
            bool ok = true;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if ((sub >> (2 * j)) & 1u) A = add_edge(A, j, M);
                if ((sub >> (2 * j + 1)) & 1u) A = add_edge(A, j, M + 1);
            }
            if (a.prune && sub) {
                // Section 4.5: a size-3 subgraph around the joining vertex k
                // spanning both sides must be a frequent size-3 pattern
#pragma unroll
                for (int j = 0; j < M; ++j) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        if (!((sub >> (2 * j + q)) & 1u) || !ok) continue;
                        const int c = M + q;
                        const bool kb = (amask(A, i) >> j) & 1u;
                        const bool kc = (amask(A, i) >> c) & 1u;
                        const int lb = lab_at(L, j), lc = lab_at(L, c);
                        if (kb && kc) ok = f3_at(f3, a.F, 1, lk, lb, lc);
                        else if (kb) ok = f3_at(f3, a.F, 0, lb, lk, lc);
                        else if (kc) ok = f3_at(f3, a.F, 0, lc, lk, lb);
                    }
                }
            }
            if (ok && dissection_is(N, ob, A, Tstar, kbit)) {
                const uint64_t key = kbase | sub;
                if (MODE == MODE_DOMAIN) {
                    record<N>(a.R, key, L, A, cv);
                    ++got;
                } else {
                    int64_t s = frequent_slot(a.R, key);
                    if (s >= 0) {
                        if (PHASE == 1) {
#pragma unroll
                            for (int p = 0; p < N; ++p) dst[p] = cv[p];
                            dst[N] = (int32_t)s;
                            dst += N + 1;
                        }
                        ++got;
                    }
                }
            }
            if (!sub || a.induced) break;
            sub = (sub - 1) & ec;
        }
    }
    return got;
}

// Two-vertex join (Section 4.1-4.3).  Work item = (parent p, position i),
// k = p[i]; one wave per work item (fetched from a queue in chunks), lanes
// over the pieces rooted at k: centre pairs (u, w) of N(k) (k-centre wedge,
// plus the triangle when u ~ w) and leaf slots (u in N(k), w in N(u)).
template <int N, int MODE>
__global__ __launch_bounds__(TPB) void k_join(JoinArgs a) {
    constexpr int M = N - 2;
    const int lane = threadIdx.x & 63;
    unsigned long long emit = 0, cands = 0, bytes = 0;
    for (;;) {
        unsigned long long w0 = 0;
        if (lane == 0) w0 = atomicAdd(a.work_ctr, (unsigned long long)JOIN_CHUNK);
        w0 = __shfl(w0, 0, 64);
        if ((int64_t)w0 >= a.nwork) break;
        const int64_t wend = min((int64_t)w0 + JOIN_CHUNK, a.nwork);
        for (int64_t wi = (int64_t)w0; wi < wend; ++wi) {
            const int64_t p = wi / M;
            const int i = (int)(wi - p * M);
            const int32_t* prow = a.par + p * (M + 1);
            int32_t cv[N];
#pragma unroll
            for (int j = 0; j < M; ++j) cv[j] = prow[j];
            const int32_t pslot = prow[M];
            const uint64_t PA = a.padj[pslot];
            const uint64_t sthr = a.item_thr ? a.item_thr[(int64_t)pslot * M + i] : a.sample_thr;
            int32_t k = cv[0], mu = INT_MAX;
            uint64_t L = 0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (j == i) k = cv[j];
                else mu = min(mu, cv[j]);
                L |= (uint64_t)a.vf[cv[j]] << (6 * j);
            }
            const int lk = a.vf[k];
            const uint8_t* f3 = a.f3 + (size_t)a.vg[k] * 2 * a.F * a.F * a.F;
            const int32_t rk = a.row[k];
            const int32_t dk = a.row[k + 1] - rk;
            const int64_t ncen = (int64_t)dk * (dk - 1) / 2;
            int64_t Pk = a.npieces[k];
            // ST at the size-4 join: the parent edge must be one of the
            // sampled edges of k's key group
            if (N == 4 && a.smp.ethr && edge_hash(a.smp.seed, 4, k, cv[1 - i]) > a.smp.ethr[k])
                Pk = 0;
            if (lane == 0) {
                cands += (unsigned long long)Pk;
                // parent row, N(k), and the N(u) rows of the k-leaf slots
                bytes += 4ull * (M + 1) + 4ull * (unsigned long long)(dk + (Pk - ncen));
            }
            int64_t base = (MODE == MODE_FILL) ? a.offsets[wi] : 0, total = 0;
            for (int64_t r0 = 0; r0 < Pk; r0 += 64) {
                const int64_t r = r0 + lane;
                int32_t u = -1, w = -1;
                uint32_t types = 0;
                if (r < Pk) {
                    bool centre = r < ncen;
                    if (centre) {
                        int32_t ia, ib;
                        decode_pair(r, &ia, &ib);
                        u = a.col[rk + ia];
                        w = a.col[rk + ib];
                    } else {
                        const int32_t rr = (int32_t)(r - ncen);
                        int32_t lo = 0, hi = dk - 1;   // last ia with leafoff[rk+ia] <= rr
                        while (lo < hi) {
                            int32_t mid = (lo + hi + 1) >> 1;
                            if (a.leafoff[rk + mid] <= rr) lo = mid; else hi = mid - 1;
                        }
                        u = a.col[rk + lo];
                        w = a.col[a.row[u] + (rr - a.leafoff[rk + lo])];
                    }
                    bool ok = w != k;
#pragma unroll
                    for (int j = 0; j < M; ++j) ok = ok && cv[j] != u && cv[j] != w;
                    // n = 4: the smallest vertex of every child lies in the
                    // accepted size-3 part (checked exhaustively for all
                    // connected graphs on 4 vertices), so a piece whose three
                    // vertices all exceed min(parent \ k) is rejected; n = 5:
                    // the piece must precede the parent's triple (lex_less3)
                    if (N == 4 && ok && min(k, min(u, w)) > mu) ok = false;
                    if (N == 5 && ok) {
                        int32_t q0, q1, q2, p0, p1, p2;
                        sort3(k, u, w, q0, q1, q2);
                        sort3(cv[0], cv[1 % M], cv[2 % M], p0, p1, p2);
                        if (!lex_less3(q0, q1, q2, p0, p1, p2)) ok = false;
                    }
                    if (ok && a.sampled && sample_hash(a.seed, N, k, u, w) >= sthr) ok = false;
                    if (ok) {
                        types = piece_types(f3, a.F, a.nh, a.xh, a.induced, centre, k, u, w, lk,
                                            a.vf[u], a.vf[w], bytes);
                        types = st_types(a.smp, N, matched_types(a.smp, types, k, u, w), k, u, w);
                    }
                }
                int64_t got = 0;
                uint32_t ec = 0;
                uint64_t Lc = 0, ob = 0;
                int lu = 0, lw = 0;
                if (types) {
                    lu = a.vf[u];
                    lw = a.vf[w];
                    cv[M] = u;
                    cv[M + 1] = w;
                    Lc = L | (uint64_t)lu << (6 * M) | (uint64_t)lw << (6 * (M + 1));
                    bool clear = true;   // vertex-induced: no edge outside G_f joins the sides
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        if (j == i) continue;
                        if (has_edge(a.nh, cv[j], u)) ec |= 1u << (2 * j);
                        if (has_edge(a.nh, cv[j], w)) ec |= 1u << (2 * j + 1);
                        if (a.induced && (blocked(a.xh, cv[j], u) || blocked(a.xh, cv[j], w)))
                            clear = false;
                    }
                    ob = rank_bits<N>(cv);
                    if (clear)
                        got = children<N, MODE, 0>(a, f3, cv, i, types, ec, PA, Lc, ob, pslot,
                                                   lu, lw, nullptr);
                    bytes += 8ull * 2 * (M - 1) + 4ull * N * (unsigned long long)got;
                }
                if (MODE == MODE_DOMAIN) {
                    emit += (unsigned long long)got;
                } else {
                    const int64_t ex = wave_excl(got, lane);
                    if (MODE == MODE_FILL && got) {
                        // same enumeration again, now writing at this lane's rows
                        const int64_t r2 = base + total + ex;
                        if (r2 + got <= a.out_rows)
                            children<N, MODE, 1>(a, f3, cv, i, types, ec, PA, Lc, ob, pslot, lu,
                                                 lw, a.out + r2 * (N + 1));
                        else
                            atomicOr(a.R.flags, ERR_FILL);
                    }
                    total += wave_sum(got);
                }
            }
            if (MODE == MODE_COUNT && lane == 0) a.counts[wi] = total;
        }
    }
    int64_t t = wave_sum((int64_t)emit);
    int64_t cc = wave_sum((int64_t)cands);
    int64_t bb = wave_sum((int64_t)bytes);
    if (lane == 0) {
        if (t) atomicAdd(a.emitted, (unsigned long long)t);
        if (cc) atomicAdd(a.cands, (unsigned long long)cc);
        if (bb) atomicAdd(a.bytes, (unsigned long long)bb);
    }
}

// Rank-space pair bit: vertices ordered by id, pair (a, b) of ranks in the
// row-major upper-triangle order of an N-vertex graph.
template <int N>
__device__ __forceinline__ uint32_t rbit(int a, int b) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return 1u << (lo * N - lo * (lo + 1) / 2 + (hi - lo - 1));
}

// ------------------------------------------ single-vertex exploration
//
// The baseline that two-vertex exploration is compared with (Section 6):
// a size-n subgraph is a size-(n-1) parent plus one vertex u joined to the
// parent's vertex k by an edge, with any subset of u's other edges into the
// parent (all of them when vertex-induced).  Each subgraph is produced once:
// u must be its largest vertex whose removal leaves it connected, k the
// smallest neighbour of u.  That rule depends only on the child's adjacency
// in id order, so it is a table (svtab): entry = rank(u) | rank(k) << 4,
// 0xff for a disconnected adjacency.

__global__ void k_single_table(int n, uint8_t* tab) {
    const uint32_t total = 1u << (n * (n - 1) / 2);
    const uint32_t all = (1u << n) - 1u;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += gridDim.x * blockDim.x) {
        uint64_t A = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if ((x >> pair_pos(i, j, n)) & 1u) A = add_edge(A, i, j);
        uint8_t e = 0xff;
        if (connected(all, A, n))
            for (int v = n - 1; v >= 0; --v)
                if (connected(all & ~(1u << v), A, n)) {
                    e = (uint8_t)(v | (__ffs(amask(A, v)) - 1) << 4);
                    break;
                }
        tab[x] = e;
    }
}

struct SingleArgs {
    const int32_t* row;      // G_f
    const int32_t* col;
    const int32_t* vf;
    const int32_t* vg;       // graph of each vertex
    NbrHash nh;
    NbrHash xh;              // vertex-induced: edges outside G_f
    int induced;
    const int32_t* par;      // parents: rows of (N-1 vertices, QP slot)
    const uint64_t* padj;    // parent level: packed adjacency per QP slot
    const uint8_t* svtab;
    Rec R;
    unsigned long long* ctr;   // [emitted, candidates, work counter, bytes]
    int64_t nwork;
    Sampling smp;            // ethr: this join's sampled neighbour lists
    int64_t* counts;
    const int64_t* offsets;
    int32_t* out;
    int64_t out_rows;
};

// Children of one (parent, position, new vertex u) candidate: the subsets
// of u's connecting edges ec (ec itself when vertex-induced) whose child
// the removal rule assigns to this (u, k).  PHASE 0 records (domain pass) or
// counts; PHASE 1 writes the rows from dst.
template <int N, int MODE, int PHASE>
__device__ int single_children(const SingleArgs& a, const int32_t (&cv)[N], int i, uint32_t ec,
                               uint64_t PA, uint32_t rpar, const int (&rkv)[N], uint8_t want,
                               uint64_t kbase, uint64_t Lc, int32_t* dst) {
    constexpr int M = N - 1;
    int got = 0;
    uint32_t sub = ec;
    for (;;) {
        uint32_t radj = rpar;
        uint64_t A = add_edge(PA, i, M);
#pragma unroll
        for (int j = 0; j < M; ++j)
            if ((sub >> j) & 1u) {
                radj |= rbit<N>(rkv[j], rkv[M]);
                A = add_edge(A, j, M);
            }
        if (a.svtab[radj] == want) {
            const uint64_t key = kbase | sub;
            if (MODE == MODE_DOMAIN) {
                record<N>(a.R, key, Lc, A, cv);
                ++got;
            } else {
                const int64_t s = frequent_slot(a.R, key);
                if (s >= 0) {
                    if (PHASE == 1) {
#pragma unroll
                        for (int q = 0; q < N; ++q) dst[q] = cv[q];
                        dst[N] = (int32_t)s;
                        dst += N + 1;
                    }
                    ++got;
                }
            }
        }
        if (!sub || a.induced) break;
        sub = (sub - 1) & ec;
    }
    return got;
}

// One wave per work item (parent p, position i), taken from a queue in
// chunks; lanes over the neighbours u of k = p[i].  MODE_DOMAIN records the
// children (the tiled kernel below does this for the library),
// MODE_COUNT / MODE_FILL count and write the frequent ones.
template <int N, int MODE>
__global__ __launch_bounds__(TPB) void k_single(SingleArgs a) {
    constexpr int M = N - 1;
    const int lane = threadIdx.x & 63;
    unsigned long long emit = 0, cands = 0, bytes = 0;
    for (;;) {
        unsigned long long w0 = 0;
        if (lane == 0) w0 = atomicAdd(&a.ctr[2], (unsigned long long)JOIN_CHUNK);
        w0 = __shfl(w0, 0, 64);
        if ((int64_t)w0 >= a.nwork) break;
        const int64_t wend = min((int64_t)w0 + JOIN_CHUNK, a.nwork);
        for (int64_t wi = (int64_t)w0; wi < wend; ++wi) {
            const int64_t p = wi / M;
            const int i = (int)(wi - p * M);
            const int32_t* prow = a.par + p * (M + 1);
            int32_t cv[N];
#pragma unroll
            for (int j = 0; j < M; ++j) cv[j] = prow[j];
            const int32_t pslot = prow[M];
            const uint64_t PA = a.padj[pslot];
            int32_t k = cv[0];
            uint64_t L = 0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (j == i) k = cv[j];
                L |= (uint64_t)a.vf[cv[j]] << (6 * j);
            }
            const int32_t rk = a.row[k], dk = a.row[k + 1] - rk;
            if (lane == 0) {
                cands += (unsigned long long)dk;
                bytes += 4ull * (M + 1) + 4ull * (unsigned long long)dk;
            }
            int64_t base = (MODE == MODE_FILL) ? a.offsets[wi] : 0, total = 0;
            for (int32_t r0 = 0; r0 < dk; r0 += 64) {
                const int32_t r = r0 + lane;
                int got = 0;
                int32_t u = -1;
                bool ok = r < dk;
                if (ok) {
                    u = a.col[rk + r];
#pragma unroll
                    for (int j = 0; j < M; ++j) ok = ok && cv[j] != u;
                    // ST: the edge (k, u) must be one of k's sampled edges
                    if (ok && a.smp.ethr && edge_hash(a.smp.seed, N, k, u) > a.smp.ethr[k])
                        ok = false;
                }
                uint32_t ec = 0;
                if (ok) {
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        if (j == i) continue;
                        if (has_edge(a.nh, cv[j], u)) ec |= 1u << j;
                        else if (a.induced && blocked(a.xh, cv[j], u)) ok = false;
                    }
                    bytes += 8ull * (M - 1);
                }
                int rkv[N];
                uint32_t rpar = 0;
                uint8_t want = 0;
                uint64_t kbase = 0, Lc = 0;
                if (ok) {
                    cv[M] = u;
                    const int lu = a.vf[u];
                    Lc = L | (uint64_t)lu << (6 * M) | (uint64_t)a.vg[k] << 48;
                    // ranks by id; the parent's edges and (k, u) in rank space
#pragma unroll
                    for (int q = 0; q < N; ++q) rkv[q] = 0;
#pragma unroll
                    for (int q = 0; q < N; ++q)
#pragma unroll
                        for (int s2 = q + 1; s2 < N; ++s2) {
                            const int c = cv[q] < cv[s2] ? 1 : 0;
                            rkv[s2] += c;
                            rkv[q] += 1 - c;
                        }
                    int rki = 0;
#pragma unroll
                    for (int q = 0; q < M; ++q)
                        if (q == i) rki = rkv[q];
#pragma unroll
                    for (int q = 0; q < M; ++q)
#pragma unroll
                        for (int s2 = q + 1; s2 < M; ++s2)
                            if ((PA >> (8 * q + s2)) & 1u) rpar |= rbit<N>(rkv[q], rkv[s2]);
                    rpar |= rbit<N>(rki, rkv[M]);
                    want = (uint8_t)(rkv[M] | rki << 4);
                    kbase = (uint64_t)pslot << 35 | (uint64_t)i << 32 | (uint64_t)lu << 24;
                    got = single_children<N, MODE, 0>(a, cv, i, ec, PA, rpar, rkv, want, kbase,
                                                      Lc, nullptr);
                    bytes += 4ull * N * (unsigned long long)got;
                }
                if (MODE == MODE_DOMAIN) {
                    emit += (unsigned long long)got;
                } else {
                    const int64_t ex = wave_excl((int64_t)got, lane);
                    if (MODE == MODE_FILL && got) {
                        const int64_t r2 = base + total + ex;
                        if (r2 + got <= a.out_rows)
                            single_children<N, MODE, 1>(a, cv, i, ec, PA, rpar, rkv, want, kbase,
                                                        Lc, a.out + r2 * (N + 1));
                        else
                            atomicOr(a.R.flags, ERR_FILL);
                    }
                    total += wave_sum((int64_t)got);
                }
            }
            if (MODE == MODE_COUNT && lane == 0) a.counts[wi] = total;
        }
    }
    const int64_t te = wave_sum((int64_t)emit);
    const int64_t tc = wave_sum((int64_t)cands);
    const int64_t tb = wave_sum((int64_t)bytes);
    if (lane == 0) {
        if (te) atomicAdd(&a.ctr[0], (unsigned long long)te);
        if (tc) atomicAdd(&a.ctr[1], (unsigned long long)tc);
        if (tb) atomicAdd(&a.ctr[3], (unsigned long long)tb);
    }
}

// ------------------------------------------------- fixed-size group samples
//
// Threshold of every group of a sampled loop (Section 5): one block per
// group, a radix select of the cap-th smallest member hash over 8-bit digits
// from the top.  Each round recomputes the members' hashes (no member list
// is stored) and histograms the next digit of those that share the digits
// chosen so far; it stops at the first digit whose bin holds exactly the
// members still needed -- every hash of that bin is kept, so the bin's upper
// end keeps the same set as the exact cap-th hash.

constexpr int SEL_TPB = 256;
enum { SEL_PIECES = 0, SEL_EDGES = 1, SEL_MATCH = 2 };

struct SelArgs {
    const int32_t* row;      // G_f
    const int32_t* col;
    const int32_t* leafoff;
    const int64_t* npieces;
    const uint32_t* vinfo;
    const int32_t* vg;
    const uint8_t* f3;
    int F;
    NbrHash nh;
    NbrHash xh;
    int induced;
    Sampling smp;            // mthr applies to the pieces' own matching
    int n;                   // join size (pieces)
    int64_t groups;          // vertices
    uint64_t cap;            // members kept per group (>= 1)
    uint64_t* thr;           // out: per group threshold
};

template <class Units>
__device__ uint64_t block_select(int64_t slots, uint64_t cap, const Units& units,
                                 unsigned long long* hist, uint64_t* sh) {
    uint64_t prefix = 0, need = cap;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = threadIdx.x; b < 256; b += blockDim.x) hist[b] = 0;
        __syncthreads();
        for (int64_t q = threadIdx.x; q < slots; q += blockDim.x)
            units(q, [&](uint64_t h) {
                if (shift == 56 || (h >> (shift + 8)) == prefix)
                    atomicAdd(&hist[(h >> shift) & 255u], 1ull);
            });
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t done = 0, res = 0;
            if (shift == 56) {
                uint64_t total = 0;
                for (int b = 0; b < 256; ++b) total += hist[b];
                if (total <= cap) {
                    done = 1;
                    res = ~0ull;
                }
            }
            if (!done) {
                uint64_t below = 0;
                int b = 0;
                for (; b < 255; ++b) {
                    if (below + hist[b] >= need) break;
                    below += hist[b];
                }
                need -= below;
                prefix = prefix << 8 | (uint64_t)b;
                if (hist[b] == need || shift == 0) {
                    done = 1;
                    res = shift == 0 ? prefix : (prefix << shift | ((1ull << shift) - 1));
                }
            }
            sh[0] = done;
            sh[1] = res;
            sh[2] = prefix;
            sh[3] = need;
        }
        __syncthreads();
        const uint64_t done = sh[0], res = sh[1];
        prefix = sh[2];
        need = sh[3];
        __syncthreads();
        if (done) return res;
    }
    return ~0ull;
}

// KIND SEL_PIECES: group = joining vertex k, members = the stored size-3
// subgraphs containing k (piece slots x their types) at the size-n join;
// SEL_EDGES: members = k's G_f edges (size-4 two-vertex join, every
// single-vertex join); SEL_MATCH: group =
// vertex c, members = the size-3 subgraphs credited to c in matching.
template <int KIND>
__global__ __launch_bounds__(SEL_TPB) void k_group_select(SelArgs a) {
    __shared__ unsigned long long hist[256];
    __shared__ uint64_t sh[4];
    for (int64_t k = blockIdx.x; k < a.groups; k += gridDim.x) {
        const int32_t rk = a.row[k], dk = a.row[k + 1] - rk;
        const int64_t ncen = (int64_t)dk * (dk - 1) / 2;
        int64_t slots = 0, most = 0;   // slots, and an upper bound on members
        if (KIND == SEL_PIECES) {
            slots = a.npieces[k];
            most = slots + ncen;
        } else if (KIND == SEL_EDGES) {
            slots = most = dk;
        } else {
            slots = ncen;
            most = 2 * ncen;
        }
        uint64_t res = ~0ull;
        if ((uint64_t)most > a.cap) {   // block-uniform
            const int32_t kk = (int32_t)k;
            if (KIND == SEL_PIECES) {
                const int lk = (int)(a.vinfo[k] >> 26);
                const uint8_t* f3 = a.f3 + (size_t)a.vg[k] * 2 * a.F * a.F * a.F;
                res = block_select(slots, a.cap, [&](int64_t q, auto&& emit) {
                    int32_t u, w;
                    const bool centre = piece_at(a.row, a.col, a.leafoff, rk, dk, ncen, q, u, w);
                    if (w == kk) return;
                    unsigned long long by = 0;
                    uint32_t types = piece_types(f3, a.F, a.nh, a.xh, a.induced, centre, kk, u, w,
                                                 lk, (int)(a.vinfo[u] >> 26),
                                                 (int)(a.vinfo[w] >> 26), by);
                    types = matched_types(a.smp, types, kk, u, w);
                    for (int t = 0; t < 3; ++t)
                        if ((types >> t) & 1u) emit(piece_hash(a.smp.seed, a.n, t, kk, u, w));
                }, hist, sh);
            } else if (KIND == SEL_EDGES) {
                res = block_select(slots, a.cap, [&](int64_t q, auto&& emit) {
                    emit(edge_hash(a.smp.seed, a.n, kk, a.col[rk + q]));
                }, hist, sh);
            } else {
                res = block_select(slots, a.cap, [&](int64_t q, auto&& emit) {
                    int32_t ia, ib;
                    decode_pair(q, &ia, &ib);
                    const int32_t u = a.col[rk + ia], w = a.col[rk + ib];
                    bool wedge, tri;
                    level3_units(a.nh, a.xh, a.induced, kk, u, w, wedge, tri);
                    if (wedge) emit(match_hash(a.smp.seed, 0, kk, u, w));
                    if (tri) emit(match_hash(a.smp.seed, 1, kk, u, w));
                }, hist, sh);
            }
        }
        if (threadIdx.x == 0) a.thr[k] = res;
        __syncthreads();
    }
}

// ST: the pieces that every joining vertex's key group keeps at the size-n
// join (a.smp.kthr), as (min, max) key / code lists in piece order, the
// format of the sorted size-5 lists -- the join then enumerates only them.
// off == null: count into cnt; else write at off[k].  One wave per vertex.
__global__ __launch_bounds__(TPB) void k_st_pieces(SelArgs a, const int64_t* off, int64_t* cnt,
                                                   uint64_t* key, uint8_t* code) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (TPB / 64);
    for (int64_t k = wave_id_global(); k < a.groups; k += nw) {
        const int32_t rk = a.row[k], dk = a.row[k + 1] - rk;
        const int64_t ncen = (int64_t)dk * (dk - 1) / 2, Q = a.npieces[k];
        const int lk = (int)(a.vinfo[k] >> 26);
        const uint8_t* f3 = a.f3 + (size_t)a.vg[k] * 2 * a.F * a.F * a.F;
        int64_t done = 0;
        for (int64_t q0 = 0; q0 < Q; q0 += 64) {
            const int64_t q = q0 + lane;
            int32_t u = -1, w = -1;
            bool centre = false, keep = false;
            if (q < Q) {
                centre = piece_at(a.row, a.col, a.leafoff, rk, dk, ncen, q, u, w);
                if (w != (int32_t)k) {
                    unsigned long long by = 0;
                    uint32_t types =
                        piece_types(f3, a.F, a.nh, a.xh, a.induced, centre, (int32_t)k, u, w, lk,
                                    (int)(a.vinfo[u] >> 26), (int)(a.vinfo[w] >> 26), by);
                    types = matched_types(a.smp, types, (int32_t)k, u, w);
                    keep = st_types(a.smp, a.n, types, (int32_t)k, u, w) != 0;
                }
            }
            const int64_t ex = wave_excl(keep ? 1 : 0, lane);
            if (off && keep) {
                const int64_t x = off[k] + done + ex;
                key[x] = (uint64_t)(uint32_t)min(u, w) << 32 | (uint32_t)max(u, w);
                code[x] = (uint8_t)((centre ? 0u : 1u) | (u > w ? 2u : 0u));
            }
            done += wave_sum(keep ? 1 : 0);
        }
        if (!off && lane == 0) cnt[k] = done;
    }
}

// Hash-table accounting (Section 6.2's memory-access comparison): the size
// of every joining vertex's key group, the stored size-3 subgraphs that
// contain it (one wave per vertex, lanes over its piece slots), and the sum
// of those sizes, capped at the ST sample, over a join's work items.
__global__ __launch_bounds__(TPB) void k_key_group_sizes(SelArgs a, int64_t* size) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (TPB / 64);
    for (int64_t k = wave_id_global(); k < a.groups; k += nw) {
        const int32_t rk = a.row[k], dk = a.row[k + 1] - rk;
        const int64_t ncen = (int64_t)dk * (dk - 1) / 2, Q = a.npieces[k];
        const int lk = (int)(a.vinfo[k] >> 26);
        const uint8_t* f3 = a.f3 + (size_t)a.vg[k] * 2 * a.F * a.F * a.F;
        int64_t c = 0;
        for (int64_t q = lane; q < Q; q += 64) {
            int32_t u, w;
            const bool centre = piece_at(a.row, a.col, a.leafoff, rk, dk, ncen, q, u, w);
            if (w == (int32_t)k) continue;
            unsigned long long by = 0;
            const uint32_t types =
                piece_types(f3, a.F, a.nh, a.xh, a.induced, centre, (int32_t)k, u, w, lk,
                            (int)(a.vinfo[u] >> 26), (int)(a.vinfo[w] >> 26), by);
            c += __popc(matched_types(a.smp, types, (int32_t)k, u, w));
        }
        c = wave_sum(c);
        if (lane == 0) size[k] = c;
    }
}

__global__ void k_degrees(const int32_t* row, int64_t n, int64_t* deg) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        deg[v] = row[v + 1] - row[v];
}

__global__ void k_item_group_sum(const int32_t* par, int64_t rows, int M, const int64_t* size,
                                 int64_t cap, unsigned long long* out) {
    unsigned long long t = 0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x)
        for (int j = 0; j < M; ++j) {
            const int64_t g = size[par[r * (M + 1) + j]];
            t += (unsigned long long)(cap > 0 && g > cap ? cap : g);
        }
    const int lane = threadIdx.x & 63;
    const int64_t s = wave_sum((int64_t)t);
    if (lane == 0 && s) atomicAdd(out, (unsigned long long)s);
}

// ------------------------------------------------------------ join, tiled
//
// Domain pass of the join, organised like the column hash tables of
// Section 4.2: work items (parent p, position i) are grouped by
// (k = p[i], parent QP, i).  A group's work is |parents| x |pieces at k|;
// it is cut into tiles of 64 pieces (one per lane, decoded once per tile)
// by up to TILE_P parents (wave-uniform, looped).  Within a tile the child
// QP of a lane depends only on the connecting edges, so a two-entry
// register cache resolves almost every QP lookup, and the bits of the
// joining vertex and of the piece's two vertices are set once per
// (lane, QP) per tile; the parent-side bits are tested before being set,
// and lanes sharing a QP read the same words.

constexpr int TILE_P_MAX = 128;

struct GroupBuild {
    const int32_t* par;
    int M;
    int64_t nwork;
    uint64_t* kv;       // key, parent count
    uint64_t mask;
    uint32_t* wslot;    // group-table slot of each work item (tables up to 2^32 slots)
    unsigned* count;    // occupied slots
    uint32_t* flags;
};

__device__ __forceinline__ uint64_t group_key(int32_t k, int32_t pq, int i) {
    return (uint64_t)(uint32_t)k << 32 | (uint64_t)(uint32_t)pq << 3 | (uint64_t)i;
}

// One thread per parent row: its M work items (p, i), i = 0..M-1.
__global__ void k_group_insert(GroupBuild b) {
    const int64_t rows = b.nwork / b.M;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < rows;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* row = b.par + p * (b.M + 1);
        const int32_t pq = row[b.M];
        for (int i = 0; i < b.M; ++i) {
            const uint64_t key = group_key(row[i], pq, i);
            const int64_t s = ht_probe(b.kv, b.mask, key, true, b.count, b.flags, OVF_QP);
            b.wslot[p * b.M + i] = (uint32_t)s;   // an overflowed attempt's slots are never read
            if (s >= 0) atomicAdd((unsigned long long*)&b.kv[2 * s + 1], 1ull);
        }
    }
}

__global__ void k_group_flags(const uint64_t* kv, uint64_t slots, int64_t* flag) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < slots;
         s += (uint64_t)gridDim.x * blockDim.x)
        flag[s] = kv[2 * s] != EMPTY_KEY ? 1 : 0;
}

// every (k, parent QP, position) sub-group takes a contiguous run of its
// key's parent range, so a key's parents come in runs of equal QP/position
__global__ void k_group_place(const uint64_t* kv, uint64_t slots, const int64_t* gid,
                              unsigned long long* kcursor, unsigned long long* goff) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < slots;
         s += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t key = kv[2 * s];
        if (key == EMPTY_KEY) continue;
        goff[gid[s]] = atomicAdd(&kcursor[(int32_t)(key >> 32)], kv[2 * s + 1]);
    }
}

// work items per joining vertex: the counts of its sub-groups (one atomic
// per occupied slot rather than one per work item)
__global__ void k_key_counts(const uint64_t* kv, uint64_t slots, unsigned long long* kpar) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < slots;
         s += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t key = kv[2 * s];
        if (key != EMPTY_KEY) atomicAdd(&kpar[(uint32_t)(key >> 32)], (unsigned long long)kv[2 * s + 1]);
    }
}

__global__ void k_key_flags(const unsigned long long* kpar, int64_t n, int64_t* flag) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        flag[v] = kpar[v] ? 1 : 0;
}

__global__ void k_key_compact(const unsigned long long* kpar, const int64_t* kpoff, int64_t n,
                              const int64_t* kid, int32_t* gk, int64_t* gcnt, int64_t* goff) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t P = (int64_t)kpar[v];
        if (!P) continue;
        const int64_t g = kid[v];
        gk[g] = (int32_t)v;
        gcnt[g] = P;
        goff[g] = kpoff[v];
    }
}

__global__ void k_key_tiles(const int32_t* gk, const int64_t* gcnt, const int64_t* npieces,
                            int64_t ngroups, int tile_p, int64_t* tiles) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ngroups;
         g += (int64_t)gridDim.x * blockDim.x)
        tiles[g] = ((gcnt[g] + tile_p - 1) / tile_p) * ((npieces[gk[g]] + 63) / 64);
}

// One thread per parent row, as in k_group_insert.
__global__ void k_group_fill(int64_t nwork, int M, const uint32_t* wslot, const int64_t* gid,
                             unsigned long long* cursor, int32_t* glist) {
    const int64_t rows = nwork / M;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < rows;
         p += (int64_t)gridDim.x * blockDim.x)
        for (int i = 0; i < M; ++i) {
            const int64_t g = gid[wslot[p * M + i]];
            glist[atomicAdd(&cursor[g], 1ull)] = (int32_t)p;
        }
}


// Kernel state is kept small (scalar registers are scarce in the loop):
// vertex label and label rank share one word, and the QP-table insert path
// reads its pointers through `rec` (device memory) only when it runs.
struct TileArgs {
    const int32_t* row;
    const int32_t* col;
    const uint32_t* vinfo;   // frequent label << 26 | rank within the label
    const int32_t* vg;       // graph of each vertex
    const int64_t* npieces;
    const int32_t* leafoff;
    NbrHash nh;
    const uint8_t* f3;
    int F;
    int tile_p;              // parents per tile
    const int32_t* par;
    const uint64_t* padj;
    const int32_t* gk;       // joining vertex of each key group
    const int64_t* goff;     // its parent range in glist
    const int64_t* gcnt;
    const int64_t* toff;     // ngroups + 1 tile offsets
    int64_t ngroups;
    int64_t ntiles;
    const int32_t* glist;
    const uint16_t* dtab;    // dissection table of this size
    uint32_t* bits;          // QP-position bitmaps
    uint32_t W;
    int32_t rbase;           // first rank of this pass's slice
    int prune;
    const Rec* rec;          // QP table (insert path)
    const uint32_t* flags;   // overflow / error bits of the pass
    unsigned long long* item_children;   // when recording: children per work item
    const uint64_t* pkey;    // size 5: sorted piece lists (null: decode pieces)
    const uint8_t* pcode;
    const int64_t* poff;
    int queue;               // 1: waves take tiles from a device counter (ctr[2]);
                             // 0: wave w takes tiles w, w + waves, ...
    unsigned long long* ctr; // [emitted, candidates, -, bytes]
    int sampled;
    uint64_t seed;
    uint64_t sample_thr;
    const uint64_t* item_thr;   // per work item sampling thresholds, or null
    int induced;                // vertex-induced: induced pieces, C = E_c only
    NbrHash xh;                 // vertex-induced: edges outside G_f
    Sampling smp;               // matching and ST sampling thresholds
    const int32_t* porb;        // as Pool::porb (EXTRA builds)
    unsigned long long* qcnt;   // as Pool::qcnt (EXTRA builds)
};

constexpr uint32_t RANK_MASK = (1u << 26) - 1;

// Two-entry per-lane caches: QP key -> slot, and the QP slots (+1) whose
// joining-vertex / piece bits this lane already set in the current tile.
struct LaneCache {
    uint64_t k0, k1;   // QP keys looked up last (persist across tiles)
    uint32_t v0, v1;   // their slots (tables hold at most 2^31 slots)
    uint32_t b0, b1;   // slots + 1 whose piece bits this lane set in the tile
};

// Adjacency of every parent vertex except k with the piece's two new
// vertices: bit 2j (2j+1) = parent position j ~ u (~ w).  The parent vertex
// is the same across the wave, so all lanes read the same small table; each
// test is two bucket reads.  Only the M - 1 positions other than i are
// probed (position j of the jj-th probe is jj, or jj + 1 past i;
// wave-uniform).  A bucket's byte offset is the lane's pre-shifted hash
// masked by the table's (bucket count - 1) << 2.  The reads are issued
// first (probe_issue) and compared later (probe_bits), so that work not
// depending on them can cover their latency.
template <int N>
struct Probe {
    int32_t bu1[N - 3], bu2[N - 3], bw1[N - 3], bw2[N - 3];
    bool live[N - 3];
};

template <int N>
__device__ __forceinline__ Probe<N> probe_issue(const NbrHash& H, const int32_t (&cv)[N], int i) {
    constexpr int M = N - 2;
    const int32_t u = cv[M], w = cv[M + 1];
    const uint32_t su1 = nbr_hash(u) << 2, su2 = nbr_hash2(u) << 2;
    const uint32_t sw1 = nbr_hash(w) << 2, sw2 = nbr_hash2(w) << 2;
    const FSM_GLOBAL int32_t* tab = gmem(H.tab);
    const FSM_CONST uint32_t* off = cmem(H.off);
    Probe<N> P;
#pragma unroll
    for (int jj = 0; jj < M - 1; ++jj) {
        const int32_t b = jj < i ? cv[jj] : cv[jj + 1];
        // cv[j] is wave-uniform: its table's base and size sit in scalar
        // registers (at most 2^29 buckets per vertex, checked when the
        // tables are built).  A vertex without a table reads bucket 0 of
        // the whole array (it exists) and its result is dropped.
        const uint32_t o = off[b], nb = off[b + 1] - o;
        P.live[jj] = nb != 0;
        const uint32_t m4 = nb ? (nb - 1) << 2 : 0u;
        const FSM_GLOBAL char* base = reinterpret_cast<const FSM_GLOBAL char*>(tab + (nb ? o : 0u));
        auto bucket = [&](uint32_t sh) {
            return *reinterpret_cast<const FSM_GLOBAL int32_t*>(base + (sh & m4));
        };
        P.bu1[jj] = bucket(su1);
        P.bu2[jj] = bucket(su2);
        P.bw1[jj] = bucket(sw1);
        P.bw2[jj] = bucket(sw2);
    }
    return P;
}

// The connecting-edge bits of an issued probe.  Connecting edges are rare:
// the bits are assembled only when some lane of the wave has one.
template <int N>
__device__ __forceinline__ uint32_t probe_bits(const Probe<N>& P, const int32_t (&cv)[N], int i) {
    constexpr int M = N - 2;
    const int32_t uu = cv[M], ww = cv[M + 1];
    bool mu[M - 1], mw[M - 1];
    bool any = false;
#pragma unroll
    for (int jj = 0; jj < M - 1; ++jj) {
        mu[jj] = P.live[jj] && (P.bu1[jj] == uu || P.bu2[jj] == uu);
        mw[jj] = P.live[jj] && (P.bw1[jj] == ww || P.bw2[jj] == ww);
        any = any || mu[jj] || mw[jj];
    }
    if (__ballot(any) == 0ull) return 0u;
    uint32_t ec = 0;
#pragma unroll
    for (int jj = 0; jj < M - 1; ++jj) {
        const int j = jj < i ? jj : jj + 1;
        if (mu[jj]) ec |= 1u << (2 * j);
        if (mw[jj]) ec |= 2u << (2 * j);
    }
    return ec;
}

template <int N>
__device__ __forceinline__ uint32_t connecting_edges(const NbrHash& H, const int32_t (&cv)[N],
                                                     int i) {
    return probe_bits<N>(probe_issue<N>(H, cv, i), cv, i);
}

// All children of one (parent, position, piece) candidate in the domain
// pass.  The dissection check is a lookup in a table indexed by the child's
// adjacency with vertices in id order (the rule depends on nothing else);
// the connecting-edge subsets that the Section 4.5 pruning rejects are
// excluded from the enumeration up front.
template <int N, bool EXTRA>
__device__ __forceinline__ int children_tile(const TileArgs& a, const uint8_t* f3,
                                             const uint16_t* __restrict__ dtab,
                                             const uint32_t* __restrict__ rb,
                                             const int32_t (&cv)[N],
                                             const int32_t (&lr)[N], int i, uint32_t types,
                                             const Probe<N>& pr, uint64_t PA, uint64_t L,
                                             int32_t pslot, int lu, int lw, LaneCache& c) {
    constexpr int M = N - 2;
    // rank of every vertex by id: the vertices are distinct, so one compare
    // per pair decides both ranks
    int rk[N];
#pragma unroll
    for (int p = 0; p < N; ++p) rk[p] = 0;
#pragma unroll
    for (int p = 0; p < N; ++p)
#pragma unroll
        for (int q = p + 1; q < N; ++q) {
            const int c = cv[p] < cv[q] ? 1 : 0;
            rk[q] += c;
            rk[p] += 1 - c;
        }
    int rki = 0;
#pragma unroll
    for (int p = 0; p < M; ++p)
        if (p == i) rki = rk[p];
    uint32_t rpar = 0;
#pragma unroll
    for (int p = 0; p < M; ++p)
#pragma unroll
        for (int q = p + 1; q < M; ++q)
            if ((PA >> (8 * p + q)) & 1u) rpar |= rb[rk[p] << 3 | rk[q]];
    const uint32_t eku = rb[rki << 3 | rk[M]], ekw = rb[rki << 3 | rk[M + 1]];
    const uint32_t euw = rb[rk[M] << 3 | rk[M + 1]];
    const uint32_t want =
        ((1u << rki) | (1u << rk[M]) | (1u << rk[M + 1])) | ((uint32_t)rki << 8);
    // the adjacency reads were issued before the work above
    const uint32_t ec = probe_bits<N>(pr, cv, i);
    // connecting edges allowed by the pruning: pieces joined to k by both
    // new vertices (k-centre wedge, triangle) and k-leaf wedges
    uint32_t allow_both = ec, allow_kl = ec;
    if (a.prune && ec) {
        const int lk = lab_at(L, i);
#pragma unroll
        for (int b = 0; b < 2 * M; ++b) {
            if (!((ec >> b) & 1u)) continue;
            const int j = b >> 1;
            const bool kb = (PA >> (8 * i + j)) & 1u;
            const int lb = lab_at(L, j), lc = (b & 1) ? lw : lu;
            const bool ok2 = kb ? f3_at(f3, a.F, 1, lk, lb, lc) : f3_at(f3, a.F, 0, lc, lk, lb);
            const bool okl = (b & 1) ? (kb ? f3_at(f3, a.F, 0, lb, lk, lc) : true) : ok2;
            if (!ok2) allow_both &= ~(1u << b);
            if (!okl) allow_kl &= ~(1u << b);
        }
    }
    int got = 0;
    // each lane walks its own piece types (nearly always one): a wave runs
    // the body as often as its lane with the most types, not once per type
    // any lane has
    for (uint32_t pend = types; pend; pend &= pend - 1u) {
        const int t = __builtin_ctz(pend);
        const uint32_t r0 =
            rpar | eku | (t == PIECE_KC ? ekw : (t == PIECE_KL ? euw : (ekw | euw)));
        const uint32_t allowed = t == PIECE_KL ? allow_kl : allow_both;
        // vertex-induced: the one child keeps every connecting edge
        if (EXTRA && a.induced && allowed != ec) continue;
        const uint64_t kbase = (uint64_t)pslot << 35 | (uint64_t)i << 32 | (uint64_t)t << 30 |
                               (uint64_t)lu << 24 | (uint64_t)lw << 18;
        uint32_t sub = allowed;
        for (;;) {
            // pair bits of the subset's connecting edges (bit 2j: position
            // j ~ u, 2j + 1: j ~ w); looked up only where a lane has a
            // non-empty subset, which most waves do not
            uint32_t radj = r0;
            if (sub) {
#pragma unroll
                for (int b = 0; b < 2 * M; ++b)
                    if ((sub >> b) & 1u) radj |= rb[rk[b >> 1] << 3 | rk[M + (b & 1)]];
            }
            if (dtab[radj] == want) {
                const uint64_t key = kbase | sub;
                int64_t s;
                if (key == c.k0) {
                    s = (int64_t)c.v0;
                } else if (key == c.k1) {
                    s = (int64_t)c.v1;
                } else {
                    uint64_t A = add_edge(PA, i, M);
                    if (t == PIECE_KC) A = add_edge(A, i, M + 1);
                    else if (t == PIECE_KL) A = add_edge(A, M, M + 1);
                    else A = add_edge(add_edge(A, i, M + 1), M, M + 1);
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        if ((sub >> (2 * j)) & 1u) A = add_edge(A, j, M);
                        if ((sub >> (2 * j + 1)) & 1u) A = add_edge(A, j, M + 1);
                    }
                    s = qp_slot(*a.rec, key, L, A);
                    if (s >= 0) {
                        c.k1 = c.k0; c.v1 = c.v0;
                        c.k0 = key; c.v0 = (uint32_t)s;
                    }
                }
                if (s >= 0 && EXTRA && (a.porb || a.qcnt)) {
                    // candidate-bitmap passes: per-QP counts, bits in the
                    // (pattern, orbit) bitmap of each position
                    if (a.qcnt) atomicAdd(&a.qcnt[s], 1ull);
                    const uint32_t s1 = (uint32_t)s + 1u;
                    const bool once = s1 != c.b0 && s1 != c.b1;
#pragma unroll
                    for (int p = 0; p < N; ++p) {
                        if ((p >= M || p == i) && !once) continue;
                        uint32_t* b = bitmap_at(Pool{a.bits, nullptr, a.W, a.rbase, a.porb},
                                                (uint64_t)s, N, p);
                        if (b) set_bit_in(b, lr[p], a.rbase, a.W);
                    }
                    if (once) {
                        c.b1 = c.b0;
                        c.b0 = s1;
                    }
                } else if (s >= 0) {
                    const uint32_t W = a.W;
                    uint32_t* base = a.bits + (uint64_t)s * N * W;
                    // joining vertex and piece vertices: once per QP per tile
                    const uint32_t s1 = (uint32_t)s + 1u;
                    if (s1 != c.b0 && s1 != c.b1) {
#pragma unroll
                        for (int p = 0; p < N; ++p) {
                            if (p < M && p != i) continue;
                            set_bit_in(base + (uint64_t)p * W, lr[p], a.rbase, W);
                        }
                        c.b1 = c.b0;
                        c.b0 = s1;
                    }
#pragma unroll
                    for (int p = 0; p < M; ++p) {
                        if (p == i) continue;
                        set_bit_in(base + (uint64_t)p * W, lr[p], a.rbase, W);
                    }
                }
                ++got;
            }
            if (!sub || (EXTRA && a.induced)) break;
            sub = (sub - 1) & allowed;
        }
    }
    return got;
}

// Occupancy hides the latency of the adjacency probes and bitmap reads
// better than extra registers would (the kernel entry below sets the waves
// per SIMD).  Wave-uniform values (the tile's group, the parent row, its
// labels, ranks and adjacency) live in scalar registers: their loads go
// through the constant address space.  EXTRA = false builds the exact
// edge-induced join without the sampling and vertex-induced paths (fewer
// live registers).
template <int N, bool EXTRA>
__device__ __forceinline__ void join_tiles(const TileArgs& a) {
    constexpr int M = N - 2;
    // LDS tables: for sizes 4 and 5 the dissection table (2^(n(n-1)/2)
    // entries, at most 2 KB); for every size the bit of the vertex pair with
    // id ranks (x, y) in the child's rank-order adjacency, srb[x * 8 + y]
    constexpr int DT_LDS = N <= 5 ? 1 << (N * (N - 1) / 2) : 1;
    __shared__ uint16_t sdt[DT_LDS];
    __shared__ uint32_t srb[64];
    if (N <= 5)
        for (int x = threadIdx.x; x < DT_LDS; x += TPB) sdt[x] = a.dtab[x];
    if (threadIdx.x < 64) {
        const int x = threadIdx.x >> 3, y = threadIdx.x & 7;
        srb[threadIdx.x] = (x < N && y < N && x != y) ? rbit<N>(x, y) : 0u;
    }
    __syncthreads();
    const uint16_t* __restrict__ dtab = N <= 5 ? sdt : a.dtab;
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (TPB / 64);
    unsigned long long emit = 0, cands = 0, bytes = 0;
    LaneCache c{EMPTY_KEY, EMPTY_KEY, 0, 0, 0, 0};
    int64_t g = 0;
    int64_t run_item = -1, run_sum = 0;   // recording: children of the current item run
    for (int64_t t = a.queue ? -1 : wave_id_global() - nw;;) {
        if (a.queue) {
            unsigned long long nt = 0;
            if (lane == 0) nt = atomicAdd(&a.ctr[2], 1ull);
            // the tile index is wave-uniform: keep it (and all that derives
            // from it: group, parent rows, their labels) in scalar registers
            nt = __shfl(nt, 0, 64);
            t = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(nt >> 32)) << 32) |
                          (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)nt));
        } else {
            t += nw;
        }
        if (t >= a.ntiles) break;
        // an overflowed pass is rerun with a larger table: stop early
        if (__builtin_amdgcn_readfirstlane(
                __hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) & OVF_QP)
            break;
        // group of tile t: last g with toff[g] <= t (t only grows: gallop)
        const auto toff = cmem(a.toff);
        {
            int64_t step = 1;
            while (g + step < a.ngroups && toff[g + step] <= t) { g += step; step <<= 1; }
            int64_t lo = g, hi = min(g + step, a.ngroups - 1);
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) >> 1;
                if (toff[mid] <= t) lo = mid; else hi = mid - 1;
            }
            g = lo;
        }
        const int32_t k = cmem(a.gk)[g];
        const int64_t Q = cmem(a.npieces)[k];
        const int64_t nqt = (Q + 63) / 64;
        const int64_t local = t - toff[g];
        const int64_t pt = local / nqt, qt = local - pt * nqt;
        const int64_t q = qt * 64 + lane;
        const int32_t rk = cmem(a.row)[k];
        const int32_t dk = cmem(a.row)[k + 1] - rk;
        const int64_t ncen = (int64_t)dk * (dk - 1) / 2;
        const int lk = (int)(cmem(a.vinfo)[k] >> 26);
        const uint64_t gid = (uint64_t)cmem(a.vg)[k];
        const uint8_t* f3 = a.f3 + (size_t)gid * 2 * a.F * a.F * a.F;
        // this lane's piece
        int32_t u = -1, w = -1, lru = 0, lrw = 0;
        uint64_t hsh = 0;   // its sampling hash
        uint32_t types = 0;
        int lu = 0, lw = 0;
        uint64_t lkey = ~0ull;   // sorted lists: this lane's (min, max) key
        if (q < Q) {
            bool centre;
            if ((N == 5 || EXTRA) && a.pkey) {
                const int64_t x = a.poff[k] + q;
                lkey = a.pkey[x];
                const uint32_t cd = a.pcode[x];
                const int32_t lo = (int32_t)(lkey >> 32), hi = (int32_t)(lkey & 0xffffffffu);
                centre = !(cd & 1u);
                u = (cd & 2u) ? hi : lo;
                w = (cd & 2u) ? lo : hi;
            } else {
                centre = piece_at(a.row, a.col, a.leafoff, rk, dk, ncen, q, u, w);
            }
            bytes += 4;
            bool ok = w != k;
            if (ok && EXTRA && a.sampled) {
                hsh = sample_hash(a.seed, N, k, u, w);
                if (!a.item_thr && hsh >= a.sample_thr) ok = false;
            }
            if (ok) {
                const uint32_t iu = a.vinfo[u], iw = a.vinfo[w];
                lu = (int)(iu >> 26);
                lw = (int)(iw >> 26);
                lru = (int32_t)(iu & RANK_MASK);
                lrw = (int32_t)(iw & RANK_MASK);
                types = piece_types(f3, a.F, a.nh, a.xh, EXTRA && a.induced, centre, k, u, w, lk, lu, lw,
                                    bytes);
                if (EXTRA) types = st_types(a.smp, N, matched_types(a.smp, types, k, u, w), k, u, w);
            }
        }
        const int32_t qmin = min(k, min(u, w));
        int32_t q0 = 0, q1 = 0, q2 = 0;
        if (N == 5 && !a.pkey) sort3(k, u, w, q0, q1, q2);
        // sorted lists: the tile's smallest key (every lane's key is >= it)
        const uint64_t tkey = (N == 5 && a.pkey) ? cmem(a.pkey)[cmem(a.poff)[k] + qt * 64] : 0;
        // parent range of the tile in glist (work items can exceed 2^31)
        const int64_t pb = cmem(a.goff)[g] + pt * a.tile_p;
        const int64_t pe = min(cmem(a.goff)[g] + cmem(a.gcnt)[g], pb + a.tile_p);
        if (lane == 0) cands += (unsigned long long)((int64_t)(pe - pb) * min((int64_t)64, Q - qt * 64));
        // no lane holds a piece the join may take (infrequent or unsampled):
        // the tile has no children
        if (__ballot(types != 0) == 0ull) continue;
        c.b0 = c.b1 = 0;
        for (int64_t pp = pb; pp < pe; ++pp) {
            const FSM_CONST int32_t* prow = cmem(a.par) + (int64_t)cmem(a.glist)[pp] * (M + 1);
            int32_t cv[N], lr[N];
            int i = 0;
            int32_t mu = INT_MAX;
            uint64_t L = 0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                cv[j] = prow[j];
                if (cv[j] == k) i = j;
            }
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const uint32_t vi = cmem(a.vinfo)[cv[j]];
                lr[j] = (int32_t)(vi & RANK_MASK);
                L |= (uint64_t)(vi >> 26) << (6 * j);
                if (j != i) mu = min(mu, cv[j]);
            }
            if (lane == 0) bytes += 4ull * (M + 1);
            uint64_t pkey = 0;   // size 5: key of the parent's other two vertices
            if (N == 5) {
                const int32_t b1 = cv[i == 0 ? 1 : 0], b2 = cv[i == 2 ? 1 : 2 % M];
                pkey = (uint64_t)(uint32_t)min(b1, b2) << 32 | (uint32_t)max(b1, b2);
                // no piece of this tile precedes the parent's triple
                if (a.pkey && tkey >= pkey) continue;
            }
            const int32_t pslot = prow[M];
            bool ok = types != 0;
#pragma unroll
            for (int j = 0; j < M; ++j) ok = ok && cv[j] != u && cv[j] != w;
            // ST at the size-4 join: the parent edge must be one of the
            // sampled edges of k's key group (wave-uniform)
            if (EXTRA && N == 4 && a.smp.ethr && edge_hash(a.smp.seed, 4, k, cv[1 - i]) > a.smp.ethr[k])
                ok = false;
            // n = 4: the smallest vertex of every child lies in the accepted
            // size-3 part (exhaustively true for connected graphs on 4
            // vertices), so a piece above min(parent \ k) is rejected; n = 5:
            // the piece must precede the parent's triple (lex_less3)
            if (N == 4 && qmin > mu) ok = false;
            if (N == 5) {
                // for a fixed k, sorted triples containing k order as the
                // (min, max) pairs of their other two vertices
                if (a.pkey) {
                    if (lkey >= pkey) ok = false;
                } else {
                    int32_t p0, p1, p2;
                    sort3(cv[0], cv[1 % M], cv[2 % M], p0, p1, p2);
                    if (!lex_less3(q0, q1, q2, p0, p1, p2)) ok = false;
                }
            }
            if (EXTRA && ok && a.item_thr && hsh >= a.item_thr[(int64_t)pslot * M + i]) ok = false;
            int got = 0;
            if (ok) {
                const uint64_t PA = cmem(a.padj)[pslot];
                cv[M] = u;
                cv[M + 1] = w;
                const Probe<N> pr = probe_issue<N>(a.nh, cv, i);
                // vertex-induced: an edge outside G_f between the two sides
                // leaves no child (of this parent; the piece stays for others)
                const uint32_t ty =
                    (EXTRA && a.induced && a.xh.off && connecting_edges<N>(a.xh, cv, i)) ? 0u : types;
                const uint64_t Lc =
                    L | (uint64_t)lu << (6 * M) | (uint64_t)lw << (6 * (M + 1)) | gid << 48;
                lr[M] = lru;
                lr[M + 1] = lrw;
                got = children_tile<N, EXTRA>(a, f3, dtab, srb, cv, lr, i, ty, pr, PA, Lc, pslot,
                                              lu, lw, c);
                emit += (unsigned long long)got;
                bytes += 8ull * 2 * (M - 1) + 4ull * N * (unsigned long long)got;
            }
            if (a.item_children) {   // uniform: every lane is on parent pp
                // parents arrive grouped by (parent QP, position): add runs
                const int64_t item = (int64_t)pslot * M + i;
                if (item != run_item) {
                    if (lane == 0 && run_sum)
                        atomicAdd(&a.item_children[run_item], (unsigned long long)run_sum);
                    run_item = item;
                    run_sum = 0;
                }
                run_sum += wave_sum((int64_t)got);
            }
        }
    }
    if (a.item_children && lane == 0 && run_sum)
        atomicAdd(&a.item_children[run_item], (unsigned long long)run_sum);
    const int64_t te = wave_sum((int64_t)emit);
    const int64_t tc = wave_sum((int64_t)cands);
    const int64_t tb = wave_sum((int64_t)bytes);
    if (lane == 0) {
        if (te) atomicAdd(&a.ctr[0], (unsigned long long)te);
        if (tc) atomicAdd(&a.ctr[1], (unsigned long long)tc);
        if (tb) atomicAdd(&a.ctr[3], (unsigned long long)tb);
    }
}

// The domain pass takes its arguments from device memory: the fields are
// read where they are used instead of being held (and spilled) in scalar
// registers for the whole kernel.
// Five waves per SIMD for the plain pass (96 VGPRs, a few spills outside
// the inner loop); the sampled / vertex-induced build keeps four.
template <int N, bool EXTRA>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(EXTRA ? 4 : 5, 8))) void
k_join_tiles_p(const TileArgs* __restrict__ a) {
    join_tiles<N, EXTRA>(*a);
}

// Domain pass of the single-vertex join, tiled like the two-vertex one:
// work items grouped by (k = p[i], parent QP, i); a tile = up to tile_p
// parents of a group x 64 neighbours u of k (one per lane; a list of D <= 32
// neighbours serves 64 / D parents at a time).  Within a group a lane's
// child QP depends only on u's connecting edges, so the two-entry QP cache
// hits, and the bits of k and u are set once per (lane, QP) per tile.
struct SingleTileArgs {
    const int32_t* row;      // G_f
    const int32_t* col;
    const uint32_t* vinfo;   // frequent label << 26 | rank within the label
    const int32_t* vg;
    NbrHash nh;
    NbrHash xh;
    int induced;
    const int32_t* par;
    const uint64_t* padj;
    const int32_t* gk;
    const int64_t* goff;
    const int64_t* gcnt;
    const int64_t* toff;
    int64_t ngroups;
    int64_t ntiles;
    const int32_t* glist;
    int tile_p;
    const uint8_t* svtab;
    uint32_t* bits;
    uint32_t W;
    int32_t rbase;
    const Rec* rec;
    const uint32_t* flags;
    unsigned long long* ctr;   // [emitted, candidates, tile counter, bytes]
    Sampling smp;              // ethr: this join's sampled neighbour lists
    const int32_t* porb;       // as Pool::porb
    unsigned long long* qcnt;  // as Pool::qcnt
};

template <int N>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_single_tiles(
    const SingleTileArgs* __restrict__ ap) {
    const SingleTileArgs& a = *ap;
    constexpr int M = N - 1;
    const int lane = threadIdx.x & 63;
    unsigned long long emit = 0, cands = 0, bytes = 0;
    LaneCache c{EMPTY_KEY, EMPTY_KEY, 0, 0, 0, 0};
    int64_t g = 0;
    for (;;) {
        unsigned long long nt = 0;
        if (lane == 0) nt = atomicAdd(&a.ctr[2], 1ull);
        // wave-uniform tile index: the group's fields load into scalar registers
        nt = __shfl(nt, 0, 64);
        const int64_t t =
            (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(nt >> 32)) << 32) |
                      (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)nt));
        if (t >= a.ntiles) break;
        if (__builtin_amdgcn_readfirstlane(
                __hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) & OVF_QP)
            break;
        const auto toff = cmem(a.toff);
        {   // group of tile t (t only grows: gallop)
            int64_t step = 1;
            while (g + step < a.ngroups && toff[g + step] <= t) { g += step; step <<= 1; }
            int64_t lo = g, hi = min(g + step, a.ngroups - 1);
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) >> 1;
                if (toff[mid] <= t) lo = mid; else hi = mid - 1;
            }
            g = lo;
        }
        const int32_t k = cmem(a.gk)[g];
        const int32_t rk = cmem(a.row)[k];
        const int64_t Q = cmem(a.row)[k + 1] - rk;
        const int64_t nqt = (Q + 63) / 64;
        const int64_t local = t - toff[g];
        const int64_t pt = local / nqt, qt = local - pt * nqt;
        // short neighbour lists (<= 32) pack 64 / D parents per step into
        // the wave, D = the list length rounded up to a power of two
        int D = 64;
        if (Q <= 32) {
            D = 1;
            while (D < Q) D <<= 1;
        }
        const int64_t q = qt * 64 + (lane & (D - 1));
        const int sub0 = lane / D, step = 64 / D;
        int32_t u = -1, lru = 0;
        int lu = 0;
        bool live = q < Q;
        if (live) {
            u = a.col[rk + q];
            bytes += 4;
            // ST: the edge (k, u) must be one of k's sampled edges
            if (a.smp.ethr && edge_hash(a.smp.seed, N, k, u) > a.smp.ethr[k]) live = false;
            const uint32_t iu = a.vinfo[u];
            lu = (int)(iu >> 26);
            lru = (int32_t)(iu & RANK_MASK);
        }
        // parent range of the tile in glist (work items can exceed 2^31)
        const int64_t pb = cmem(a.goff)[g] + pt * a.tile_p;
        const int64_t pe = min(cmem(a.goff)[g] + cmem(a.gcnt)[g], pb + a.tile_p);
        if (lane == 0) cands += (unsigned long long)((int64_t)(pe - pb) * min((int64_t)64, Q - qt * 64));
        if (__ballot(live) == 0ull) continue;
        c.b0 = c.b1 = 0;
        const uint64_t gid = (uint64_t)cmem(a.vg)[k];
        for (int64_t pp = pb + sub0; pp < pe; pp += step) {
            const FSM_GLOBAL int32_t* prow = gmem(a.par) + (int64_t)gmem(a.glist)[pp] * (M + 1);
            int32_t cv[N], lr[N];
            int i = 0;
            uint64_t L = 0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                cv[j] = prow[j];
                if (cv[j] == k) i = j;
            }
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const uint32_t vi = gmem(a.vinfo)[cv[j]];
                lr[j] = (int32_t)(vi & RANK_MASK);
                L |= (uint64_t)(vi >> 26) << (6 * j);
            }
            if ((lane & (D - 1)) == 0) bytes += 4ull * (M + 1);
            const int32_t pslot = prow[M];
            bool ok = live;
#pragma unroll
            for (int j = 0; j < M; ++j) ok = ok && cv[j] != u;
            int got = 0;
            if (ok) {
                const uint64_t PA = gmem(a.padj)[pslot];
                uint32_t ec = 0;
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    if (j == i) continue;
                    if (has_edge(a.nh, cv[j], u)) ec |= 1u << j;
                    else if (a.induced && blocked(a.xh, cv[j], u)) ok = false;
                }
                bytes += 8ull * (M - 1);
                cv[M] = u;
                lr[M] = lru;
                int rkv[N];
#pragma unroll
                for (int x = 0; x < N; ++x) rkv[x] = 0;
#pragma unroll
                for (int x = 0; x < N; ++x)
#pragma unroll
                    for (int y = x + 1; y < N; ++y) {
                        const int cc = cv[x] < cv[y] ? 1 : 0;
                        rkv[y] += cc;
                        rkv[x] += 1 - cc;
                    }
                int rki = 0;
#pragma unroll
                for (int x = 0; x < M; ++x)
                    if (x == i) rki = rkv[x];
                uint32_t rpar = rbit<N>(rki, rkv[M]);
#pragma unroll
                for (int x = 0; x < M; ++x)
#pragma unroll
                    for (int y = x + 1; y < M; ++y)
                        if ((PA >> (8 * x + y)) & 1u) rpar |= rbit<N>(rkv[x], rkv[y]);
                const uint8_t want = (uint8_t)(rkv[M] | rki << 4);
                const uint64_t kbase =
                    (uint64_t)pslot << 35 | (uint64_t)i << 32 | (uint64_t)lu << 24;
                const uint64_t Lc = L | (uint64_t)lu << (6 * M) | gid << 48;
                uint32_t sub = ec;
                while (ok) {
                    uint32_t radj = rpar;
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        if ((sub >> j) & 1u) radj |= rbit<N>(rkv[j], rkv[M]);
                    if (a.svtab[radj] == want) {
                        const uint64_t key = kbase | sub;
                        int64_t sl;
                        if (key == c.k0) {
                            sl = (int64_t)c.v0;
                        } else if (key == c.k1) {
                            sl = (int64_t)c.v1;
                        } else {
                            uint64_t A = add_edge(PA, i, M);
#pragma unroll
                            for (int j = 0; j < M; ++j)
                                if ((sub >> j) & 1u) A = add_edge(A, j, M);
                            sl = qp_slot(*a.rec, key, Lc, A);
                            if (sl >= 0) {
                                c.k1 = c.k0; c.v1 = c.v0;
                                c.k0 = key; c.v0 = (uint32_t)sl;
                            }
                        }
                        if (sl >= 0) {
                            if (a.qcnt) atomicAdd(&a.qcnt[sl], 1ull);
                            auto bm = [&](int p) -> uint32_t* {
                                if (a.porb) {
                                    const int32_t x = a.porb[(uint64_t)sl * N + p];
                                    return x < 0 ? nullptr : a.bits + (uint64_t)x * a.W;
                                }
                                return a.bits + ((uint64_t)sl * N + p) * a.W;
                            };
                            // k and u: once per QP per tile
                            const uint32_t s1 = (uint32_t)sl + 1u;
                            if (s1 != c.b0 && s1 != c.b1) {
                                if (uint32_t* b = bm(i)) set_bit_in(b, lr[i], a.rbase, a.W);
                                if (uint32_t* b = bm(M)) set_bit_in(b, lr[M], a.rbase, a.W);
                                c.b1 = c.b0;
                                c.b0 = s1;
                            }
#pragma unroll
                            for (int j = 0; j < M; ++j) {
                                if (j == i) continue;
                                if (uint32_t* b = bm(j)) set_bit_in(b, lr[j], a.rbase, a.W);
                            }
                        }
                        ++got;
                    }
                    if (!sub || a.induced) break;
                    sub = (sub - 1) & ec;
                }
                emit += (unsigned long long)got;
                bytes += 4ull * N * (unsigned long long)got;
            }
        }
    }
    const int64_t te = wave_sum((int64_t)emit);
    const int64_t tc = wave_sum((int64_t)cands);
    const int64_t tb = wave_sum((int64_t)bytes);
    if (lane == 0) {
        if (te) atomicAdd(&a.ctr[0], (unsigned long long)te);
        if (tc) atomicAdd(&a.ctr[1], (unsigned long long)tc);
        if (tb) atomicAdd(&a.ctr[3], (unsigned long long)tb);
    }
}

// Dissection table of size n: entry x (pair bits of a connected n-vertex
// graph whose vertex i has the i-th smallest id) = l | v' << 8, the split
// dissect() picks; 0 for disconnected graphs.
__global__ void k_dissect_table(int n, uint16_t* tab) {
    const uint32_t total = 1u << (n * (n - 1) / 2);
    uint64_t ob = 0;
    for (int r = 0; r < n; ++r) ob |= (uint64_t)(1u << r) << (8 * r);
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += gridDim.x * blockDim.x) {
        uint64_t A = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if ((x >> pair_pos(i, j, n)) & 1u) A = add_edge(A, i, j);
        uint16_t e = 0;
        if (connected((1u << n) - 1u, A, n)) {
            uint32_t vb = 0;
            const uint32_t l = dissect(n, ob, A, &vb);
            e = (uint16_t)(l | ((uint32_t)__ffs(vb) - 1u) << 8);
        }
        tab[x] = e;
    }
}

// ------------------------------------------------- canonical patterns

struct CanonArgs {
    QPTab q;
    CodeTab c;
    uint32_t* flags;
    int n;
    uint64_t slots;
    uint64_t ngraphs;   // graphs of the call: every packed graph id is below it
};

// One thread per QP: canonical form (the one isomorphism computation of
// its group), pattern slot, and the orbit slot of each QP position.
__device__ __forceinline__ void qp_canon(const CanonArgs& a) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < a.slots;
         s += (uint64_t)gridDim.x * blockDim.x) {
        if (a.q.kv[2 * s] == EMPTY_KEY) continue;
        const uint64_t L = a.q.lab[s];
        const uint64_t gid = L >> 48;
        if (gid >= a.ngraphs) {   // a corrupted key layout, never a valid graph
            atomicOr(a.flags, ERR_GRAPH);
            continue;
        }
        const Canon cn = canonicalize(a.n, L, a.q.adj[s]);
        if (gid && !code_has_graph(a.n)) {
            atomicOr(a.flags, ERR_BATCH);
            continue;
        }
        const uint64_t code = cn.code | gid << CODE_GRAPH_SHIFT;
        const int64_t p = ht_probe(a.c.kv, a.c.mask, code, true, a.c.count, a.flags, OVF_CODE);
        if (p < 0) continue;
        a.c.info[p] = VALID | cn.orbits;   // same value from every QP of the pattern
        a.q.pat[s] = (int32_t)p;
        a.q.kv[2 * s + 1] = VALID | cn.slots;
    }
}

struct MergeArgs {
    QPTab q;
    const uint32_t* qbits;     // QP slot s, position p: bitmap s*n+p of Wsrc words
    uint32_t* pbits;           // pattern slot P, orbit slot o: bitmap P*n+o of W words
    uint32_t Wsrc;
    uint32_t woff;             // words woff .. woff+W-1 of every QP bitmap
    uint32_t W;
    int n;
    uint64_t items;            // QP slots * n
};

// OR every QP position bitmap into its (pattern, orbit) bitmap.
__device__ __forceinline__ void qp_merge(const MergeArgs& a) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nw = (uint64_t)gridDim.x * (TPB / 64);
    for (uint64_t it = (uint64_t)wave_id_global(); it < a.items; it += nw) {
        const uint64_t s = it / a.n;
        const int p = (int)(it - s * a.n);
        const uint64_t v = a.q.kv[2 * s + 1];
        if (a.q.kv[2 * s] == EMPTY_KEY || !(v & VALID)) continue;
        const uint32_t o = (uint32_t)(v >> (3 * p)) & 7u;
        const uint32_t* src = a.qbits + it * a.Wsrc + a.woff;
        uint32_t* dst = a.pbits + ((uint64_t)a.q.pat[s] * a.n + o) * a.W;
        for (uint32_t w = lane; w < a.W; w += 64) {
            const uint32_t x = src[w];
            if (x && (dst[w] & x) != x) atomicOr(&dst[w], x);
        }
    }
}

// --------------------------------------------------------- MNI reduction

struct MniArgs {
    CodeTab c;
    Pool pool;
    int n;
    uint64_t slots;
    uint64_t* out_key;
    int64_t* out_sup;
    unsigned* out_n;
    unsigned out_cap;
};

// One wavefront per pattern slot: add the popcount of each orbit bitmap
// of this pass's rank slice to the orbit's domain size.
__device__ __forceinline__ void orbit_count(const MniArgs& a, int64_t* ocnt) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nw = (uint64_t)gridDim.x * (TPB / 64);
    for (uint64_t s = (uint64_t)wave_id_global(); s < a.slots; s += nw) {
        if (a.c.kv[2 * s] == EMPTY_KEY) continue;
        const uint64_t info = a.c.info[s];
        if (!(info & VALID)) continue;
        const uint32_t* base = a.pool.words + s * a.n * a.pool.W;
        for (int cp = 0; cp < a.n; ++cp) {
            if ((int)((info >> (3 * cp)) & 7u) != cp) continue;
            const uint32_t* bm = base + (uint64_t)cp * a.pool.W;
            int64_t cnt = 0;
            for (uint32_t i = lane; i < a.pool.W; i += 64) cnt += __popc(bm[i]);
            cnt = wave_sum(cnt);
            if (lane == 0) ocnt[s * a.n + cp] += cnt;
        }
    }
}

// MNI support of every pattern slot (Section 2.2): the smallest orbit
// domain; one thread per slot.
__device__ __forceinline__ void mni(const MniArgs& a, const int64_t* ocnt) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < a.slots;
         s += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t key = a.c.kv[2 * s];
        if (key == EMPTY_KEY) continue;
        const uint64_t info = a.c.info[s];
        int64_t best = -1;
        if (info & VALID)
            for (int cp = 0; cp < a.n; ++cp) {
                if ((int)((info >> (3 * cp)) & 7u) != cp) continue;
                const int64_t c = ocnt[s * a.n + cp];
                if (best < 0 || c < best) best = c;
            }
        if (best < 0) best = 0;
        a.c.sup[s] = best;
        const unsigned idx = atomicAdd(a.out_n, 1u);
        if (idx < a.out_cap) {
            a.out_key[idx] = key;
            a.out_sup[idx] = best;
        }
    }
}

__global__ void k_qp_canon(CanonArgs a) { qp_canon(a); }
__global__ __launch_bounds__(TPB) void k_qp_merge(MergeArgs a) { qp_merge(a); }
__global__ __launch_bounds__(TPB) void k_orbit_count(MniArgs a, int64_t* ocnt) {
    orbit_count(a, ocnt);
}
__global__ void k_mni(MniArgs a, const int64_t* ocnt) { mni(a, ocnt); }

// ------------------------------------------------ captured join levels
//
// A batched call runs the last join level of each chunk as one replay of a
// HIP graph: reset of the level's tables, domain pass, canonical forms,
// merge into (pattern, orbit) bitmaps, orbit popcounts and MNI.  The reset
// and the domain pass read their arguments from a device descriptor; the
// other kernels' arguments are set in the executable graph before each
// replay.  One instantiated graph serves every chunk of the same level size
// and grid; the host writes the chunk's descriptor, replays, and
// synchronises once to read the overflow flags and the patterns.  Nothing is
// cleared by memset nodes: k_level_reset fills.
struct LevelDesc {
    TileArgs t;
    CanonArgs ca;
    MergeArgs ma;
    MniArgs m;
    int64_t* ocnt;
    uint32_t* pool;            // QP-position bitmaps
    uint32_t* ppool;           // pattern-orbit bitmaps
    unsigned long long* counters;
    uint32_t* flags;
    uint64_t qslots, cslots, pool_words, ppool_words, ocnt_items;
};

// Grid-stride fill of n words (16-byte stores where aligned).
__device__ __forceinline__ void fill_words(uint32_t* p, uint64_t n, uint64_t tid, uint64_t nth) {
    const uint64_t n4 = ((uintptr_t)p & 15) ? 0 : n / 4;
    uint4* q = reinterpret_cast<uint4*>(p);
    for (uint64_t x = tid; x < n4; x += nth) q[x] = make_uint4(0, 0, 0, 0);
    for (uint64_t x = n4 * 4 + tid; x < n; x += nth) p[x] = 0;
}

__global__ void k_level_reset(const LevelDesc* __restrict__ d) {
    const QPTab& q = d->ca.q;
    const CodeTab& c = d->ca.c;
    const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = tid; x < d->qslots; x += nth) {
        q.kv[2 * x] = EMPTY_KEY;
        q.kv[2 * x + 1] = 0;
        q.adj[x] = 0;
        q.lab[x] = 0;
        q.pat[x] = 0;
    }
    for (uint64_t x = tid; x < d->cslots; x += nth) {
        c.kv[2 * x] = EMPTY_KEY;
        c.kv[2 * x + 1] = 0;
        c.info[x] = 0;
        c.sup[x] = 0;
    }
    fill_words(d->pool, d->pool_words, tid, nth);
    fill_words(d->ppool, d->ppool_words, tid, nth);
    for (uint64_t x = tid; x < d->ocnt_items; x += nth) d->ocnt[x] = 0;
    if (tid == 0) {
        *q.count = 0;
        *c.count = 0;
        *d->m.out_n = 0;
        *d->flags = 0;
        for (int k = 0; k < 4; ++k) d->counters[k] = 0;
    }
}


// Levels whose domains take more than one rank slice keep bitmaps only for
// candidate patterns.  The automorphisms of a subgraph map an orbit o onto
// itself, so every subgraph puts exactly |o| vertices into o's domain and a
// pattern's MNI support is at most (its subgraph count) x (its smallest
// orbit's size); a pattern below t on that bound is infrequent.  Its support
// from the first slice is a lower bound below t; the later slices set bits
// directly in one bitmap per candidate (pattern, orbit).
__global__ void k_pattern_counts(QPTab q, uint64_t slots, const unsigned long long* qcnt,
                                 unsigned long long* pcnt) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < slots;
         s += (uint64_t)gridDim.x * blockDim.x) {
        if (q.kv[2 * s] == EMPTY_KEY || !(q.kv[2 * s + 1] & VALID)) continue;
        if (qcnt[s]) atomicAdd(&pcnt[q.pat[s]], qcnt[s]);
    }
}

// cand[s*n+o] = 1 for the orbit representatives o of candidate pattern slots.
__global__ void k_candidate_flags(CodeTab c, uint64_t slots, int n,
                                  const unsigned long long* pcnt, const int64_t* tg,
                                  int ngraphs, int64_t* cand, uint32_t* flags) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < slots * n;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t s = x / n;
        const int p = (int)(x - s * n);
        int64_t f = 0;
        const uint64_t key = c.kv[2 * s];
        if (key != EMPTY_KEY) {
            const uint64_t info = c.info[s];
            const int gi = code_graph(key, n);
            if (gi >= ngraphs) atomicOr(flags, ERR_GRAPH);
            if ((info & VALID) && gi < ngraphs && (int)((info >> (3 * p)) & 7u) == p) {
                int smallest = n;   // smallest orbit size
                for (int r = 0; r < n; ++r) {
                    if ((int)((info >> (3 * r)) & 7u) != r) continue;
                    int size = 0;
                    for (int q = 0; q < n; ++q) size += (int)((info >> (3 * q)) & 7u) == r;
                    smallest = min(smallest, size);
                }
                if (pcnt[s] * (unsigned long long)smallest >= (unsigned long long)tg[gi])
                    f = 1;
            }
        }
        cand[x] = f;
    }
}

__global__ void k_po_map(const int64_t* cand, const int64_t* poidx, uint64_t items,
                         int64_t* pomap) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < items;
         x += (uint64_t)gridDim.x * blockDim.x)
        if (cand[x]) pomap[poidx[x]] = (int64_t)x;
}

// porb[s*n+p]: the candidate (pattern, orbit) bitmap of QP slot s's
// position p, or -1.
__global__ void k_qp_orbit_map(QPTab q, uint64_t slots, int n, const int64_t* cand,
                               const int64_t* poidx, int32_t* porb) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < slots * n;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t s = x / n;
        const int p = (int)(x - s * n);
        int32_t r = -1;
        const uint64_t v = q.kv[2 * s + 1];
        if (q.kv[2 * s] != EMPTY_KEY && (v & VALID)) {
            const uint64_t y = (uint64_t)q.pat[s] * n + ((v >> (3 * p)) & 7u);
            if (cand[y]) r = (int32_t)poidx[y];
        }
        porb[x] = r;
    }
}

// Popcount of every candidate bitmap of a direct slice into its orbit's
// domain size; one wavefront per bitmap.
__global__ __launch_bounds__(TPB) void k_dense_count(const uint32_t* words, uint64_t nbm,
                                                     uint32_t W, const int64_t* pomap,
                                                     int64_t* ocnt) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nw = (uint64_t)gridDim.x * (TPB / 64);
    for (uint64_t b = (uint64_t)wave_id_global(); b < nbm; b += nw) {
        const uint32_t* bm = words + b * W;
        int64_t cnt = 0;
        for (uint32_t i = lane; i < W; i += 64) cnt += __popc(bm[i]);
        cnt = wave_sum(cnt);
        if (lane == 0 && cnt) ocnt[pomap[b]] += cnt;
    }
}

// Move every QP of `from` into the smaller table `to` (same keys, values,
// ordered subgraphs and pattern slots).
__global__ void k_qp_rehash(QPTab from, uint64_t slots, QPTab to, uint32_t* flags) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < slots;
         s += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t key = from.kv[2 * s];
        if (key == EMPTY_KEY) continue;
        const int64_t h = ht_probe(to.kv, to.mask, key, true, to.count, flags, OVF_QP);
        if (h < 0) continue;
        to.kv[2 * h + 1] = from.kv[2 * s + 1];
        to.adj[h] = from.adj[s];
        to.lab[h] = from.lab[s];
        to.pat[h] = from.pat[s];
    }
}

// FREQ bit on every QP whose pattern reached its graph's threshold
__global__ void k_mark_frequent(QPTab q, uint64_t slots, const uint64_t* ckv, const int64_t* sup,
                                const int64_t* tg, int ngraphs, int n, uint32_t* flags) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < slots;
         s += (uint64_t)gridDim.x * blockDim.x) {
        if (q.kv[2 * s] == EMPTY_KEY) continue;
        uint64_t v = q.kv[2 * s + 1];
        if (!(v & VALID)) continue;
        const int32_t p = q.pat[s];
        const int gi = code_graph(ckv[2 * p], n);
        if (gi >= ngraphs) {
            atomicOr(flags, ERR_GRAPH);
            continue;
        }
        if (sup[p] >= tg[gi]) q.kv[2 * s + 1] = v | FREQ;
    }
}

// ------------------------------------------------ cost-model work items
//
// A work item of the size-n join is (parent QP slot s, joining position i);
// its id is s * (n - 2) + i.  Child QP keys start with (s, i), so the items'
// child QP sets are disjoint and sum to the level's QP count.

// Parent embeddings per QP slot and the G_f degree sum of each position.
// Integer sums keep the features, and so the predictions and the sampling
// proposal, independent of the order of the atomics.
__global__ void k_item_stats(const int32_t* par, int64_t rows, int M, const int32_t* frow,
                             unsigned* cnt, unsigned long long* degsum) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* pr = par + r * (M + 1);
        const int64_t s = pr[M];
        atomicAdd(&cnt[s], 1u);
        for (int i = 0; i < M; ++i)
            atomicAdd(&degsum[s * M + i], (unsigned long long)(frow[pr[i] + 1] - frow[pr[i]]));
    }
}

__global__ void k_item_flags(const unsigned* cnt, int64_t items, int M, int64_t* flag) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < items;
         x += (int64_t)gridDim.x * blockDim.x)
        flag[x] = cnt[x / M] ? 1 : 0;
}

struct FeatArgs {
    const int64_t* pos;      // exclusive scan of the item flags
    int32_t* graph;          // rows: graph id of the item (batches)
    const unsigned* cnt;
    const unsigned long long* degsum;
    const uint64_t* qadj;    // parent QP tables
    const uint64_t* qlab;
    const int32_t* qpat;
    const int64_t* csup;
    const int64_t* tg;
    int64_t items;
    int M, n;
    float* x;                // rows x FSM_FEATURES
    int32_t* item;           // rows
};

// Features of every item with parent embeddings, at row pos[item] (the
// layout fsm.h documents under FSM_FEATURES).
__global__ void k_item_features(FeatArgs a) {
    for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < a.items;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = it / a.M;
        const int i = (int)(it - s * a.M);
        const unsigned c = a.cnt[s];
        if (!c) continue;
        float* x = a.x + a.pos[it] * FSM_FEATURES;
        a.item[a.pos[it]] = (int32_t)it;
        const uint64_t L = a.qlab[s];
        a.graph[a.pos[it]] = (int32_t)(L >> 48);
        const int npairs = a.M * (a.M - 1) / 2;
        x[0] = (float)a.n / 8.0f;
        x[1] = (float)(__popcll(a.qadj[s]) / 2) / (float)(npairs > 0 ? npairs : 1);
        x[2] = log1pf((float)c) / 16.0f;
        x[3] = log1pf((float)((double)a.degsum[it] / (double)c)) / 8.0f;
        x[4] = log1pf((float)a.csup[a.qpat[s]]) / 16.0f;
        x[5] = log1pf((float)a.tg[L >> 48]) / 16.0f;
        for (int b = 0; b < 2 * FSM_FEATURE_LABELS; ++b) x[6 + b] = 0.0f;
        for (int p = 0; p < a.M; ++p) {
            const int l = min(lab_at(L, p), FSM_FEATURE_LABELS - 1);
            x[6 + l] += 1.0f / (float)a.M;
            if (p == i) x[6 + FSM_FEATURE_LABELS + l] = 1.0f;
        }
    }
}

// Targets of every row: log1p(children), log1p(child QPs) of its item.
__global__ void k_item_targets(const int32_t* item, int64_t rows,
                               const unsigned long long* children, const unsigned* qps, float* t) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t it = item[r];
        t[2 * r] = log1pf((float)children[it]);
        t[2 * r + 1] = log1pf((float)qps[it]);
    }
}

// Predicted children per parent embedding of every item.
__global__ void k_item_rowcost(const float* y, const int32_t* item, int64_t rows, int M,
                               const unsigned* cnt, float* rowcost) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t it = item[r];
        rowcost[it] = expm1f(fmaxf(y[2 * r], 0.0f)) / (float)max(cnt[it / M], 1u);
    }
}

// Predicted cost per tile of every key group: the predicted children of its
// parent embeddings over its tile count.  One wavefront per group.
__global__ void k_group_cost(const int32_t* gk, const int64_t* goff, const int64_t* gcnt,
                             const int64_t* tiles, int64_t ngroups, const int32_t* glist,
                             const int32_t* par, int M, const float* rowcost, float* gcost) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t g = wave_id_global(); g < ngroups; g += nw) {
        const int32_t k = gk[g];
        float acc = 0.f;
        for (int64_t j = lane; j < gcnt[g]; j += 64) {
            const int32_t* row = par + (int64_t)glist[goff[g] + j] * (M + 1);
            int i = 0;
            for (int p = 0; p < M; ++p)
                if (row[p] == k) i = p;
            acc += rowcost[(int64_t)row[M] * M + i];
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
        if (lane == 0) gcost[g] = acc / (float)max(tiles[g], (int64_t)1);
    }
}

// Sum of expm1 of one prediction column (the predicted level total).
__global__ void k_pred_total(const float* y, int64_t rows, int col, double* out) {
    double acc = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x)
        acc += expm1((double)fmaxf(y[2 * r + col], 0.0f));
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0 && acc != 0.0) atomicAdd(out, acc);
}

// ================================================================== host

// One graph of a batch copied into the union CSR: vertex ids shifted by
// voff, CSR offsets by eoff, labels mapped to the batch's label ids.
__global__ void k_union_graph(const int32_t* row, const int32_t* col, const int32_t* lab,
                              int64_t n, int64_t nnz, int64_t voff, int64_t eoff,
                              const int32_t* lmap, int32_t gid, int32_t* urow, int32_t* ucol,
                              int32_t* ulab, int32_t* uvg) {
    const int64_t items = n > nnz ? n : nnz;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < items;
         x += (int64_t)gridDim.x * blockDim.x) {
        if (x < n) {
            urow[voff + x] = (int32_t)(row[x] + eoff);
            ulab[voff + x] = lmap[lab[x]];
            uvg[voff + x] = gid;
        }
        if (x < nnz) ucol[eoff + x] = (int32_t)(col[x] + voff);
    }
}

__global__ void k_offsets32(const int64_t* in, int64_t n, int32_t* out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)in[i];
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// The graph a mining call works on: one built graph, or the disjoint union
// of a batch (every connected pattern lies in one graph, so keying patterns
// by graph id keeps the graphs' results apart).
struct GraphView {
    int64_t n = 0, nnz = 0;
    const int32_t* row = nullptr;
    const int32_t* col = nullptr;
    const int32_t* lab = nullptr;       // label id 0..L-1
    const int32_t* vg = nullptr;        // graph id per vertex
    DBuf<int32_t> urow, ucol, ulab, uvg;
    int32_t ngraphs = 1, L = 0;
    std::vector<int32_t> label_value;   // label id -> caller's label
    std::vector<int64_t> count;         // [graph * L + label] vertices

    void single(const fsm_graph* g) {
        n = g->n;
        nnz = g->nnz;
        row = g->row.p;
        col = g->col.p;
        lab = g->lab.p;
        ngraphs = 1;
        L = g->num_labels;
        label_value = g->label_value;
        count = g->label_count;
        uvg.alloc((size_t)n);
        uvg.zero();
        vg = uvg.p;
    }

    void batch(const fsm_graph* const* gs, int32_t k) {
        ngraphs = k;
        std::vector<int32_t> vals;
        for (int32_t i = 0; i < k; ++i) {
            n += gs[i]->n;
            nnz += gs[i]->nnz;
            vals.insert(vals.end(), gs[i]->label_value.begin(), gs[i]->label_value.end());
        }
        if (n > INT32_MAX || nnz > INT32_MAX)
            fail(FSM_EUNSUPPORTED, "batch exceeds 2^31-1 vertices or CSR entries");
        std::sort(vals.begin(), vals.end());
        vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
        label_value = vals;
        L = (int32_t)vals.size();
        count.assign((size_t)k * L, 0);
        urow.alloc((size_t)n + 1);
        ucol.alloc((size_t)(nnz > 0 ? nnz : 1));
        ulab.alloc((size_t)n);
        uvg.alloc((size_t)n);
        int64_t voff = 0, eoff = 0;
        hipStream_t st = stream();
        std::vector<DBuf<int32_t>> maps;
        for (int32_t i = 0; i < k; ++i) {
            const fsm_graph* g = gs[i];
            std::vector<int32_t> lm((size_t)g->num_labels);
            for (int32_t r = 0; r < g->num_labels; ++r) {
                lm[(size_t)r] = (int32_t)(std::lower_bound(vals.begin(), vals.end(),
                                                           g->label_value[(size_t)r]) -
                                          vals.begin());
                count[(size_t)i * L + lm[(size_t)r]] = g->label_count[(size_t)r];
            }
            maps.emplace_back(lm.size());
            to_device(maps.back().p, lm.data(), lm.size());
            const int64_t items = std::max(g->n, g->nnz);
            k_union_graph<<<grid_for(items, 256), 256, 0, st>>>(
                g->row.p, g->col.p, g->lab.p, g->n, g->nnz, voff, eoff, maps.back().p, i, urow.p,
                ucol.p, ulab.p, uvg.p);
            FSM_LAUNCH_CHECK();
            voff += g->n;
            eoff += g->nnz;
        }
        k_fill_i32<<<1, 1, 0, st>>>(urow.p + n, 1, (int32_t)nnz);
        FSM_LAUNCH_CHECK();
        sync_stream(st);
        row = urow.p;
        col = ucol.p;
        lab = ulab.p;
        vg = uvg.p;
    }
};

struct Tables {
    DBuf<uint64_t> qkv, qadj, qlab, ckv, cinfo;
    DBuf<int32_t> qpat;
    DBuf<int64_t> csup;
    DBuf<unsigned> qcount, ccount;
    uint64_t qcap = 0, ccap = 0;

    void alloc(uint64_t qc, uint64_t cc) {
        qcap = qc;
        ccap = cc;
        qkv.alloc(2 * qc);
        qadj.alloc(qc);
        qlab.alloc(qc);
        qpat.alloc(qc);
        ckv.alloc(2 * cc);
        cinfo.alloc(cc);
        csup.alloc(cc);
        qcount.alloc(1);
        ccount.alloc(1);
    }
    // Replace the QP part by an empty table of qc slots (the code part stays).
    void take_qp(Tables& o) {
        qkv.swap(o.qkv);
        qadj.swap(o.qadj);
        qlab.swap(o.qlab);
        qpat.swap(o.qpat);
        qcount.swap(o.qcount);
        std::swap(qcap, o.qcap);
    }
    void reset_qp() {
        k_init_table<<<grid_for((int64_t)qcap, TPB), TPB, 0, stream()>>>(qkv.p, qcap);
        FSM_LAUNCH_CHECK();
        qadj.zero();
        qlab.zero();
        qpat.zero();
        qcount.zero();
    }
    void reset_codes() {
        k_init_table<<<grid_for((int64_t)ccap, TPB), TPB, 0, stream()>>>(ckv.p, ccap);
        FSM_LAUNCH_CHECK();
        cinfo.zero();
        csup.zero();
        ccount.zero();
    }
    void alloc_codes(uint64_t cc) {
        ccap = cc;
        ckv.alloc(2 * cc);
        cinfo.alloc(cc);
        csup.alloc(cc);
    }
};

struct Level {
    int n = 0;
    Tables tab;
    DBuf<int32_t> emb;       // rows of (n vertices, QP slot), frequent patterns only
    int64_t rows = 0;
    std::vector<std::pair<uint64_t, int64_t>> freq;   // (code, support), support >= t
    fsm_level_stats st{};
};

// Shapes chosen by fsm_tune_batch, used where a call leaves them at 0.
struct Tuning {
    std::atomic<int64_t> chunk_vertices{0};
    std::atomic<int32_t> tiles_per_wave{0};
};
Tuning g_tuning;

uint64_t pow2_at_least(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Two HIP events timing device work on one stream; inert (no events, 0 ms)
// when timing is off, as in calls that must not create runtime objects.
struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    Timer(bool on, hipStream_t st) : s(st) {
        if (!on) return;
        FSM_HIP(hipEventCreate(&a));
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            a = nullptr;
            fail(FSM_EDEVICE, "hipEventCreate failed");
        }
    }
    Timer(const Timer&) = delete;
    Timer& operator=(const Timer&) = delete;
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void start() {
        if (a) FSM_HIP(hipEventRecord(a, s));
    }
    float stop() {
        if (!a) return 0.f;
        FSM_HIP(hipEventRecord(b, s));
        ++host_syncs();
        FSM_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        FSM_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
};

// Captured join levels of one batched call: a stream of its own for the
// replays, and per level size a device descriptor and an instantiated
// graph of six kernel nodes: the table reset and the domain pass read their
// arguments from the descriptor; the canonical-form, merge, orbit-count and
// MNI nodes are the kernels of the eager path, whose arguments and grids
// are set per chunk on the instantiated graph (hipGraphExecKernelNodeSetParams)
// before it is replayed.
constexpr unsigned CAPTURE_GRID = 1u << 14;

template <int N>
void enqueue_level(hipStream_t s, LevelDesc* d, unsigned grid) {
    k_level_reset<<<CAPTURE_GRID, TPB, 0, s>>>(d);
    k_join_tiles_p<N, false><<<grid, TPB, 0, s>>>(&d->t);
    // placeholders: every replay sets these nodes' arguments first
    k_qp_canon<<<1, TPB, 0, s>>>(CanonArgs{});
    k_qp_merge<<<1, TPB, 0, s>>>(MergeArgs{});
    k_orbit_count<<<1, TPB, 0, s>>>(MniArgs{}, nullptr);
    k_mni<<<1, TPB, 0, s>>>(MniArgs{}, nullptr);
}

struct LevelGraphs {
    struct Entry {
        DBuf<LevelDesc> desc;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraphNode_t canon = nullptr, merge = nullptr, orbit = nullptr, mni = nullptr;
    };
    hipStream_t cs = nullptr;
    hipEvent_t ev = nullptr;
    std::map<std::array<uint64_t, 2>, std::unique_ptr<Entry>> cache;
    int32_t fallbacks = 0;
    int64_t replays = 0;

    LevelGraphs() = default;
    LevelGraphs(const LevelGraphs&) = delete;
    LevelGraphs& operator=(const LevelGraphs&) = delete;
    ~LevelGraphs() {
        for (auto& kv : cache) {
            if (kv.second->exec) (void)hipGraphExecDestroy(kv.second->exec);
            if (kv.second->graph) (void)hipGraphDestroy(kv.second->graph);
        }
        if (ev) (void)hipEventDestroy(ev);
        if (cs) (void)hipStreamDestroy(cs);
    }
    void init() {
        if (cs) return;
        FSM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        FSM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    // the graph of a level size, captured on first use
    Entry& get(int n, unsigned grid) {
        const std::array<uint64_t, 2> key{(uint64_t)n, (uint64_t)grid};
        auto it = cache.find(key);
        if (it != cache.end()) return *it->second;
        auto e = std::make_unique<Entry>();
        e->desc.alloc(1);
        FSM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        switch (n) {
            case 4: enqueue_level<4>(cs, e->desc.p, grid); break;
            case 5: enqueue_level<5>(cs, e->desc.p, grid); break;
            case 6: enqueue_level<6>(cs, e->desc.p, grid); break;
            default: {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(cs, &g);
                if (g) (void)hipGraphDestroy(g);
                fail(FSM_EINVAL, "no captured level of size %d", n);
            }
        }
        const hipError_t le = hipGetLastError();
        const hipError_t ce = hipStreamEndCapture(cs, &e->graph);
        if (le != hipSuccess || ce != hipSuccess)
            fail(FSM_EDEVICE, "capture of the size-%d level failed: %s", n,
                 hipGetErrorString(le != hipSuccess ? le : ce));
        // the nodes whose arguments change per chunk, found by their kernel
        size_t count = 0;
        FSM_HIP(hipGraphGetNodes(e->graph, nullptr, &count));
        std::vector<hipGraphNode_t> nodes(count);
        FSM_HIP(hipGraphGetNodes(e->graph, nodes.data(), &count));
        for (hipGraphNode_t nd : nodes) {
            hipGraphNodeType ty;
            FSM_HIP(hipGraphNodeGetType(nd, &ty));
            if (ty != hipGraphNodeTypeKernel) continue;
            hipKernelNodeParams kp{};
            FSM_HIP(hipGraphKernelNodeGetParams(nd, &kp));
            if (kp.func == reinterpret_cast<void*>(&k_qp_canon)) e->canon = nd;
            else if (kp.func == reinterpret_cast<void*>(&k_qp_merge)) e->merge = nd;
            else if (kp.func == reinterpret_cast<void*>(&k_orbit_count)) e->orbit = nd;
            else if (kp.func == reinterpret_cast<void*>(&k_mni)) e->mni = nd;
        }
        if (!e->canon || !e->merge || !e->orbit || !e->mni)
            fail(FSM_EDEVICE, "captured size-%d level: kernel nodes not found", n);
        FSM_HIP(hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0));
        Entry& ref = *e;
        cache.emplace(key, std::move(e));
        return ref;
    }
    // point a kernel node of the instantiated graph at new arguments
    static void set_node(hipGraphExec_t exec, hipGraphNode_t nd, void* func, unsigned blocks,
                         void** args) {
        hipKernelNodeParams kp{};
        kp.func = func;
        kp.gridDim = dim3(blocks);
        kp.blockDim = dim3(TPB);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        FSM_HIP(hipGraphExecKernelNodeSetParams(exec, nd, &kp));
    }
};

struct Miner {
    GraphView gv;
    const GraphView* g = &gv;
    fsm_options opt;
    hipStream_t st;
    std::vector<int64_t> tg;              // support threshold of each graph
    DBuf<int64_t> dtg;
    int F = 0;
    std::vector<int32_t> fvalue;          // frequent id -> caller label
    DBuf<int32_t> vf;                     // frequent id per vertex or -1
    DBuf<int32_t> frow, fcol;             // G_f
    int64_t fnnz = 0;
    DBuf<uint32_t> nhoff;
    DBuf<int32_t> nhtab;
    NbrHash nh() const { return NbrHash{nhoff.p, nhtab.p}; }
    // vertex-induced mode: tables of the edges outside G_f (empty: none)
    DBuf<uint32_t> xhoff;
    DBuf<int32_t> xhtab;
    NbrHash xh() const { return NbrHash{xhoff.p, xhtab.p}; }
    DBuf<uint64_t> mthr;            // matching sampling thresholds
    Sampling sampling() const {
        Sampling s;
        s.seed = opt.seed;
        s.mthr = mthr.p;
        return s;
    }
    void group_thresholds(int kind, int n, uint64_t cap, DBuf<uint64_t>& thr);
    SelArgs sel_args(int n) const;
    void st_pieces(int n, const Sampling& smp, DBuf<int64_t>& cnt, DBuf<int64_t>& off,
                   DBuf<uint64_t>& key, DBuf<uint8_t>& code);
    void neighbour_tables(const int32_t* row, const int32_t* col, DBuf<uint32_t>& off,
                          DBuf<int32_t>& tab);
    DBuf<int64_t> npieces;
    DBuf<int32_t> leafoff;
    DBuf<uint8_t> f3;
    DBuf<uint32_t> pool, ppool;     // QP-position bitmaps, pattern-orbit bitmaps
    uint64_t pool_words = 0, ppool_words = 0;
    uint64_t pool_budget = 0;     // bytes for the QP and pattern bitmap pools
    uint64_t released_pool_bytes = 0;   // pools released by the last level
    uint32_t pass_W = 0;          // current domain pass: words per bitmap,
    int32_t pass_rbase = 0;       // first rank of its slice,
    const int32_t* pass_porb = nullptr;        // its candidate bitmap map,
    unsigned long long* pass_qcnt = nullptr;   // its per-QP subgraph counts
    DBuf<int32_t> lrank;
    DBuf<uint32_t> vinfo;
    DBuf<Rec> drec;     // device copy of the recording context of the join
    Rec hrec{};
    DBuf<TileArgs> dtile;   // device copy of the domain pass's arguments
    TileArgs htile{};
    DBuf<SingleTileArgs> dstile;   // the same for the single-vertex domain pass
    SingleTileArgs hstile{};
    DBuf<unsigned long long> counters;   // [emitted, candidates, work queue, bytes]
    DBuf<uint32_t> flags;
    uint32_t W = 1;
    unsigned grid_persistent = 1024;
    bool timing = true;          // per-level HIP-event timings (off: 0 ms)
    LevelGraphs* lg = nullptr;   // batched calls: captured last join levels
    LevelDesc hdesc{};           // host copy of the descriptor being replayed
    int32_t captured = 0;        // levels of this pass run as graph replays
    Level lv[FSM_MAX_SIZE + 1];
    std::vector<fsm_result*> res;         // one per graph

    uint64_t qhint[FSM_MAX_SIZE + 1] = {};   // first QP table size per level (0: default)
    uint64_t chint[FSM_MAX_SIZE + 1] = {};   // captured levels: pattern table size
    const Model* model = nullptr;          // FSM_LEARNED: sizes the join tables
    std::vector<float> rx, rt;             // recorded work-item rows (features, targets)
    std::vector<int32_t> rl, rg;           // their join size and graph id

    // work items of the size-n join: features of every (parent QP, position)
    // with parent embeddings
    struct ItemRows {
        DBuf<float> x;
        DBuf<int32_t> item, graph;
        DBuf<unsigned> cnt;   // parent embeddings per parent QP slot
        int64_t rows = 0;
    };
    void item_rows(const Level& P, int n, ItemRows& IR);

    // Release the bitmap pools of the previous level and size the budget of
    // the next: QP and pattern bitmap pools may take 40% of the device
    // memory free now (of the scratch arena's free bytes in an
    // allocation-free call), counting the pools just released, which a
    // caching allocator may keep.
    void release_pools() {
        released_pool_bytes = (pool_words + ppool_words) * sizeof(uint32_t);
        pool.reset();
        ppool.reset();
        pool_words = ppool_words = 0;
    }
    void refresh_pool_budget() {
        const uint64_t held = (pool_words + ppool_words) * sizeof(uint32_t);
        release_pools();
        const uint64_t released = std::max(held, released_pool_bytes);
        size_t fr = 0, tot = 0;
        if (Arena* a = active_arena()) fr = a->free_bytes();
        else FSM_HIP(hipMemGetInfo(&fr, &tot));
        const uint64_t avail = active_arena() ? (uint64_t)fr : (uint64_t)fr + released;
        pool_budget = std::max<uint64_t>((uint64_t)(0.4 * (double)avail), (uint64_t)1 << 26);
        if (opt.pool_budget_mib > 0) pool_budget = (uint64_t)opt.pool_budget_mib << 20;
    }

    uint64_t qcap0() const {
        if (opt.force_overflow) return 2;
        uint64_t c = opt.hash_capacity_min > 0 ? (uint64_t)opt.hash_capacity_min : (1ull << 14);
        return pow2_at_least(c);
    }

    // Graph of a pattern key decoded on the host, checked against the
    // call's graphs: a key-layout mistake is reported, never used to index.
    size_t graph_of(uint64_t code, int n) const {
        const int32_t gi = checked_code_graph(code, n, g->ngraphs);
        if (gi < 0)
            fail(FSM_EDEVICE, "pattern key 0x%llx of size %d names no graph of the call (%d graphs)",
                 (unsigned long long)code, n, g->ngraphs);
        return (size_t)gi;
    }

    // Next QP table size after an overflow: 16 times larger, or less when
    // that table would not fit the free device memory (36 bytes per slot:
    // key, value, ordered adjacency and labels, pattern slot).
    uint64_t grown_qp_capacity(uint64_t qcap, int n) const {
        size_t fr = 0, tot = 0;
        if (Arena* a = active_arena()) fr = a->free_bytes();
        else FSM_HIP(hipMemGetInfo(&fr, &tot));
        const uint64_t room = (uint64_t)fr + qcap * 36ull;   // the old table is freed first
        uint64_t next = qcap * 16;
        while (next > qcap * 2 && next * 36ull > room / 2) next /= 2;
        if (fsm_trace())
            std::fprintf(stderr, "[fsm] size %d: QP table %llu -> %llu slots\n", n,
                         (unsigned long long)qcap, (unsigned long long)next);
        return next;
    }

    Rec rec(Level& L) {
        Rec R;
        R.q = {L.tab.qkv.p, L.tab.qcap - 1, L.tab.qadj.p, L.tab.qlab.p, L.tab.qpat.p,
               L.tab.qcount.p};
        R.c = {L.tab.ckv.p, L.tab.ccap - 1, L.tab.cinfo.p, L.tab.csup.p, L.tab.ccount.p};
        R.pool = {pool.p, lrank.p, pass_W, pass_rbase, pass_porb, pass_qcnt};
        R.flags = flags.p;
        R.n = L.n;
        return R;
    }

    // Bitmap words per (QP slot, position) in one pass: W (every rank at
    // once) unless the QP pool of `slots` slots would exceed half the pool
    // budget; then the ranks are covered in slices.  (The pattern pool takes
    // the other half: slices are merged into it in parts.)
    uint32_t slice_words(uint64_t slots, int n) const {
        const uint64_t per_word = slots * (uint64_t)n * sizeof(uint32_t);
        const uint64_t fit = pool_budget / 2 / (per_word ? per_word : 1);
        return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(W, fit));
    }

    void ensure_pool(DBuf<uint32_t>& p, uint64_t& have, uint64_t words) {
        if (words > have) {
            p.alloc(words);
            have = words;
        }
        FSM_HIP(hipMemsetAsync(p.p, 0, words * sizeof(uint32_t), st));
    }

    // Domain passes of one level.  Pass 0 inserts the quick patterns
    // (rerun with a larger table on overflow) and sets the domain bits of
    // the first rank slice; the canonical pass follows; later passes
    // repeat the enumeration for the remaining rank slices (lookups only).
    // After every pass the slice's QP bitmaps are merged into (pattern,
    // orbit) bitmaps and popcounted into per-orbit domain sizes; the MNI
    // support is their minimum.  Fills L.freq and the FREQ bits of the QP
    // table.  launch(R, pass) runs the level's domain kernel.
    template <class Launch>
    void domain_level(Level& L, Launch&& launch) {
        refresh_pool_budget();
        uint64_t qcap = L.tab.qcap ? L.tab.qcap
                                   : (opt.force_overflow ? qcap0() : std::max(qcap0(), qhint[L.n]));
        DBuf<unsigned long long> qcnt;
        const int64_t ranks = (int64_t)W * 32;
        uint32_t w0 = W;
        // child keys of a later join carry this level's QP slots in 29 bits;
        // the last level's slots go into no key (the joins' lane caches hold
        // slots in 32 bits, so a table has at most 2^31 slots)
        const bool parent_level = (opt.mode & FSM_SINGLE) ? L.n + 1 <= opt.max_size
                                                          : L.n + 2 <= opt.max_size;
        const uint64_t qcap_max = parent_level ? (1ull << 29) : (1ull << 31);
        for (int attempt = 0;; ++attempt) {
            L.st.domain_passes = attempt + 1;
            L.st.qp_capacity = (int64_t)qcap;
            if (qcap > qcap_max)
                fail(FSM_EOVERFLOW, "more than %llu quick patterns at size %d%s",
                     (unsigned long long)(qcap_max / 2), L.n,
                     parent_level ? " (a later join keys children by 29-bit parent slots)" : "");
            if (L.tab.qcap != qcap) L.tab.alloc(qcap, 1);
            L.tab.reset_qp();
            w0 = slice_words(qcap, L.n);
            pass_W = w0;
            pass_rbase = 0;
            ensure_pool(pool, pool_words, qcap * (uint64_t)L.n * w0);
            // more slices to come: count the subgraphs of every QP
            if ((int64_t)w0 * 32 < ranks) {
                qcnt.alloc(qcap);
                qcnt.zero();
                pass_qcnt = qcnt.p;
            }
            counters.zero();
            flags.zero();
            launch(rec(L), 0);
            pass_qcnt = nullptr;
            const uint32_t f = scalar_to_host(flags.p);
            if (fsm_trace())
                std::fprintf(stderr, "[fsm] size %d pass 0 attempt %d: qp capacity %llu, "
                             "%u of %u words, flags %u\n", L.n, attempt,
                             (unsigned long long)qcap, w0, W, f);
            if (f & (ERR_MISSING | ERR_FILL))
                fail(FSM_EDEVICE, "internal consistency check failed at size %d (flags %u)", L.n, f);
            if (!(f & OVF_QP)) break;
            if (attempt >= (opt.force_overflow ? 16 : 8))
                fail(FSM_EOVERFLOW, "QP table kept overflowing at size %d", L.n);
            qcap = std::min(grown_qp_capacity(qcap, L.n), std::max(qcap * 2, qcap_max));
        }
        std::vector<unsigned long long> cnt;
        to_host(cnt, counters.p, 4);
        L.st.emitted = (int64_t)cnt[0];
        L.st.candidates = (int64_t)cnt[1];
        L.st.algorithmic_bytes = (int64_t)cnt[3];
        const unsigned nqp = scalar_to_host(L.tab.qcount.p);
        L.st.quick_patterns = nqp;
        // canonical forms: pattern table sized for every QP being its own pattern
        uint64_t ccap = opt.force_overflow
                            ? 2
                            : pow2_at_least(std::max<uint64_t>(
                                  2ull * nqp + 16,
                                  (uint64_t)std::max<int64_t>(opt.pattern_capacity_min, 16)));
        for (int attempt = 0;; ++attempt) {
            L.tab.alloc_codes(ccap);
            L.tab.reset_codes();
            flags.zero();
            CanonArgs ca{{L.tab.qkv.p, L.tab.qcap - 1, L.tab.qadj.p, L.tab.qlab.p, L.tab.qpat.p,
                          L.tab.qcount.p},
                         {L.tab.ckv.p, L.tab.ccap - 1, L.tab.cinfo.p, L.tab.csup.p,
                          L.tab.ccount.p},
                         flags.p, L.n, L.tab.qcap, (uint64_t)g->ngraphs};
            k_qp_canon<<<grid_for((int64_t)L.tab.qcap, TPB), TPB, 0, st>>>(ca);
            FSM_LAUNCH_CHECK();
            // one canonical form per quick pattern (Section 4.4: one
            // isomorphism computation per quick-pattern group)
            L.st.canonical_forms += nqp;
            const uint32_t cf = scalar_to_host(flags.p);
            if (cf & ERR_GRAPH)
                fail(FSM_EDEVICE, "a quick pattern at size %d names no graph of the call", L.n);
            if (cf & ERR_BATCH)
                fail(FSM_EUNSUPPORTED, "batches of several graphs support sizes up to 6");
            if (!(cf & OVF_CODE)) break;
            if (attempt >= (opt.force_overflow ? 16 : 4))
                fail(FSM_EOVERFLOW, "pattern table overflow at size %d", L.n);
            ccap *= 4;
        }
        const unsigned npat = scalar_to_host(L.tab.ccount.p);
        L.st.patterns = npat;
        QPTab q{L.tab.qkv.p, L.tab.qcap - 1, L.tab.qadj.p, L.tab.qlab.p, L.tab.qpat.p,
                L.tab.qcount.p};
        DBuf<int64_t> ocnt((size_t)(ccap * (uint64_t)L.n));
        ocnt.zero();
        DBuf<uint64_t> okey(npat ? npat : 1);
        DBuf<int64_t> osup(npat ? npat : 1);
        DBuf<unsigned> on(1);
        on.zero();
        const CodeTab ct{L.tab.ckv.p, L.tab.ccap - 1, L.tab.cinfo.p, L.tab.csup.p, L.tab.ccount.p};
        // merge and count the slice of the pass just run (wr words per QP
        // bitmap), in parts whose pattern bitmaps fit the budget
        auto reduce_slice = [&](uint32_t wr) {
            const uint64_t per_word = ccap * (uint64_t)L.n * sizeof(uint32_t);
            const uint32_t part = (uint32_t)std::max<uint64_t>(
                1, std::min<uint64_t>(wr, pool_budget / 2 / (per_word ? per_word : 1)));
            for (uint32_t off = 0; off < wr; off += part) {
                const uint32_t len = std::min(part, wr - off);
                ensure_pool(ppool, ppool_words, ccap * (uint64_t)L.n * len);
                MergeArgs ma{q, pool.p, ppool.p, wr, off, len, L.n, L.tab.qcap * (uint64_t)L.n};
                k_qp_merge<<<grid_for((int64_t)ma.items, TPB / 64, 1u << 16), TPB, 0, st>>>(ma);
                FSM_LAUNCH_CHECK();
                MniArgs m{ct, {ppool.p, lrank.p, len, 0}, L.n, L.tab.ccap, okey.p, osup.p, on.p,
                          npat};
                k_orbit_count<<<grid_for((int64_t)L.tab.ccap, TPB / 64, 1u << 16), TPB, 0, st>>>(
                    m, ocnt.p);
                FSM_LAUNCH_CHECK();
            }
        };
        reduce_slice(w0);
        // more slices to come: candidate patterns (subgraphs x n >= t) and a
        // dense index of their (pattern, orbit) bitmaps
        DBuf<int64_t> cand, poidx, pomap;
        int64_t npo = -1;
        if ((int64_t)w0 * 32 < ranks) {
            DBuf<unsigned long long> pcnt(ccap);
            pcnt.zero();
            k_pattern_counts<<<grid_for((int64_t)qcap, TPB), TPB, 0, st>>>(q, qcap, qcnt.p, pcnt.p);
            FSM_LAUNCH_CHECK();
            const uint64_t items = ccap * (uint64_t)L.n;
            cand.alloc(items);
            poidx.alloc(items);
            flags.zero();
            k_candidate_flags<<<grid_for((int64_t)items, TPB), TPB, 0, st>>>(
                ct, ccap, L.n, pcnt.p, dtg.p, g->ngraphs, cand.p, flags.p);
            FSM_LAUNCH_CHECK();
            if (scalar_to_host(flags.p) & ERR_GRAPH)
                fail(FSM_EDEVICE, "a pattern at size %d names no graph of the call", L.n);
            npo = scan_exclusive(cand.p, poidx.p, (int64_t)items);
            if (npo >= (int64_t)INT32_MAX)
                fail(FSM_EUNSUPPORTED, "more than 2^31 candidate orbit domains at size %d", L.n);
            pomap.alloc((size_t)std::max<int64_t>(npo, 1));
            k_po_map<<<grid_for((int64_t)items, TPB), TPB, 0, st>>>(cand.p, poidx.p, items, pomap.p);
            FSM_LAUNCH_CHECK();
            qcnt.reset();
        }
        // more slices to come: move the QPs into a table sized for them
        // (an overflow rerun grows the table 16-fold), so that every later
        // slice can be wider
        if ((int64_t)w0 * 32 < ranks) {
            const uint64_t want = pow2_at_least(2ull * nqp + 16);
            if (want < qcap) {
                Tables nt;
                nt.alloc(want, 1);
                nt.reset_qp();
                flags.zero();
                const QPTab to{nt.qkv.p, want - 1, nt.qadj.p, nt.qlab.p, nt.qpat.p, nt.qcount.p};
                k_qp_rehash<<<grid_for((int64_t)qcap, TPB), TPB, 0, st>>>(q, qcap, to, flags.p);
                FSM_LAUNCH_CHECK();
                if (scalar_to_host(flags.p) & OVF_QP)
                    fail(FSM_EDEVICE, "QP table compaction overflowed at size %d", L.n);
                L.tab.take_qp(nt);
                qcap = want;
                q = QPTab{L.tab.qkv.p, L.tab.qcap - 1, L.tab.qadj.p, L.tab.qlab.p, L.tab.qpat.p,
                          L.tab.qcount.p};
            }
        }
        int slices = 1;
        if (npo >= 0) {
            // direct slices: bits go straight into the candidate bitmaps
            DBuf<int32_t> porb((size_t)qcap * L.n);
            k_qp_orbit_map<<<grid_for((int64_t)(qcap * L.n), TPB), TPB, 0, st>>>(
                q, qcap, L.n, cand.p, poidx.p, porb.p);
            FSM_LAUNCH_CHECK();
            const uint64_t per_word = (uint64_t)std::max<int64_t>(npo, 1) * sizeof(uint32_t);
            for (int64_t lo = (int64_t)w0 * 32; npo > 0 && lo < ranks; ++slices) {
                const uint32_t wr = (uint32_t)std::max<uint64_t>(
                    1, std::min<uint64_t>((uint64_t)(ranks - lo + 31) / 32,
                                          pool_budget / 2 / per_word));
                pass_W = wr;
                pass_rbase = (int32_t)lo;
                pass_porb = porb.p;
                ensure_pool(pool, pool_words, (uint64_t)npo * wr);
                counters.zero();
                flags.zero();
                launch(rec(L), slices);
                pass_porb = nullptr;
                const uint32_t f = scalar_to_host(flags.p);
                if (f) fail(FSM_EDEVICE, "domain slice %d of size %d failed (flags %u)", slices, L.n, f);
                k_dense_count<<<grid_for(npo, TPB / 64, 1u << 16), TPB, 0, st>>>(
                    pool.p, (uint64_t)npo, wr, pomap.p, ocnt.p);
                FSM_LAUNCH_CHECK();
                lo += (int64_t)wr * 32;
                if (fsm_trace())
                    std::fprintf(stderr, "[fsm] size %d direct slice %d: %u words, ranks up to "
                                 "%lld of %lld, %lld candidate orbit bitmaps of %u patterns\n",
                                 L.n, slices, wr, (long long)lo, (long long)ranks,
                                 (long long)npo, npat);
            }
        }
        for (int64_t lo = (int64_t)w0 * 32; npo < 0 && lo < ranks; ++slices) {
            const uint32_t wr = slice_words(qcap, L.n);
            pass_W = wr;
            pass_rbase = (int32_t)lo;
            ensure_pool(pool, pool_words, qcap * (uint64_t)L.n * wr);
            counters.zero();
            flags.zero();
            launch(rec(L), slices);
            const uint32_t f = scalar_to_host(flags.p);
            if (f) fail(FSM_EDEVICE, "domain slice %d of size %d failed (flags %u)", slices, L.n, f);
            reduce_slice(wr);
            lo += (int64_t)wr * 32;
            if (fsm_trace())
                std::fprintf(stderr, "[fsm] size %d slice %d: %u words, ranks up to %lld of "
                             "%lld, %u QPs, %u patterns\n", L.n, slices, wr, (long long)lo,
                             (long long)ranks, nqp, npat);
        }
        L.st.rank_slices = slices;
        pass_W = W;
        pass_rbase = 0;
        MniArgs m{ct, {ppool.p, lrank.p, W, 0}, L.n, L.tab.ccap, okey.p, osup.p, on.p, npat};
        k_mni<<<grid_for((int64_t)L.tab.ccap, TPB), TPB, 0, st>>>(m, ocnt.p);
        FSM_LAUNCH_CHECK();
        flags.zero();
        k_mark_frequent<<<grid_for((int64_t)L.tab.qcap, TPB), TPB, 0, st>>>(
            q, L.tab.qcap, L.tab.ckv.p, L.tab.csup.p, dtg.p, g->ngraphs, L.n, flags.p);
        FSM_LAUNCH_CHECK();
        std::vector<uint64_t> hk;
        std::vector<int64_t> hs;
        to_host(hk, okey.p, npat);
        to_host(hs, osup.p, npat);
        if (scalar_to_host(flags.p) & ERR_GRAPH)
            fail(FSM_EDEVICE, "a pattern at size %d names no graph of the call", L.n);
        L.freq.clear();
        for (unsigned i = 0; i < npat; ++i)
            if (hs[i] >= tg[graph_of(hk[i], L.n)]) L.freq.emplace_back(hk[i], hs[i]);
        std::sort(L.freq.begin(), L.freq.end());
        L.st.frequent = (int64_t)L.freq.size();
        release_pools();
    }

    // count / scan / fill of the frequent embeddings of level L
    template <class Launch>
    void materialize(Level& L, int64_t nwork, Launch&& launch) {
        DBuf<int64_t> counts((size_t)(nwork > 0 ? nwork : 1));
        counts.zero();
        flags.zero();
        counters.zero();
        launch(MODE_COUNT, counts.p, (const int64_t*)nullptr, (int32_t*)nullptr, (int64_t)0);
        int64_t total = scan_exclusive(counts.p, counts.p, nwork);
        L.rows = total;
        L.emb.alloc((size_t)(total * (L.n + 1) + 1));
        counters.zero();
        if (total > 0) launch(MODE_FILL, (int64_t*)nullptr, (const int64_t*)counts.p, L.emb.p, total);
        uint32_t f = scalar_to_host(flags.p);
        if (f) fail(FSM_EDEVICE, "materialisation of size %d failed (flags %u)", L.n, f);
        L.st.stored = total;
    }

    struct Groups {
        DBuf<int32_t> gk, glist;
        DBuf<int64_t> goff, gcnt, toff;
        int64_t ngroups = 0, ntiles = 0;
        int tile_p = TILE_P_MAX;
        const int64_t* pieces = nullptr;   // candidates per joining vertex
    };
    void build_groups(const Level& P, int M, int64_t nwork, Groups& G,
                      const int64_t* pieces = nullptr);
    void sorted_pieces(DBuf<int64_t>& poff, DBuf<uint64_t>& key, DBuf<uint8_t>& code);
    void order_groups(const Level& P, int M, const ItemRows& IR, const float* y, Groups& G);
    void proposal_thresholds(const ItemRows& IR, const float* y, int64_t nitems,
                             DBuf<uint64_t>& thr);

    template <class MakeArgs>
    bool captured_level(Level& L, MakeArgs&& make_args);
    void run();
    void level2();
    void build_gf();
    void level3();
    void join(int n);
    void join_single(int n);
    void emit_results();
};

// The last join level of a batch chunk as one graph replay.  Tables are
// sized up front (the level's hint: cost model or earlier chunks) and the
// code table as large as the QP table, so only a QP-table overflow can
// spoil the replay; then the level is rerun with eager launches from a
// grown table.  Returns false when the level must run eagerly.
template <class MakeArgs>
bool Miner::captured_level(Level& L, MakeArgs&& make_args) {
    const int n = L.n;
    refresh_pool_budget();
    const uint64_t qcap = opt.force_overflow ? qcap0() : std::max(qcap0(), qhint[n]);
    // pattern table: the density earlier chunks needed, never above the QP
    // table (every pattern has a quick pattern)
    const uint64_t ccap = opt.force_overflow ? 2 : std::min(qcap, std::max<uint64_t>(chint[n], 1024));
    const uint32_t Wq = W;
    const uint64_t words = qcap * (uint64_t)n * Wq;
    const uint64_t pwords = ccap * (uint64_t)n * Wq;
    if (words * sizeof(uint32_t) > pool_budget / 2 || qcap > (1ull << 29)) return false;
    lg->init();
    LevelGraphs::Entry& e = lg->get(n, grid_persistent);
    L.tab.alloc(qcap, ccap);
    if (words > pool_words) { pool.alloc(words); pool_words = words; }
    if (pwords > ppool_words) { ppool.alloc(pwords); ppool_words = pwords; }
    DBuf<int64_t> ocnt((size_t)(ccap * n));
    DBuf<uint64_t> okey((size_t)ccap);
    DBuf<int64_t> osup((size_t)ccap);
    DBuf<unsigned> on(1);
    pass_W = Wq;
    pass_rbase = 0;
    pass_porb = nullptr;
    pass_qcnt = nullptr;
    const Rec R = rec(L);
    pass_W = W;
    LevelDesc& d = hdesc;
    d.t = make_args(R);
    const QPTab q{L.tab.qkv.p, qcap - 1, L.tab.qadj.p, L.tab.qlab.p, L.tab.qpat.p, L.tab.qcount.p};
    const CodeTab ct{L.tab.ckv.p, ccap - 1, L.tab.cinfo.p, L.tab.csup.p, L.tab.ccount.p};
    d.ca = CanonArgs{q, ct, flags.p, n, qcap, (uint64_t)g->ngraphs};
    d.ma = MergeArgs{q, pool.p, ppool.p, Wq, 0, Wq, n, qcap * (uint64_t)n};
    d.m = MniArgs{ct, {ppool.p, lrank.p, Wq, 0}, n, ccap, okey.p, osup.p, on.p, (unsigned)ccap};
    d.ocnt = ocnt.p;
    d.pool = pool.p;
    d.ppool = ppool.p;
    d.counters = counters.p;
    d.flags = flags.p;
    d.qslots = qcap;
    d.cslots = ccap;
    d.pool_words = words;
    d.ppool_words = pwords;
    d.ocnt_items = ccap * (uint64_t)n;
    FSM_HIP(hipMemcpyAsync(e.desc.p, &d, sizeof(LevelDesc), hipMemcpyHostToDevice, st));
    {
        void* ca[] = {&d.ca};
        void* ma[] = {&d.ma};
        void* oa[] = {&d.m, &d.ocnt};
        void* na[] = {&d.m, &d.ocnt};
        LevelGraphs::set_node(e.exec, e.canon, reinterpret_cast<void*>(&k_qp_canon),
                              grid_for((int64_t)qcap, TPB), ca);
        LevelGraphs::set_node(e.exec, e.merge, reinterpret_cast<void*>(&k_qp_merge),
                              grid_for((int64_t)(qcap * n), TPB / 64, 1u << 16), ma);
        LevelGraphs::set_node(e.exec, e.orbit, reinterpret_cast<void*>(&k_orbit_count),
                              grid_for((int64_t)ccap, TPB / 64, 1u << 16), oa);
        LevelGraphs::set_node(e.exec, e.mni, reinterpret_cast<void*>(&k_mni),
                              grid_for((int64_t)ccap, TPB), na);
    }
    FSM_HIP(hipEventRecord(lg->ev, st));
    FSM_HIP(hipStreamWaitEvent(lg->cs, lg->ev, 0));
    {
        Timer gt(timing, lg->cs);
        gt.start();
        FSM_HIP(hipGraphLaunch(e.exec, lg->cs));
        L.st.join_ms = gt.stop();
    }
    sync_stream(lg->cs);
    ++lg->replays;
    const uint32_t f = scalar_to_host(flags.p);
    if (f & (ERR_MISSING | ERR_FILL))
        fail(FSM_EDEVICE, "internal consistency check failed at size %d (flags %u)", n, f);
    if (f & ERR_GRAPH) fail(FSM_EDEVICE, "a quick pattern at size %d names no graph of the call", n);
    if (f & ERR_BATCH) fail(FSM_EUNSUPPORTED, "batches of several graphs support sizes up to 6");
    if (f & (OVF_QP | OVF_CODE)) {
        if (f & OVF_QP) qhint[n] = grown_qp_capacity(qcap, n);
        if (f & OVF_CODE) chint[n] = std::min(qcap, ccap * 4);
        L.tab = Tables();
        ++lg->fallbacks;
        return false;
    }
    std::vector<unsigned long long> cnt;
    to_host(cnt, counters.p, 4);
    const unsigned nqp = scalar_to_host(L.tab.qcount.p);
    const unsigned npat = scalar_to_host(on.p);
    L.st.domain_passes = 1;
    L.st.qp_capacity = (int64_t)qcap;
    L.st.emitted = (int64_t)cnt[0];
    L.st.candidates = (int64_t)cnt[1];
    L.st.algorithmic_bytes = (int64_t)cnt[3];
    L.st.quick_patterns = nqp;
    L.st.canonical_forms = nqp;
    L.st.patterns = npat;
    L.st.rank_slices = 1;
    std::vector<uint64_t> hk;
    std::vector<int64_t> hs;
    to_host(hk, okey.p, npat);
    to_host(hs, osup.p, npat);
    L.freq.clear();
    for (unsigned i = 0; i < npat; ++i)
        if (hs[i] >= tg[graph_of(hk[i], n)]) L.freq.emplace_back(hk[i], hs[i]);
    std::sort(L.freq.begin(), L.freq.end());
    L.st.frequent = (int64_t)L.freq.size();
    release_pools();
    ++captured;
    return true;
}

void Miner::level2() {
    Level& L = lv[2];
    L.n = 2;
    auto launch = [&](Rec R, int) {
        L2Args a{g->row, g->col, vf.p, g->vg, g->n, R, counters.p, nullptr, nullptr, nullptr, 0};
        k_level2<MODE_DOMAIN><<<grid_persistent, TPB, 0, st>>>(a);
        FSM_LAUNCH_CHECK();
    };
    domain_level(L, launch);
}

void Miner::build_gf() {
    // frequent labelled edges of every graph from the size-2 results
    std::vector<uint8_t> f2((size_t)g->ngraphs * F * F, 0);
    for (auto& kv : lv[2].freq) {
        const int a = code_label(kv.first, 2, 0), b = code_label(kv.first, 2, 1);
        uint8_t* t = f2.data() + graph_of(kv.first, 2) * F * F;
        t[(size_t)a * F + b] = t[(size_t)b * F + a] = 1;
    }
    DBuf<uint8_t> df2(f2.size());
    to_device(df2.p, f2.data(), f2.size());
    const int64_t n = g->n;
    DBuf<int64_t> cnt((size_t)n + 1);
    k_gf_count<<<grid_for(n, TPB), TPB, 0, st>>>(g->row, g->col, vf.p, g->vg, n, df2.p, F, 1,
                                                  cnt.p);
    FSM_LAUNCH_CHECK();
    fnnz = scan_exclusive(cnt.p, cnt.p, n);
    frow.alloc((size_t)n + 1);
    fcol.alloc((size_t)(fnnz > 0 ? fnnz : 1));
    k_gf_fill<<<grid_for(n + 1, TPB), TPB, 0, st>>>(g->row, g->col, vf.p, g->vg, n, df2.p, F, 1,
                                                     cnt.p, fnnz, frow.p, fcol.p);
    FSM_LAUNCH_CHECK();
    // per-vertex neighbour hash tables (load <= 1/2) and piece counts
    neighbour_tables(frow.p, fcol.p, nhoff, nhtab);
    if (opt.mode & FSM_INDUCED) {
        // the graph edges between frequent-label vertices outside G_f
        k_gf_count<<<grid_for(n, TPB), TPB, 0, st>>>(g->row, g->col, vf.p, g->vg, n, df2.p, F,
                                                      0, cnt.p);
        FSM_LAUNCH_CHECK();
        const int64_t xnnz = scan_exclusive(cnt.p, cnt.p, n);
        if (xnnz > 0) {
            DBuf<int32_t> xrow((size_t)n + 1), xcol((size_t)xnnz);
            k_gf_fill<<<grid_for(n + 1, TPB), TPB, 0, st>>>(g->row, g->col, vf.p, g->vg, n,
                                                             df2.p, F, 0, cnt.p, xnnz, xrow.p,
                                                             xcol.p);
            FSM_LAUNCH_CHECK();
            neighbour_tables(xrow.p, xcol.p, xhoff, xhtab);
        }
    }
    npieces.alloc((size_t)n);
    leafoff.alloc((size_t)(fnnz > 0 ? fnnz : 1));
    k_pieces<<<grid_for(n, TPB), TPB, 0, st>>>(frow.p, fcol.p, n, npieces.p, leafoff.p);
    FSM_LAUNCH_CHECK();
    for (fsm_result* r : res) r->stats.filtered_edges = fnnz / 2;
}

// Per-vertex two-choice cuckoo neighbour tables of the CSR (row, col):
// buckets of two slots, grown for the vertices whose insertion failed.
void Miner::neighbour_tables(const int32_t* row, const int32_t* col, DBuf<uint32_t>& off,
                             DBuf<int32_t>& tab) {
    const int64_t n = g->n;
    DBuf<int64_t> nb((size_t)n + 1);
    DBuf<uint8_t> grow((size_t)n), failed((size_t)n);
    DBuf<unsigned> nfailed(1), big(1);
    grow.zero();
    for (int attempt = 0;; ++attempt) {
        big.zero();
        k_nbr_sizes<<<grid_for(n, TPB), TPB, 0, st>>>(row, n, grow.p, nb.p, big.p);
        FSM_LAUNCH_CHECK();
        const int64_t total = scan_exclusive(nb.p, nb.p, n);
        if (total >= (int64_t)UINT32_MAX)
            fail(FSM_EUNSUPPORTED, "neighbour tables exceed 2^32 buckets");
        if (scalar_to_host(big.p))
            fail(FSM_EUNSUPPORTED, "a vertex's neighbour table exceeds %lld buckets",
                 (long long)NB_MAX);
        off.alloc((size_t)n + 1);
        tab.alloc((size_t)(total > 0 ? total : 1));
        failed.zero();
        nfailed.zero();
        k_nbr_fill<<<grid_for(n + 1, TPB), TPB, 0, st>>>(row, col, n, nb.p, total, off.p, tab.p,
                                                        failed.p, nfailed.p);
        FSM_LAUNCH_CHECK();
        if (scalar_to_host(nfailed.p) == 0) break;
        if (attempt >= 8) fail(FSM_EDEVICE, "neighbour table construction kept failing");
        k_grow_failed<<<grid_for(n, TPB), TPB, 0, st>>>(failed.p, n, grow.p);
        FSM_LAUNCH_CHECK();
    }
}

// Thresholds of every vertex's group of a fixed-size sample (Section 5):
// kind SEL_MATCH (size-3 subgraphs credited to the vertex), SEL_PIECES
// (stored size-3 subgraphs containing the joining vertex, size-n join) or
// SEL_EDGES (its G_f edges at a size-n edge join); cap members per group.
SelArgs Miner::sel_args(int n) const {
    SelArgs a;
    a.row = frow.p; a.col = fcol.p; a.leafoff = leafoff.p; a.npieces = npieces.p;
    a.vinfo = vinfo.p; a.vg = g->vg; a.f3 = f3.p; a.F = F;
    a.nh = nh(); a.xh = xh();
    a.induced = (opt.mode & FSM_INDUCED) ? 1 : 0;
    a.smp = sampling();
    a.n = n; a.groups = g->n; a.cap = 0; a.thr = nullptr;
    return a;
}

// ST: every joining vertex's kept pieces at the size-n join as lists (key
// order at size 5, as the join's size-5 filter needs); left empty (the join
// then decodes and tests every piece) beyond 2^31 pieces.
void Miner::st_pieces(int n, const Sampling& smp, DBuf<int64_t>& cnt, DBuf<int64_t>& off,
                      DBuf<uint64_t>& key, DBuf<uint8_t>& code) {
    const int64_t nv = g->n;
    SelArgs a = sel_args(n);
    a.smp = smp;
    cnt.alloc((size_t)nv);
    off.alloc((size_t)nv + 1);
    k_st_pieces<<<grid_for(nv, TPB / 64), TPB, 0, st>>>(a, nullptr, cnt.p, nullptr, nullptr);
    FSM_LAUNCH_CHECK();
    const int64_t total = scan_exclusive(cnt.p, off.p, nv);
    if (total >= (int64_t)INT32_MAX) {
        cnt.reset();
        off.reset();
        return;
    }
    FSM_HIP(hipMemcpyAsync(off.p + nv, &total, sizeof(int64_t), hipMemcpyHostToDevice, st));
    const size_t len = (size_t)std::max<int64_t>(total, 1);
    key.alloc(len);
    code.alloc(len);
    if (n != 5) {
        k_st_pieces<<<grid_for(nv, TPB / 64), TPB, 0, st>>>(a, off.p, nullptr, key.p, code.p);
        FSM_LAUNCH_CHECK();
        return;
    }
    DBuf<uint64_t> k0(len);
    DBuf<uint8_t> c0(len);
    k_st_pieces<<<grid_for(nv, TPB / 64), TPB, 0, st>>>(a, off.p, nullptr, k0.p, c0.p);
    FSM_LAUNCH_CHECK();
    if (total > 0) {
        DBuf<int32_t> off32((size_t)nv + 1);
        k_offsets32<<<grid_for(nv + 1, TPB), TPB, 0, st>>>(off.p, nv + 1, off32.p);
        FSM_LAUNCH_CHECK();
        sort_segments(k0.p, key.p, c0.p, code.p, (int)total, (int)nv, off32.p);
    }
}

void Miner::group_thresholds(int kind, int n, uint64_t cap, DBuf<uint64_t>& thr) {
    thr.alloc((size_t)g->n);
    SelArgs a = sel_args(n);
    a.cap = cap;
    a.thr = thr.p;
    const unsigned grid = grid_for(g->n, 1, 1u << 16);
    switch (kind) {
        case SEL_PIECES: k_group_select<SEL_PIECES><<<grid, SEL_TPB, 0, st>>>(a); break;
        case SEL_EDGES: k_group_select<SEL_EDGES><<<grid, SEL_TPB, 0, st>>>(a); break;
        default: k_group_select<SEL_MATCH><<<grid, SEL_TPB, 0, st>>>(a); break;
    }
    FSM_LAUNCH_CHECK();
}

void Miner::level3() {
    Level& L = lv[3];
    L.n = 3;
    // matching sampling: t subgraphs kept per credited vertex (Section 5)
    if (opt.match_threshold > 0) group_thresholds(SEL_MATCH, 3, (uint64_t)opt.match_threshold, mthr);
    auto launch = [&](Rec R, int) {
        L3Args a{frow.p, fcol.p, vf.p, g->vg, g->n, nh(), R, counters.p,
                 nullptr, nullptr, nullptr, 0};
        a.induced = (opt.mode & FSM_INDUCED) ? 1 : 0;
        a.xh = xh();
        a.smp = sampling();
        k_level3<MODE_DOMAIN><<<grid_persistent, TPB, 0, st>>>(a);
        FSM_LAUNCH_CHECK();
    };
    domain_level(L, launch);
    // rooted frequent size-3 table for the joins and the pruning
    const size_t FF = (size_t)F * F * F;
    std::vector<uint8_t> t2(2 * FF * (size_t)g->ngraphs, 0);
    for (auto& kv : L.freq) {
        const uint64_t code = kv.first;
        uint8_t* t = t2.data() + 2 * FF * graph_of(code, 3);
        int l0 = code_label(code, 3, 0), l1 = code_label(code, 3, 1), l2 = code_label(code, 3, 2);
        const uint32_t seq = (uint32_t)(code & 7u);   // bits: (0,1) (0,2) (1,2)
        int ls[3] = {l0, l1, l2};
        if (seq == 7u) {
            int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
            for (auto& pm : perm)
                t[FF + ((size_t)ls[pm[0]] * F + ls[pm[1]]) * F + ls[pm[2]]] = 1;
        } else {
            int c = seq == 6u ? 0 : (seq == 5u ? 1 : 2);   // the vertex on both edges
            int x = (c + 1) % 3, y = (c + 2) % 3;
            t[((size_t)ls[c] * F + ls[x]) * F + ls[y]] = 1;
            t[((size_t)ls[c] * F + ls[y]) * F + ls[x]] = 1;
        }
    }
    f3.alloc(t2.size());
    to_device(f3.p, t2.data(), t2.size());
}

// Group the work items (p, i) of a join by (p[i], parent QP, i) and count
// the (parents x pieces) tiles of every group.
// pieces: candidates per joining vertex (null: its size-3 piece slots)
void Miner::build_groups(const Level& P, int M, int64_t nwork, Groups& G,
                         const int64_t* pieces) {
    if (nwork > (int64_t)INT32_MAX * M)
        fail(FSM_EUNSUPPORTED, "more than 2^31-1 parent embeddings");
    G.pieces = pieces ? pieces : npieces.p;
    const int64_t n = g->n;
    uint64_t cap = std::min<uint64_t>(
        pow2_at_least((uint64_t)std::min<int64_t>(nwork, n * 16) * 2 + 16), 1ull << 32);
    DBuf<uint32_t> wslot((size_t)nwork);
    DBuf<uint64_t> kv;
    DBuf<unsigned> cnt(1);
    DBuf<unsigned long long> kpar((size_t)n);
    // sub-groups (k, parent QP, position) and per-key work-item counts
    for (int attempt = 0;; ++attempt) {
        kv.alloc(2 * cap);
        k_init_table<<<grid_for((int64_t)cap, TPB), TPB, 0, st>>>(kv.p, cap);
        FSM_LAUNCH_CHECK();
        cnt.zero();
        flags.zero();
        GroupBuild b{P.emb.p, M, nwork, kv.p, cap - 1, wslot.p, cnt.p, flags.p};
        k_group_insert<<<grid_for(nwork / M, TPB), TPB, 0, st>>>(b);
        FSM_LAUNCH_CHECK();
        if (!(scalar_to_host(flags.p) & OVF_QP)) break;
        // slots are stored as 32-bit words
        if (attempt >= 6 || cap * 4 > (1ull << 32))
            fail(FSM_EOVERFLOW, "join grouping table overflow (%llu slots)",
                 (unsigned long long)cap);
        cap *= 4;
    }
    // parent range of every key, then each sub-group's run inside it
    DBuf<int64_t> kpoff((size_t)n);
    kpar.zero();
    k_key_counts<<<grid_for((int64_t)cap, TPB), TPB, 0, st>>>(kv.p, cap, kpar.p);
    FSM_LAUNCH_CHECK();
    scan_exclusive(reinterpret_cast<int64_t*>(kpar.p), kpoff.p, n);
    DBuf<unsigned long long> kcursor((size_t)n);
    FSM_HIP(hipMemcpyAsync(kcursor.p, kpoff.p, sizeof(int64_t) * (size_t)n,
                           hipMemcpyDeviceToDevice, st));
    DBuf<int64_t> gid(cap);
    k_group_flags<<<grid_for((int64_t)cap, TPB), TPB, 0, st>>>(kv.p, cap, gid.p);
    FSM_LAUNCH_CHECK();
    const int64_t nsub = scan_exclusive(gid.p, gid.p, (int64_t)cap);
    DBuf<unsigned long long> soff((size_t)std::max<int64_t>(nsub, 1));
    k_group_place<<<grid_for((int64_t)cap, TPB), TPB, 0, st>>>(kv.p, cap, gid.p, kcursor.p,
                                                              soff.p);
    FSM_LAUNCH_CHECK();
    G.glist.alloc((size_t)nwork);
    k_group_fill<<<grid_for(nwork / M, TPB), TPB, 0, st>>>(nwork, M, wslot.p, gid.p, soff.p,
                                                       G.glist.p);
    FSM_LAUNCH_CHECK();
    // key groups = vertices with work, with their tile counts
    DBuf<int64_t> kid((size_t)n);
    k_key_flags<<<grid_for(n, TPB), TPB, 0, st>>>(kpar.p, n, kid.p);
    FSM_LAUNCH_CHECK();
    G.ngroups = scan_exclusive(kid.p, kid.p, n);
    const size_t ng = (size_t)std::max<int64_t>(G.ngroups, 1);
    G.gk.alloc(ng); G.gcnt.alloc(ng); G.goff.alloc(ng); G.toff.alloc(ng + 1);
    DBuf<int64_t> tiles(ng);
    k_key_compact<<<grid_for(n, TPB), TPB, 0, st>>>(kpar.p, kpoff.p, n, kid.p, G.gk.p, G.gcnt.p,
                                                    G.goff.p);
    FSM_LAUNCH_CHECK();
    // parents per tile: as many as keep every wave of the grid busy
    const int32_t tuned = g_tuning.tiles_per_wave.load();
    const int tpw = opt.tiles_per_wave > 0 ? opt.tiles_per_wave : (tuned > 0 ? tuned : 16);
    const int64_t want = (int64_t)tpw * grid_persistent * (TPB / 64);
    for (G.tile_p = TILE_P_MAX;; G.tile_p /= 2) {
        k_key_tiles<<<grid_for(G.ngroups, TPB), TPB, 0, st>>>(
            G.gk.p, G.gcnt.p, G.pieces, G.ngroups, G.tile_p, tiles.p);
        FSM_LAUNCH_CHECK();
        G.ntiles = scan_exclusive(tiles.p, G.toff.p, G.ngroups);
        if (G.tile_p == 1 || G.ntiles >= want) break;
    }
    FSM_HIP(hipMemcpyAsync(G.toff.p + G.ngroups, &G.ntiles, sizeof(int64_t),
                           hipMemcpyHostToDevice, st));
    sync_stream(st);
}

// Longest-processing-time order of the key groups for the work queue:
// groups sorted by predicted cost per tile, largest first, then the tile
// offsets rebuilt in that order.
void Miner::order_groups(const Level& P, int M, const ItemRows& IR, const float* y, Groups& G) {
    const int64_t ng = G.ngroups;
    if (ng < 2) return;
    const int64_t nitems = (int64_t)P.tab.qcap * M;
    DBuf<float> rowcost((size_t)nitems);
    rowcost.zero();
    k_item_rowcost<<<grid_for(IR.rows, TPB), TPB, 0, st>>>(y, IR.item.p, IR.rows, M, IR.cnt.p,
                                                           rowcost.p);
    FSM_LAUNCH_CHECK();
    DBuf<int64_t> tiles((size_t)ng);
    k_key_tiles<<<grid_for(ng, TPB), TPB, 0, st>>>(G.gk.p, G.gcnt.p, G.pieces, ng, G.tile_p,
                                                   tiles.p);
    FSM_LAUNCH_CHECK();
    DBuf<float> gcost((size_t)ng);
    k_group_cost<<<grid_for(ng, TPB / 64), TPB, 0, st>>>(G.gk.p, G.goff.p, G.gcnt.p, tiles.p, ng,
                                                       G.glist.p, P.emb.p, M, rowcost.p, gcost.p);
    FSM_LAUNCH_CHECK();
    std::vector<float> hc;
    std::vector<int32_t> hk;
    std::vector<int64_t> ho, hn;
    to_host(hc, gcost.p, (size_t)ng);
    to_host(hk, G.gk.p, (size_t)ng);
    to_host(ho, G.goff.p, (size_t)ng);
    to_host(hn, G.gcnt.p, (size_t)ng);
    std::vector<int64_t> ord((size_t)ng);
    for (int64_t g = 0; g < ng; ++g) ord[(size_t)g] = g;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int64_t a, int64_t b) { return hc[(size_t)a] > hc[(size_t)b]; });
    std::vector<int32_t> pk((size_t)ng);
    std::vector<int64_t> po((size_t)ng), pn((size_t)ng);
    for (int64_t g = 0; g < ng; ++g) {
        pk[(size_t)g] = hk[(size_t)ord[(size_t)g]];
        po[(size_t)g] = ho[(size_t)ord[(size_t)g]];
        pn[(size_t)g] = hn[(size_t)ord[(size_t)g]];
    }
    to_device(G.gk.p, pk.data(), (size_t)ng);
    to_device(G.goff.p, po.data(), (size_t)ng);
    to_device(G.gcnt.p, pn.data(), (size_t)ng);
    k_key_tiles<<<grid_for(ng, TPB), TPB, 0, st>>>(G.gk.p, G.gcnt.p, G.pieces, ng, G.tile_p,
                                                   tiles.p);
    FSM_LAUNCH_CHECK();
    const int64_t nt = scan_exclusive(tiles.p, G.toff.p, ng);
    if (nt != G.ntiles) fail(FSM_EDEVICE, "tile count changed by reordering (%lld vs %lld)",
                             (long long)nt, (long long)G.ntiles);
    FSM_HIP(hipMemcpyAsync(G.toff.p + ng, &G.ntiles, sizeof(int64_t), hipMemcpyHostToDevice, st));
    sync_stream(st);
}

// Sampling proposal: keep rate min(1, lambda / c_i) for work item i, where
// c_i is its predicted children -- every item's expected work is capped at
// lambda, so items with few children (rare child patterns) are enumerated
// whole and only heavy, redundant items are thinned; lambda makes the
// expected work sum(rate_i c_i) equal sampling_rate * sum(c_i), the
// uniform rate's.
void Miner::proposal_thresholds(const ItemRows& IR, const float* y, int64_t nitems,
                                DBuf<uint64_t>& thr) {
    std::vector<float> hy;
    std::vector<int32_t> hi;
    to_host(hy, y, (size_t)(IR.rows * MODEL_OUT));
    to_host(hi, IR.item.p, (size_t)IR.rows);
    const size_t R = (size_t)IR.rows;
    std::vector<float> pred(R);
    for (size_t r = 0; r < R; ++r) pred[r] = hy[2 * r];
    std::vector<uint64_t> rt(R);
    proposal_keep_thresholds(pred.data(), (int64_t)R, opt.sampling_rate, rt.data());
    const uint64_t uni = (uint64_t)std::ldexp(opt.sampling_rate, 64);
    std::vector<uint64_t> h((size_t)nitems, uni);
    for (size_t r = 0; r < R; ++r) {
        if (hi[r] < 0 || (int64_t)hi[r] >= nitems)
            fail(FSM_EDEVICE, "work-item row %zu names item %d of %lld", r, hi[r],
                 (long long)nitems);
        h[(size_t)hi[r]] = rt[r];
    }
    thr.alloc((size_t)nitems);
    to_device(thr.p, h.data(), h.size());
}

// Piece lists of G_f sorted by key within every joining vertex; left empty
// (the join then decodes pieces) when there are 2^31 pieces or more.
void Miner::sorted_pieces(DBuf<int64_t>& poff, DBuf<uint64_t>& key, DBuf<uint8_t>& code) {
    const int64_t n = g->n;
    poff.alloc((size_t)n + 1);
    const int64_t total = scan_exclusive(npieces.p, poff.p, n);
    if (total <= 0 || total >= (int64_t)INT32_MAX) {
        poff.reset();
        return;
    }
    FSM_HIP(hipMemcpyAsync(poff.p + n, &total, sizeof(int64_t), hipMemcpyHostToDevice, st));
    DBuf<uint64_t> k0((size_t)total);
    DBuf<uint8_t> c0((size_t)total);
    k_piece_fill<<<grid_for(n, TPB / 64), TPB, 0, st>>>(frow.p, fcol.p, leafoff.p, npieces.p,
                                                        poff.p, n, k0.p, c0.p);
    FSM_LAUNCH_CHECK();
    DBuf<int32_t> off32((size_t)n + 1);
    k_offsets32<<<grid_for(n + 1, TPB), TPB, 0, st>>>(poff.p, n + 1, off32.p);
    FSM_LAUNCH_CHECK();
    key.alloc((size_t)total);
    code.alloc((size_t)total);
    sort_segments(k0.p, key.p, c0.p, code.p, (int)total, (int)n, off32.p);
}

void Miner::item_rows(const Level& P, int n, ItemRows& IR) {
    const int M = n - 2;
    const int64_t nitems = (int64_t)P.tab.qcap * M;
    DBuf<unsigned>& cnt = IR.cnt;
    cnt.alloc((size_t)P.tab.qcap);
    DBuf<unsigned long long> dsum((size_t)nitems);
    cnt.zero();
    dsum.zero();
    k_item_stats<<<grid_for(P.rows, TPB), TPB, 0, st>>>(P.emb.p, P.rows, M, frow.p, cnt.p, dsum.p);
    FSM_LAUNCH_CHECK();
    DBuf<int64_t> pos((size_t)nitems);
    k_item_flags<<<grid_for(nitems, TPB), TPB, 0, st>>>(cnt.p, nitems, M, pos.p);
    FSM_LAUNCH_CHECK();
    IR.rows = scan_exclusive(pos.p, pos.p, nitems);
    IR.x.alloc((size_t)(IR.rows * FSM_FEATURES));
    IR.item.alloc((size_t)IR.rows);
    IR.graph.alloc((size_t)IR.rows);
    FeatArgs fa{pos.p, IR.graph.p, cnt.p, dsum.p, P.tab.qadj.p, P.tab.qlab.p, P.tab.qpat.p,
                P.tab.csup.p, dtg.p, nitems, M, n, IR.x.p, IR.item.p};
    k_item_features<<<grid_for(nitems, TPB), TPB, 0, st>>>(fa);
    FSM_LAUNCH_CHECK();
}

void Miner::join(int n) {
    Level& L = lv[n];
    Level& P = lv[n - 2];
    L.n = n;
    const int M = n - 2;
    const int64_t nwork = P.rows * M;
    L.st.parents = P.rows;
    L.st.work_items = nwork;
    if (fsm_trace())
        std::fprintf(stderr, "[fsm] size %d join: %lld parents, %lld work items\n", n,
                     (long long)P.rows, (long long)nwork);
    // cost-model work items: predictions size the QP table; recorded
    // targets come from the domain pass
    const bool learned = (opt.mode & FSM_LEARNED) && model != nullptr;
    const bool record = opt.record != 0;
    double pred_raw = 0.0;
    ItemRows IR;
    DBuf<float> y;
    if ((learned || record) && P.rows > 0) item_rows(P, n, IR);
    if (learned && IR.rows > 0) {
        y.alloc((size_t)(IR.rows * MODEL_OUT));
        model->predict(IR.x.p, IR.rows, y.p);
        DBuf<double> tot(1);
        tot.zero();
        k_pred_total<<<grid_for(IR.rows, TPB, 1024), TPB, 0, st>>>(y.p, IR.rows, 1, tot.p);
        FSM_LAUNCH_CHECK();
        const double raw = scalar_to_host(tot.p);
        const double pq = raw * (model->calib[n] > 0 ? model->calib[n] : 1.0);
        L.st.qp_predicted = (int64_t)std::llround(pq);
        // load <= 1/2, 25% slack; an underestimate still overflows and
        // reruns, an overestimate is capped at 2^26 slots; a density hint
        // from earlier chunks of a batch is kept when it is larger
        qhint[n] = std::max(qhint[n], pow2_at_least((uint64_t)std::min(2.5 * pq + 64, 67108864.0)));
        pred_raw = raw;
    }
    const int64_t nitems = (int64_t)P.tab.qcap * M;
    // sampled + learned: per-item keep rates from the model (the proposal)
    DBuf<uint64_t> ithr;
    if (learned && (opt.mode & FSM_SAMPLED) && IR.rows > 0 && opt.sampling_rate < 1.0)
        proposal_thresholds(IR, y.p, nitems, ithr);
    DBuf<unsigned long long> ich;
    DBuf<unsigned> iqp;
    if (record && IR.rows > 0) {
        ich.alloc((size_t)nitems);
        iqp.alloc((size_t)nitems);
    }
    const uint64_t thr =
        opt.sampling_rate >= 1.0 ? ~0ull
                                 : (uint64_t)std::ldexp(opt.sampling_rate, 64);
    // hash-table bytes: 12 per stored size-3 subgraph of each work item's
    // key group (capped at the ST sample)
    if (nwork > 0) {
        DBuf<int64_t> gsize((size_t)g->n);
        const SelArgs sa = sel_args(n);
        k_key_group_sizes<<<grid_for(g->n, TPB / 64), TPB, 0, st>>>(sa, gsize.p);
        FSM_LAUNCH_CHECK();
        DBuf<unsigned long long> hb(1);
        hb.zero();
        const int64_t cap = opt.join_threshold > 0 ? opt.join_threshold * opt.join_threshold : 0;
        k_item_group_sum<<<grid_for(P.rows, TPB, 4096), TPB, 0, st>>>(P.emb.p, P.rows, M, gsize.p,
                                                                     cap, hb.p);
        FSM_LAUNCH_CHECK();
        L.st.hash_bytes = 12 * (int64_t)scalar_to_host(hb.p);
    }
    // ST x (Section 5): x^2 size-3 subgraphs per key group at every join,
    // and x edges per key group at the size-4 join
    Sampling smp = sampling();
    DBuf<uint64_t> kthr, ethr;
    if (opt.join_threshold > 0 && nwork > 0) {
        const uint64_t x = (uint64_t)opt.join_threshold;
        group_thresholds(SEL_PIECES, n, x * x, kthr);
        smp.kthr = kthr.p;
        if (n == 4) {
            group_thresholds(SEL_EDGES, n, x, ethr);
            smp.ethr = ethr.p;
        }
    }
    auto args = [&](Rec R, int64_t* counts, const int64_t* offsets, int32_t* out, int64_t rows) {
        JoinArgs a;
        a.row = frow.p; a.col = fcol.p; a.vf = vf.p;
        a.npieces = npieces.p; a.leafoff = leafoff.p;
        a.nh = nh();
        a.vg = g->vg;
        a.f3 = f3.p; a.F = F;
        a.par = P.emb.p; a.padj = P.tab.qadj.p;
        a.R = R;
        a.work_ctr = counters.p + 2; a.nwork = nwork;
        a.emitted = counters.p; a.cands = counters.p + 1; a.bytes = counters.p + 3;
        a.prune = opt.disable_pruning ? 0 : 1;
        a.sampled = (opt.mode & FSM_SAMPLED) ? 1 : 0;
        a.seed = opt.seed; a.sample_thr = thr; a.item_thr = ithr.p;
        a.induced = (opt.mode & FSM_INDUCED) ? 1 : 0;
        a.xh = xh();
        a.smp = smp;
        a.counts = counts; a.offsets = offsets; a.out = out; a.out_rows = rows;
        return a;
    };
    auto launch_mode = [&](int mode, const JoinArgs& a) {
#define FSM_JOIN_CASE(NN)                                                           \
    case NN:                                                                        \
        if (mode == MODE_COUNT) k_join<NN, MODE_COUNT><<<grid_persistent, TPB, 0, st>>>(a); \
        else k_join<NN, MODE_FILL><<<grid_persistent, TPB, 0, st>>>(a);            \
        break;
        switch (n) {
            FSM_JOIN_CASE(4)
            FSM_JOIN_CASE(5)
            FSM_JOIN_CASE(6)
            FSM_JOIN_CASE(7)
            default: fail(FSM_EINVAL, "bad join size %d", n);
        }
#undef FSM_JOIN_CASE
        FSM_LAUNCH_CHECK();
    };
    // ST: the domain pass enumerates only each key group's sampled pieces
    DBuf<int64_t> stcnt, poff;
    DBuf<uint64_t> pkey;
    DBuf<uint8_t> pcode;
    if (smp.kthr && nwork > 0) st_pieces(n, smp, stcnt, poff, pkey, pcode);
    Groups G;
    if (nwork > 0) build_groups(P, M, nwork, G, stcnt.p);
    if (y.p && G.ntiles > 0 && opt.schedule == FSM_SCHEDULE_QUEUE) order_groups(P, M, IR, y.p, G);
    // size 5: pieces of every joining vertex sorted by their (min, max) key,
    // so that the pieces preceding a parent's triple are a prefix of a tile
    if (n == 5 && G.ntiles > 0 && !stcnt.p) sorted_pieces(poff, pkey, pcode);
    const uint32_t dsize = 1u << (n * (n - 1) / 2);
    DBuf<uint16_t> dtab(dsize);
    k_dissect_table<<<grid_for(dsize, TPB), TPB, 0, st>>>(n, dtab.p);
    FSM_LAUNCH_CHECK();
    auto tile_args = [&](Rec R) {
        hrec = R;
        FSM_HIP(hipMemcpyAsync(drec.p, &hrec, sizeof(Rec), hipMemcpyHostToDevice, st));
        TileArgs t;
        t.row = frow.p; t.col = fcol.p; t.vinfo = vinfo.p; t.vg = g->vg;
        t.npieces = stcnt.p ? stcnt.p : npieces.p; t.leafoff = leafoff.p;
        t.nh = nh();
        t.f3 = f3.p; t.F = F;
        t.par = P.emb.p; t.padj = P.tab.qadj.p;
        t.gk = G.gk.p;
        t.goff = G.goff.p; t.gcnt = G.gcnt.p; t.toff = G.toff.p;
        t.ngroups = G.ngroups; t.ntiles = G.ntiles; t.glist = G.glist.p;
        t.tile_p = G.tile_p;
        t.bits = R.pool.words; t.W = R.pool.W; t.rbase = R.pool.rbase; t.rec = drec.p;
        t.porb = R.pool.porb; t.qcnt = R.pool.qcnt;
        t.flags = R.flags;
        t.item_children = nullptr;
        t.pkey = pkey.p;
        t.pcode = pcode.p;
        t.poff = poff.p;
        t.queue = opt.schedule == FSM_SCHEDULE_STATIC ? 0 : 1;
        t.ctr = counters.p;
        t.prune = opt.disable_pruning ? 0 : 1;
        t.sampled = (opt.mode & FSM_SAMPLED) ? 1 : 0;
        t.seed = opt.seed; t.sample_thr = thr; t.item_thr = ithr.p;
        t.induced = (opt.mode & FSM_INDUCED) ? 1 : 0;
        t.xh = xh();
        t.smp = smp;
        t.dtab = dtab.p;
        return t;
    };
    // the plain exact join runs a build of the tile kernel without the
    // sampling, vertex-induced and candidate-bitmap paths
    const bool extra = (opt.mode & (FSM_SAMPLED | FSM_INDUCED)) || ithr.p || smp.kthr ||
                       smp.ethr || smp.mthr;
    // batched calls: the last level as a replay of its captured graph
    if (lg && !extra && !ich.p && n + 2 > opt.max_size && n <= 6 && G.ntiles > 0 &&
        captured_level(L, tile_args)) {
        if (pred_raw > 0.0 && L.st.quick_patterns > 0)
            model->calib[n] = (double)L.st.quick_patterns / pred_raw;
        return;
    }
    {
        Timer jt(timing, st);
        float join_total = 0.f;
        domain_level(L, [&](Rec R, int pass) {
            // recording: pass 0 sees every child and inserts every QP
            if (ich.p && pass == 0) {
                ich.zero();
                iqp.zero();
                R.item_qps = iqp.p;
            }
            if (pass == 0) join_total = 0.f;   // a new attempt
            jt.start();
            if (G.ntiles > 0) {
                htile = tile_args(R);
                htile.item_children = pass == 0 ? ich.p : nullptr;
                const bool ex = extra || htile.porb || htile.qcnt;
                FSM_HIP(hipMemcpyAsync(dtile.p, &htile, sizeof(TileArgs), hipMemcpyHostToDevice,
                                       st));
#define FSM_TILES_CASE(NN)                                                          \
    case NN:                                                                        \
        if (ex) k_join_tiles_p<NN, true><<<grid_persistent, TPB, 0, st>>>(dtile.p);  \
        else k_join_tiles_p<NN, false><<<grid_persistent, TPB, 0, st>>>(dtile.p);    \
        break;
                switch (n) {
                    FSM_TILES_CASE(4)
                    FSM_TILES_CASE(5)
                    FSM_TILES_CASE(6)
                    FSM_TILES_CASE(7)
                    default: fail(FSM_EINVAL, "bad join size %d", n);
                }
#undef FSM_TILES_CASE
                FSM_LAUNCH_CHECK();
            }
            join_total += jt.stop();
        });
        L.st.join_ms = join_total;
    }
    if (pred_raw > 0.0 && L.st.quick_patterns > 0)
        model->calib[n] = (double)L.st.quick_patterns / pred_raw;
    if (ich.p) {
        DBuf<float> t((size_t)(IR.rows * MODEL_OUT));
        k_item_targets<<<grid_for(IR.rows, TPB), TPB, 0, st>>>(IR.item.p, IR.rows, ich.p, iqp.p,
                                                               t.p);
        FSM_LAUNCH_CHECK();
        const size_t o = rt.size() / MODEL_OUT;
        rx.resize((o + (size_t)IR.rows) * FSM_FEATURES);
        rt.resize((o + (size_t)IR.rows) * MODEL_OUT);
        rg.resize(o + (size_t)IR.rows);
        to_host_into(rx.data() + o * FSM_FEATURES, IR.x.p, (size_t)IR.rows * FSM_FEATURES);
        to_host_into(rt.data() + o * MODEL_OUT, t.p, (size_t)IR.rows * MODEL_OUT);
        to_host_into(rg.data() + o, IR.graph.p, (size_t)IR.rows);
        rl.resize(o + (size_t)IR.rows, n);
    }
    if (n + 2 <= opt.max_size) {
        materialize(L, nwork, [&](int mode, int64_t* counts, const int64_t* offsets, int32_t* out,
                                  int64_t rows) {
            if (nwork > 0) launch_mode(mode, args(rec(L), counts, offsets, out, rows));
        });
    }
}

// Single-vertex join of size n: parents of size n-1 joined with one edge
// at each of their vertices (the baseline of Section 6).
void Miner::join_single(int n) {
    Level& L = lv[n];
    Level& P = lv[n - 1];
    L.n = n;
    const int M = n - 1;
    const int64_t nwork = P.rows * M;
    L.st.parents = P.rows;
    L.st.work_items = nwork;
    Sampling smp = sampling();
    DBuf<uint64_t> ethr;
    if (opt.join_threshold > 0 && nwork > 0) {
        group_thresholds(SEL_EDGES, n, (uint64_t)opt.join_threshold, ethr);
        smp.ethr = ethr.p;
    }
    // hash-table bytes: 8 per G_f edge of each work item's joining vertex
    // (capped at the ST sample)
    DBuf<int64_t> deg((size_t)g->n);
    k_degrees<<<grid_for(g->n, TPB), TPB, 0, st>>>(frow.p, g->n, deg.p);
    FSM_LAUNCH_CHECK();
    if (nwork > 0) {
        DBuf<unsigned long long> hb(1);
        hb.zero();
        k_item_group_sum<<<grid_for(P.rows, TPB, 4096), TPB, 0, st>>>(
            P.emb.p, P.rows, M, deg.p, opt.join_threshold, hb.p);
        FSM_LAUNCH_CHECK();
        L.st.hash_bytes = 8 * (int64_t)scalar_to_host(hb.p);
    }
    const uint32_t tsize = 1u << (n * (n - 1) / 2);
    DBuf<uint8_t> svtab(tsize);
    k_single_table<<<grid_for(tsize, TPB), TPB, 0, st>>>(n, svtab.p);
    FSM_LAUNCH_CHECK();
    auto args = [&](Rec R, int64_t* counts, const int64_t* offsets, int32_t* out, int64_t rows) {
        SingleArgs a;
        a.row = frow.p; a.col = fcol.p; a.vf = vf.p; a.vg = g->vg;
        a.nh = nh(); a.xh = xh();
        a.induced = (opt.mode & FSM_INDUCED) ? 1 : 0;
        a.par = P.emb.p; a.padj = P.tab.qadj.p;
        a.svtab = svtab.p;
        a.R = R;
        a.ctr = counters.p;
        a.nwork = nwork;
        a.smp = smp;
        a.counts = counts; a.offsets = offsets; a.out = out; a.out_rows = rows;
        return a;
    };
    auto launch = [&](int mode, const SingleArgs& a) {
#define FSM_SINGLE_CASE(NN)                                                                  \
    case NN:                                                                                 \
        if (mode == MODE_COUNT) k_single<NN, MODE_COUNT><<<grid_persistent, TPB, 0, st>>>(a); \
        else k_single<NN, MODE_FILL><<<grid_persistent, TPB, 0, st>>>(a);                     \
        break;
        switch (n) {
            FSM_SINGLE_CASE(3)
            FSM_SINGLE_CASE(4)
            FSM_SINGLE_CASE(5)
            FSM_SINGLE_CASE(6)
            FSM_SINGLE_CASE(7)
            default: fail(FSM_EINVAL, "bad join size %d", n);
        }
#undef FSM_SINGLE_CASE
        FSM_LAUNCH_CHECK();
    };
    Groups G;
    if (nwork > 0) build_groups(P, M, nwork, G, deg.p);
    auto tile_args = [&](Rec R) {
        hrec = R;
        FSM_HIP(hipMemcpyAsync(drec.p, &hrec, sizeof(Rec), hipMemcpyHostToDevice, st));
        SingleTileArgs t;
        t.row = frow.p; t.col = fcol.p; t.vinfo = vinfo.p; t.vg = g->vg;
        t.nh = nh(); t.xh = xh();
        t.induced = (opt.mode & FSM_INDUCED) ? 1 : 0;
        t.par = P.emb.p; t.padj = P.tab.qadj.p;
        t.gk = G.gk.p; t.goff = G.goff.p; t.gcnt = G.gcnt.p; t.toff = G.toff.p;
        t.ngroups = G.ngroups; t.ntiles = G.ntiles; t.glist = G.glist.p; t.tile_p = G.tile_p;
        t.svtab = svtab.p;
        t.bits = R.pool.words; t.W = R.pool.W; t.rbase = R.pool.rbase; t.rec = drec.p;
        t.porb = R.pool.porb; t.qcnt = R.pool.qcnt;
        t.flags = R.flags;
        t.ctr = counters.p;
        t.smp = smp;
        return t;
    };
    {
        Timer jt(timing, st);
        float join_total = 0.f;
        domain_level(L, [&](Rec R, int pass) {
            if (pass == 0) join_total = 0.f;
            jt.start();
            if (G.ntiles > 0) {
                // arguments from device memory: as kernel arguments they
                // would take scalar registers the loop needs
                hstile = tile_args(R);
                FSM_HIP(hipMemcpyAsync(dstile.p, &hstile, sizeof(SingleTileArgs),
                                       hipMemcpyHostToDevice, st));
                const SingleTileArgs* t = dstile.p;
                switch (n) {
                    case 3: k_single_tiles<3><<<grid_persistent, TPB, 0, st>>>(t); break;
                    case 4: k_single_tiles<4><<<grid_persistent, TPB, 0, st>>>(t); break;
                    case 5: k_single_tiles<5><<<grid_persistent, TPB, 0, st>>>(t); break;
                    case 6: k_single_tiles<6><<<grid_persistent, TPB, 0, st>>>(t); break;
                    case 7: k_single_tiles<7><<<grid_persistent, TPB, 0, st>>>(t); break;
                    default: fail(FSM_EINVAL, "bad join size %d", n);
                }
                FSM_LAUNCH_CHECK();
            }
            join_total += jt.stop();
        });
        L.st.join_ms = join_total;
    }
    if (n + 1 <= opt.max_size) {
        materialize(L, nwork, [&](int mode, int64_t* counts, const int64_t* offsets, int32_t* out,
                                  int64_t rows) {
            if (nwork > 0) launch(mode, args(rec(L), counts, offsets, out, rows));
        });
    }
}

void Miner::emit_results() {
    if (opt.record) {
        const size_t rows = rl.size();
        for (size_t r = 0; r < rows; ++r) {
            if (rg[r] < 0 || rg[r] >= g->ngraphs)
                fail(FSM_EDEVICE, "training row %zu names graph %d of %d", r, rg[r], g->ngraphs);
            fsm_result* out = res[(size_t)rg[r]];
            out->tx.insert(out->tx.end(), rx.begin() + (long)(r * FSM_FEATURES),
                           rx.begin() + (long)((r + 1) * FSM_FEATURES));
            out->tt.insert(out->tt.end(), rt.begin() + (long)(r * MODEL_OUT),
                           rt.begin() + (long)((r + 1) * MODEL_OUT));
            out->tl.push_back(rl[r]);
        }
    }
    for (int n = 2; n <= opt.max_size; ++n) {
        const int npairs = n * (n - 1) / 2;
        for (auto& kv : lv[n].freq) {
            fsm_code c;
            memset(&c, 0, sizeof(c));
            c.n = n;
            for (int i = 0; i < FSM_MAX_SIZE; ++i) c.label[i] = -1;
            for (int i = 0; i < n; ++i) c.label[i] = fvalue[(size_t)code_label(kv.first, n, i)];
            const uint32_t seq = code_seq(kv.first, n);
            for (int k = 0; k < npairs; ++k)
                if ((seq >> (npairs - 1 - k)) & 1u) c.adj |= 1u << k;
            fsm_result* r = res[graph_of(kv.first, n)];
            r->size.push_back(n);
            r->code.push_back(c);
            r->support.push_back(kv.second);
        }
    }
}

void Miner::run() {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t syncs0 = host_syncs();
    st = stream();
    for (fsm_result* r : res) r->stats.max_size = opt.max_size;
    const int32_t G = g->ngraphs, NL = g->L;
    // frequent labels: a pattern vertex of label l has at most count(l)
    // images, so (graph, label) is kept when its graph's threshold allows
    std::vector<int32_t> lid((size_t)NL, -1);       // label -> frequent id
    std::vector<int32_t> fmap((size_t)G * NL, -1);  // (graph, label) -> frequent id or -1
    for (int32_t gi = 0; gi < G; ++gi)
        for (int32_t l = 0; l < NL; ++l)
            if (g->count[(size_t)gi * NL + l] >= tg[(size_t)gi]) {
                if (lid[(size_t)l] < 0) {
                    if (F >= FSM_MAX_FREQ_LABELS)
                        fail(FSM_EUNSUPPORTED, "more than %d labels reach the support threshold",
                             FSM_MAX_FREQ_LABELS);
                    lid[(size_t)l] = F++;
                    fvalue.push_back(g->label_value[(size_t)l]);
                }
                fmap[(size_t)gi * NL + l] = lid[(size_t)l];
            }
    for (fsm_result* r : res) r->stats.frequent_labels = F;
    if (F == 0 || g->nnz == 0) {
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (fsm_result* r : res) r->stats.total_ms = ms;
        return;
    }
    dtg.alloc(tg.size());
    to_device(dtg.p, tg.data(), tg.size());
    int dev = 0;
    FSM_HIP(hipGetDevice(&dev));
    int cus = 0;
    FSM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    grid_persistent = (unsigned)std::max(1, cus) * 8;
    DBuf<int32_t> dmap(fmap.size());
    to_device(dmap.p, fmap.data(), fmap.size());
    vf.alloc((size_t)g->n);
    k_vertex_flabel<<<grid_for(g->n, TPB), TPB, 0, st>>>(g->lab, g->vg, NL, g->n, dmap.p, vf.p);
    FSM_LAUNCH_CHECK();
    // bitmaps are indexed by rank within (graph, label): as many bits as the
    // most populous frequent (graph, label) has vertices
    int64_t maxcount = 1;
    for (size_t x = 0; x < fmap.size(); ++x)
        if (fmap[x] >= 0) maxcount = std::max(maxcount, g->count[x]);
    W = (uint32_t)((maxcount + 31) / 32);
    pass_W = W;
    refresh_pool_budget();
    lrank.alloc((size_t)g->n);
    {
        DBuf<unsigned> lcnt((size_t)G * F);
        lcnt.zero();
        k_label_rank<<<grid_for(g->n, TPB), TPB, 0, st>>>(vf.p, g->vg, F, g->n, lcnt.p, lrank.p);
        FSM_LAUNCH_CHECK();
    }
    if (maxcount > (int64_t)RANK_MASK)
        fail(FSM_EUNSUPPORTED, "a frequent label has more than 2^26 vertices");
    vinfo.alloc((size_t)g->n);
    k_vinfo<<<grid_for(g->n, TPB), TPB, 0, st>>>(vf.p, lrank.p, g->n, vinfo.p);
    FSM_LAUNCH_CHECK();
    drec.alloc(1);
    dtile.alloc(1);
    dstile.alloc(1);
    counters.alloc(4);
    flags.alloc(1);

    Timer lt(timing, st);
    auto timed = [&](int n, auto&& body) {
        lt.start();
        body();
        lv[n].st.kernel_ms = lt.stop();
    };
    // level-2 embeddings: the edges of G_f (u < w)
    auto materialize_edges = [&] {
        Level& L = lv[2];
        materialize(L, g->n, [&](int mode, int64_t* counts, const int64_t* offsets, int32_t* out,
                                 int64_t rows) {
            L2Args a{frow.p, fcol.p, vf.p, g->vg, g->n, rec(L), counters.p, counts, offsets, out,
                     rows};
            if (mode == MODE_COUNT) k_level2<MODE_COUNT><<<grid_persistent, TPB, 0, st>>>(a);
            else k_level2<MODE_FILL><<<grid_persistent, TPB, 0, st>>>(a);
            FSM_LAUNCH_CHECK();
        });
    };
    {
        timed(2, [&] { level2(); });
        build_gf();
        if (opt.mode & FSM_SINGLE) {
            // single-vertex exploration: one-edge joins from the edges up
            if (opt.max_size >= 3) materialize_edges();
            else lv[2].tab = Tables();
            for (int n = 3; n <= opt.max_size; ++n) {
                timed(n, [&] { join_single(n); });
                lv[n - 1].emb.reset();
                lv[n - 1].tab = Tables();
                if (n + 1 > opt.max_size) lv[n].tab = Tables();
            }
        } else {
            if (opt.max_size >= 3) timed(3, [&] { level3(); });
            // the edges are the parents of the size-4 join
            if (opt.max_size >= 4) materialize_edges();
            if (opt.max_size >= 5) {
                Level& L = lv[3];
                materialize(L, g->n, [&](int mode, int64_t* counts, const int64_t* offsets,
                                         int32_t* out, int64_t rows) {
                    L3Args a{frow.p, fcol.p, vf.p, g->vg, g->n, nh(), rec(L), counters.p,
                             counts, offsets, out, rows};
                    a.induced = (opt.mode & FSM_INDUCED) ? 1 : 0;
                    a.xh = xh();
                    a.smp = sampling();
                    if (mode == MODE_COUNT) k_level3<MODE_COUNT><<<grid_persistent, TPB, 0, st>>>(a);
                    else k_level3<MODE_FILL><<<grid_persistent, TPB, 0, st>>>(a);
                    FSM_LAUNCH_CHECK();
                });
            }
            if (opt.max_size < 4) lv[2].tab = Tables();
            if (opt.max_size < 5) lv[3].tab = Tables();
            for (int n = 4; n <= opt.max_size; ++n) {
                timed(n, [&] { join(n); });
                if (fsm_trace())
                    std::fprintf(stderr, "[fsm] size %d done: %lld children, %lld QPs, "
                                 "%lld patterns, %lld slices, %.1f ms\n", n,
                                 (long long)lv[n].st.emitted, (long long)lv[n].st.quick_patterns,
                                 (long long)lv[n].st.patterns, (long long)lv[n].st.rank_slices,
                                 lv[n].st.kernel_ms);
                // size n-2 embeddings and their QP table are no longer needed,
                // nor the size-n table when no later join reads it
                lv[n - 2].emb.reset();
                lv[n - 2].tab = Tables();
                if (n + 2 > opt.max_size) lv[n].tab = Tables();
            }
        }
    }
    for (fsm_result* r : res)
        for (int n = 2; n <= opt.max_size; ++n) r->stats.level[n] = lv[n].st;
    emit_results();
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (fsm_result* r : res) {
        r->stats.total_ms = ms;
        r->stats.captured_levels = captured;
        r->stats.host_syncs = host_syncs() - syncs0;
    }
}

}  // namespace

// Keep thresholds of the sampling proposal from per-row predictions
// (log1p of predicted children).  Every sum runs over the predicted costs
// in ascending order, so the result depends on the multiset of rows and not
// on their order (work-item rows come out in QP-slot order, which CAS races
// decide); a row's rate, relative to the uniform rate, is rounded to 2^-20
// before it becomes a threshold, so an item whose rate equals the uniform
// one gets exactly the uniform threshold.  With no predicted work every row
// keeps everything.
void proposal_keep_thresholds(const float* pred, int64_t rows, double rate, uint64_t* thr) {
    const size_t R = (size_t)std::max<int64_t>(rows, 0);
    std::vector<double> c(R);
    for (size_t r = 0; r < R; ++r) c[r] = std::expm1(std::max(0.0, (double)pred[r]));
    std::vector<double> sc(c);
    std::sort(sc.begin(), sc.end());
    double total = 0.0;
    for (double v : sc) total += v;
    const double budget = rate * total;
    if (!(rate < 1.0) || !(budget > 0.0)) {
        for (size_t r = 0; r < R; ++r) thr[r] = ~0ull;
        return;
    }
    auto work = [&](double lam) {
        double s = 0.0;
        for (double v : sc) s += std::min(1.0, lam / std::max(v, 1.0)) * v;
        return s;
    };
    double lo = 0.0, hi = 1.0;
    while (work(hi) < budget && hi < 1e30) hi *= 2.0;
    for (int it = 0; it < 100; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (work(mid) < budget) lo = mid; else hi = mid;
    }
    const double lam = hi;
    for (size_t r = 0; r < R; ++r) {
        const double rel = std::min(1.0, lam / std::max(c[r], 1.0)) / rate;
        const double q = std::nearbyint(rel * 1048576.0) / 1048576.0;   // 2^-20 grid
        const double keep = rate * q;
        thr[r] = keep >= 1.0 ? ~0ull : (uint64_t)std::ldexp(keep, 64);
    }
}

void mine(const fsm_graph* g, const fsm_options& opt, fsm_result* r) {
    Miner m;
    m.gv.single(g);
    m.opt = opt;
    m.model = opt.model ? &opt.model->m : nullptr;
    m.tg.assign(1, opt.support);
    m.res.assign(1, r);
    r->stats.dropped_self_loops = g->dropped_loops;
    r->stats.dropped_duplicates = g->dropped_dups;
    r->stats.batch_chunks = 1;
    m.run();
}

void mine_in_arena(const fsm_graph* g, const fsm_options& opt, fsm_result* r) {
    Miner m;
    m.timing = false;
    m.gv.single(g);
    m.opt = opt;
    m.model = opt.model ? &opt.model->m : nullptr;
    m.tg.assign(1, opt.support);
    m.res.assign(1, r);
    r->stats.dropped_self_loops = g->dropped_loops;
    r->stats.dropped_duplicates = g->dropped_dups;
    r->stats.batch_chunks = 1;
    m.run();
}

// Most populous label of a graph: its bitmaps need ceil(that / 32) words.
int64_t widest_label(const fsm_graph* g) {
    int64_t m = 0;
    for (int64_t c : g->label_count) m = std::max(m, c);
    return m;
}

void mine_batch(const fsm_graph* const* gs, int32_t count, const int64_t* supports,
                const fsm_batch_options& bo, fsm_result* const* rs) {
    const int64_t tuned = g_tuning.chunk_vertices.load();
    const int64_t budget = bo.chunk_vertices > 0 ? bo.chunk_vertices
                           : (tuned > 0 ? tuned : (int64_t)1 << 14);
    // order by bitmap width (widest first), then pack consecutive graphs
    std::vector<int32_t> ord((size_t)count);
    for (int32_t i = 0; i < count; ++i) ord[(size_t)i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return widest_label(gs[a]) > widest_label(gs[b]);
    });
    std::deque<std::vector<int32_t>> todo;
    std::vector<int32_t> cur;
    int64_t acc = 0;
    for (int32_t i : ord) {
        if (!cur.empty() && acc + gs[i]->n > budget) {
            todo.push_back(std::move(cur));
            cur.clear();
            acc = 0;
        }
        cur.push_back(i);
        acc += gs[i]->n;
    }
    todo.push_back(std::move(cur));

    fsm_options o;
    memset(&o, 0, sizeof(o));
    o.max_size = bo.max_size;
    o.mode = bo.mode & (FSM_LEARNED | FSM_INDUCED);
    o.model = bo.model;
    o.record = bo.learn && bo.model ? 1 : 0;
    o.disable_pruning = bo.disable_pruning;
    o.tiles_per_wave = bo.tiles_per_wave;
    o.pool_budget_mib = bo.pool_budget_mib;
    o.sampling_rate = 1.0;
    o.hash_capacity_min = bo.hash_capacity_min;
    o.pattern_capacity_min = bo.pattern_capacity_min;
    // quick patterns per union vertex seen so far, per level: the next
    // chunk's tables start at that density (load <= 1/2, 25% slack)
    double qpv[FSM_MAX_SIZE + 1] = {};   // and canonical patterns per union vertex
    double ppv[FSM_MAX_SIZE + 1] = {};
    int32_t chunk = 0, splits = 0;
    LevelGraphs lgs;
    std::vector<int32_t> chunk_of((size_t)count, 0);
    while (!todo.empty()) {
        std::vector<int32_t> part = std::move(todo.front());
        todo.pop_front();
        std::vector<const fsm_graph*> pg;
        std::vector<fsm_result*> pr;
        int64_t nv = 0;
        for (int32_t i : part) {
            pg.push_back(gs[i]);
            pr.push_back(rs[i]);
            nv += gs[i]->n;
        }
        Miner m;
        m.opt = o;
        m.model = bo.model ? &bo.model->m : nullptr;
        if (!bo.eager_levels) m.lg = &lgs;
        for (int n = 2; n <= FSM_MAX_SIZE; ++n) {
            if (qpv[n] > 0) m.qhint[n] = pow2_at_least((uint64_t)(2.5 * qpv[n] * (double)nv) + 16);
            if (ppv[n] > 0) m.chint[n] = pow2_at_least((uint64_t)(2.5 * ppv[n] * (double)nv) + 16);
        }
        try {
            m.gv.batch(pg.data(), (int32_t)pg.size());
            for (int32_t i : part) m.tg.push_back(supports[i]);
            m.res = pr;
            m.run();
        } catch (const Failure& f) {
            if ((f.code != FSM_EOVERFLOW && f.code != FSM_ENOMEM) || part.size() < 2) throw;
            (void)hipGetLastError();
            sync_stream(stream());
            for (fsm_result* r : pr) *r = fsm_result();
            const size_t h = part.size() / 2;
            todo.push_front(std::vector<int32_t>(part.begin() + (long)h, part.end()));
            todo.push_front(std::vector<int32_t>(part.begin(), part.begin() + (long)h));
            ++splits;
            continue;
        }
        for (int n = 2; n <= o.max_size; ++n) {
            qpv[n] = std::max(qpv[n], (double)m.lv[n].st.quick_patterns / (double)std::max<int64_t>(nv, 1));
            ppv[n] = std::max(ppv[n], (double)m.lv[n].st.patterns / (double)std::max<int64_t>(nv, 1));
        }
        // online learning: the next chunks are sized by a model that has
        // seen this chunk's work items
        if (bo.learn && bo.model && !m.rl.empty()) {
            const int64_t rows = (int64_t)m.rl.size();
            DBuf<float> x((size_t)rows * FSM_FEATURES), t((size_t)rows * MODEL_OUT);
            to_device(x.p, m.rx.data(), m.rx.size());
            to_device(t.p, m.rt.data(), m.rt.size());
            bo.model->m.train(x.p, t.p, rows, bo.train_steps > 0 ? bo.train_steps : 200,
                              bo.lr > 0.f ? bo.lr : 3e-3f);
        }
        for (int32_t i : part) chunk_of[(size_t)i] = chunk;
        ++chunk;
    }
    for (int32_t i = 0; i < count; ++i) {
        rs[i]->stats.dropped_self_loops = gs[i]->dropped_loops;
        rs[i]->stats.dropped_duplicates = gs[i]->dropped_dups;
        rs[i]->stats.batch_chunk = chunk_of[(size_t)i];
        rs[i]->stats.batch_chunks = chunk;
        rs[i]->stats.batch_splits = splits;
        rs[i]->stats.captured_graphs = (int32_t)lgs.cache.size();
        rs[i]->stats.level_fallbacks = lgs.fallbacks;
    }
}

void set_tuning(int64_t chunk_vertices, int32_t tiles_per_wave) {
    g_tuning.chunk_vertices = chunk_vertices;
    g_tuning.tiles_per_wave = tiles_per_wave;
}

}  // namespace fsm
