// common.h -- host+device helpers of the miner: packed small-graph
// representation, connectivity, the smallest-vertex-first dissection rule,
// canonical forms, hashing.
//
// A subgraph of n <= 7 vertices in a fixed vertex order is held as
//   A: 8 bits per position p (bits 0..6 = positions adjacent to p),
//   L: 6 bits per position (frequent-label id 0..63).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FSM_HD __host__ __device__ __forceinline__

namespace fsm {

constexpr int MAXN = 7;
constexpr uint64_t EMPTY_KEY = ~0ull;

// splitmix64 finalizer (Steele, Lea, Flood 2014) -- hash of 64-bit keys.
FSM_HD uint64_t mix64(uint64_t x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

// Position of the unordered pair (i<j) in row-major upper-triangle order.
FSM_HD int pair_pos(int i, int j, int n) { return i * n - i * (i + 1) / 2 + (j - i - 1); }

FSM_HD uint32_t amask(uint64_t A, int p) { return (uint32_t)(A >> (8 * p)) & 0x7fu; }

FSM_HD uint64_t add_edge(uint64_t A, int p, int q) {
    return A | (1ull << (8 * p + q)) | (1ull << (8 * q + p));
}

FSM_HD int lab_at(uint64_t L, int p) { return (int)((L >> (6 * p)) & 63u); }

// Is the vertex subset S (bitmask over positions 0..n-1) connected in A?
FSM_HD bool connected(uint32_t S, uint64_t A, int n) {
    if (!S) return false;
    uint32_t r = S & (0u - S);
    for (int it = 0; it < n; ++it) {
        uint32_t nb = 0;
        for (int p = 0; p < n; ++p)
            if ((r >> p) & 1u) nb |= amask(A, p);
        uint32_t x = r | (nb & S);
        if (x == r) break;
        r = x;
    }
    return r == S;
}

// Rank-ordered position bits: byte r of the result is the bit of the
// position holding the r-th smallest id.
template <int N>
FSM_HD uint64_t rank_bits(const int32_t (&id)[N]) {
    uint64_t ob = 0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
        int r = 0;
#pragma unroll
        for (int q = 0; q < N; ++q) r += (id[q] < id[p]) ? 1 : 0;
        ob |= (uint64_t)(1u << p) << (8 * r);
    }
    return ob;
}

FSM_HD uint32_t ob_at(uint64_t ob, int r) { return (uint32_t)(ob >> (8 * r)) & 0xffu; }

// Smallest-vertex-first dissection (Section 4.3, Algorithm 1; the greedy
// span of the printed algorithm can miss the only valid split when n >= 6,
// so the rule is stated on the split itself): among all sorted id triples,
// take the lexicographically smallest triple l that is connected and has a
// member v' with (V \ l) + v' connected; v' is the smallest such member.
// Theorem 1 guarantees one exists for every connected graph.
// Inputs: n, rank-ordered position bits `ob`, adjacency A.
// Returns l as a position mask (0 if none) and v' as a position bit.
FSM_HD uint32_t dissect(int n, uint64_t ob, uint64_t A, uint32_t* vbit) {
    const uint32_t all = (1u << n) - 1u;
    for (int x = 0; x < n - 2; ++x)
        for (int y = x + 1; y < n - 1; ++y)
            for (int z = y + 1; z < n; ++z) {
                uint32_t bx = ob_at(ob, x), by = ob_at(ob, y), bz = ob_at(ob, z);
                uint32_t T = bx | by | bz;
                if (!connected(T, A, n)) continue;
                uint32_t rest = all & ~T;
                if (connected(rest | bx, A, n)) { *vbit = bx; return T; }
                if (connected(rest | by, A, n)) { *vbit = by; return T; }
                if (connected(rest | bz, A, n)) { *vbit = bz; return T; }
            }
    *vbit = 0;
    return 0;
}

// Does the dissection of (V', E') equal (l = Tstar, v' = kbit)?  Same rule as
// dissect(), stopping at the first triple that decides the answer.
FSM_HD bool dissection_is(int n, uint64_t ob, uint64_t A, uint32_t Tstar, uint32_t kbit) {
    const uint32_t all = (1u << n) - 1u;
    for (int x = 0; x < n - 2; ++x)
        for (int y = x + 1; y < n - 1; ++y)
            for (int z = y + 1; z < n; ++z) {
                uint32_t bx = ob_at(ob, x), by = ob_at(ob, y), bz = ob_at(ob, z);
                uint32_t T = bx | by | bz;
                uint32_t rest = all & ~T;
                if (T == Tstar) {
                    // the piece is connected and (V\l)+k is the parent: valid;
                    // v' must be k, i.e. no smaller member works
                    if (bx != kbit && connected(rest | bx, A, n)) return false;
                    if (bx == kbit) return true;
                    if (by != kbit && connected(rest | by, A, n)) return false;
                    return true;   // by == kbit, or bz == kbit after bx, by failed
                }
                if (!connected(T, A, n)) continue;
                if (connected(rest | bx, A, n) || connected(rest | by, A, n) ||
                    connected(rest | bz, A, n))
                    return false;
            }
    return false;
}

// Canonical form of an ordered labelled graph (n <= 7): the vertex order
// whose (label sequence, pair-bit sequence) is lexicographically smallest.
// The pair-bit sequence is packed with pair (0,1) as its most significant
// bit, so smaller integer = smaller sequence.  The label sequence of the
// minimum is the sorted labels, so only label-respecting orders are tried.
struct Canon {
    uint64_t code;    // labels (6 bits each, first vertex most significant) << n(n-1)/2 | sequence
    uint32_t slots;   // 3 bits per ORIGINAL position: min canonical position of its orbit
    uint32_t orbits;  // 3 bits per CANONICAL position: min canonical position of its orbit
};

FSM_HD uint32_t seq_under(int n, uint64_t A, const int* ord) {
    uint32_t s = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            s = (s << 1) | ((amask(A, ord[i]) >> ord[j]) & 1u);
    return s;
}

// Next lexicographic permutation of a[lo..hi); on wrap-around the range is
// restored to ascending order and false is returned.
FSM_HD bool next_perm_range(int* a, int lo, int hi) {
    int i = hi - 2;
    while (i >= lo && a[i] >= a[i + 1]) --i;
    int t;
    if (i >= lo) {
        int j = hi - 1;
        while (a[j] <= a[i]) --j;
        t = a[i]; a[i] = a[j]; a[j] = t;
    }
    for (int l = i + 1, r = hi - 1; l < r; ++l, --r) { t = a[l]; a[l] = a[r]; a[r] = t; }
    return i >= lo;
}

// kept out of line: it is the cold path of the recording kernels
__host__ __device__ inline __attribute__((noinline)) Canon canonicalize(int n, uint64_t L, uint64_t A) {
    // base order: positions sorted by label (stable)
    int ord[MAXN], best[MAXN], start[MAXN + 1];
    int k = 0;
    for (int l = 0; l < 64 && k < n; ++l)
        for (int p = 0; p < n; ++p)
            if (lab_at(L, p) == l) ord[k++] = p;
    // label classes = runs of equal labels in ord
    int ncls = 0;
    for (int i = 0; i < n; ++i)
        if (i == 0 || lab_at(L, ord[i]) != lab_at(L, ord[i - 1])) start[ncls++] = i;
    start[ncls] = n;
    // each class starts at its smallest permutation (ord is ascending per class)
    uint32_t bestseq = 0xffffffffu;
    int orb[MAXN];   // orbit representative of each canonical position
    for (int i = 0; i < n; ++i) { best[i] = ord[i]; orb[i] = i; }
    for (;;) {
        uint32_t s = seq_under(n, A, ord);
        if (s < bestseq) {
            bestseq = s;
            for (int i = 0; i < n; ++i) { best[i] = ord[i]; orb[i] = i; }
        } else if (s == bestseq) {
            // ord and best both reach the minimum: canonical positions
            // pos_best(p) and pos_ord(p) of each original vertex p share an orbit
            for (int i = 0; i < n; ++i) {
                int p = ord[i];
                int j = 0;
                while (best[j] != p) ++j;
                int a = orb[i], b = orb[j];
                int lo = a < b ? a : b, hi = a < b ? b : a;
                if (lo != hi)
                    for (int c = 0; c < n; ++c)
                        if (orb[c] == hi) orb[c] = lo;
            }
        }
        // advance the mixed-radix product of per-class permutations; a class
        // that wraps is back in ascending order and carries into the next
        int c = ncls - 1;
        while (c >= 0 && !next_perm_range(ord, start[c], start[c + 1])) --c;
        if (c < 0) break;
    }
    Canon r;
    uint64_t labs = 0;
    for (int i = 0; i < n; ++i) labs = (labs << 6) | (uint64_t)lab_at(L, best[i]);
    r.code = (labs << (n * (n - 1) / 2)) | bestseq;
    r.slots = 0;
    r.orbits = 0;
    for (int i = 0; i < n; ++i) {
        r.orbits |= (uint32_t)orb[i] << (3 * i);
        r.slots |= (uint32_t)orb[i] << (3 * best[i]);
    }
    return r;
}

// Fields of a pattern-table key: canonical code in the low bits (labels then
// pair-bit sequence), graph id of a batch from bit 52.  A size-n code takes
// n(n-1)/2 + 6n bits: 51 at n = 6, 63 at n = 7, so only sizes <= 6 carry a
// graph id (size 7 is mined one graph at a time).
constexpr int CODE_GRAPH_SHIFT = 52;

FSM_HD constexpr bool code_has_graph(int n) { return n * (n - 1) / 2 + 6 * n <= CODE_GRAPH_SHIFT; }

FSM_HD int code_label(uint64_t code, int n, int i) {
    return (int)((code >> (n * (n - 1) / 2 + 6 * (n - 1 - i))) & 63u);
}

FSM_HD uint32_t code_seq(uint64_t code, int n) {
    return (uint32_t)(code & ((1ull << (n * (n - 1) / 2)) - 1));
}

FSM_HD int code_graph(uint64_t code, int n) {
    return code_has_graph(n) ? (int)(code >> CODE_GRAPH_SHIFT) : 0;
}

// Graph id of a size-n pattern key, or -1 when it names no graph of a call
// with `graphs` graphs.
FSM_HD int checked_code_graph(uint64_t code, int n, int graphs) {
    if (n < 2 || n > MAXN) return -1;
    const int gi = code_graph(code, n);
    return gi < graphs ? gi : -1;
}

}  // namespace fsm
