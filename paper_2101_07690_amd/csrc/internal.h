// internal.h -- host-side plumbing shared by the library's sources: device
// buffers through the caller's allocation hooks, the current stream, error
// reporting, and the graph / result objects behind the C ABI handles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fsm.h"

namespace fsm {

// Internal failure carrying an fsm_status; caught at the ABI boundary.
struct Failure {
    int code;
};

void set_error(const char* fmt, ...);
[[noreturn]] void fail(int code, const char* fmt, ...);

#define FSM_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            ::fsm::fail(e_ == hipErrorOutOfMemory ? FSM_ENOMEM : FSM_EDEVICE,      \
                        "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__,  \
                        __LINE__);                                                 \
    } while (0)

#define FSM_LAUNCH_CHECK() FSM_HIP(hipGetLastError())

hipStream_t stream();

// First-fit arena over one device range (the allocation-free entry point's
// scratch array): device buffers of a call come from it while it is the
// thread's active arena, and go back to it when released.
struct Arena {
    uint8_t* base;
    size_t size;
    size_t in_use = 0, peak = 0;
    Arena(uint8_t* b, size_t n);
    void* alloc(size_t bytes);     // nullptr when no free range is large enough
    void release(void* p);
    size_t free_bytes() const { return size - in_use; }
    size_t largest_free() const;

  private:
    std::map<size_t, size_t> free_, used_;   // offset -> length
};

Arena* active_arena();   // this thread's arena, or nullptr
struct ArenaScope {      // makes an arena this thread's active one
    Arena* prev;
    explicit ArenaScope(Arena* a);
    ~ArenaScope();
    ArenaScope(const ArenaScope&) = delete;
    ArenaScope& operator=(const ArenaScope&) = delete;
};
size_t scratch_bytes();           // size of the scratch array
uint8_t* scratch_base(int dev);   // its device address on `dev` (current)
std::mutex& scratch_lock(int dev);

void* raw_alloc(size_t bytes, void** release_ctx, void (**release)(void*, void*));

// Device allocation owned by one object; freed with the hook that made it.
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    void (*rel)(void*, void*) = nullptr;
    void* ctx = nullptr;

    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept { swap(o); }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) { reset(); swap(o); }
        return *this;
    }
    ~DBuf() { reset(); }

    void swap(DBuf& o) noexcept {
        std::swap(p, o.p); std::swap(n, o.n); std::swap(rel, o.rel); std::swap(ctx, o.ctx);
    }
    void alloc(size_t count) {
        reset();
        if (count == 0) count = 1;
        p = static_cast<T*>(raw_alloc(count * sizeof(T), &ctx, &rel));
        n = count;
    }
    void reset() {
        if (p && rel) rel(p, ctx);
        p = nullptr; n = 0; rel = nullptr; ctx = nullptr;
    }
    size_t bytes() const { return n * sizeof(T); }
    void zero() {
        if (p) FSM_HIP(hipMemsetAsync(p, 0, bytes(), stream()));
    }
    void fill_bytes(int v) {
        if (p) FSM_HIP(hipMemsetAsync(p, v, bytes(), stream()));
    }
};

// Host waits on the device made by this thread (stream or event
// synchronisations), counted for the call statistics.
int64_t& host_syncs();

inline void sync_stream(hipStream_t s) {
    ++host_syncs();
    FSM_HIP(hipStreamSynchronize(s));
}

template <class T>
void to_host(std::vector<T>& h, const T* d, size_t count) {
    h.resize(count);
    if (count) FSM_HIP(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, stream()));
    sync_stream(stream());
}

template <class T>
void to_host_into(T* h, const T* d, size_t count) {
    if (count) FSM_HIP(hipMemcpyAsync(h, d, count * sizeof(T), hipMemcpyDeviceToHost, stream()));
    sync_stream(stream());
}

template <class T>
T scalar_to_host(const T* d) {
    T v;
    FSM_HIP(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, stream()));
    sync_stream(stream());
    return v;
}

template <class T>
void to_device(T* d, const T* h, size_t count) {
    if (count) FSM_HIP(hipMemcpyAsync(d, h, count * sizeof(T), hipMemcpyHostToDevice, stream()));
}

// Exclusive prefix sum of n int64 values (in == out allowed); returns the total.
int64_t scan_exclusive(const int64_t* in, int64_t* out, int64_t n);

// Sort (key, value) pairs by key within every segment [off[s], off[s+1]).
void sort_segments(const uint64_t* keys_in, uint64_t* keys_out, const uint8_t* vals_in,
                   uint8_t* vals_out, int items, int segments, const int32_t* off);

inline unsigned grid_for(int64_t items, int per_block, unsigned cap = 1u << 20) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (int64_t)cap) g = cap;
    return (unsigned)g;
}

}  // namespace fsm

// Objects behind the opaque ABI handles.
struct fsm_graph {
    int device = 0;
    int64_t n = 0;             // vertices
    int64_t nnz = 0;           // directed CSR entries (2 x undirected edges)
    int32_t num_labels = 0;    // distinct labels
    fsm::DBuf<int32_t> row;    // n+1
    fsm::DBuf<int32_t> col;    // nnz, ascending within each row
    fsm::DBuf<int32_t> lab;    // n, dense label rank 0..num_labels-1
    std::vector<int32_t> label_value;   // rank -> caller's label
    std::vector<int64_t> label_count;   // vertices per rank
    int64_t dropped_loops = 0;
    int64_t dropped_dups = 0;
};

struct fsm_result {
    std::vector<int32_t> size;
    std::vector<fsm_code> code;
    std::vector<int64_t> support;
    fsm_stats stats{};
    std::vector<float> tx, tt;      // recorded work-item rows: features, targets
    std::vector<int32_t> tl;        // join size of each row
};

namespace fsm {
void build_graph(fsm_graph* g, int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                 const int32_t* labels);
void mine(const fsm_graph* g, const fsm_options& opt, fsm_result* r);
// fsm_mine_ex with every device buffer taken from the thread's active arena
// and no HIP events (timings 0).
void mine_in_arena(const fsm_graph* g, const fsm_options& opt, fsm_result* r);
void mine_batch(const fsm_graph* const* gs, int32_t count, const int64_t* supports,
                const fsm_batch_options& opt, fsm_result* const* rs);
// Shapes used where a call leaves chunk_vertices / tiles_per_wave at 0
// (0: the built-in defaults).
void set_tuning(int64_t chunk_vertices, int32_t tiles_per_wave);
void tune_batch(const fsm_graph* const* gs, int32_t count, const int64_t* supports,
                int32_t max_size, fsm_tuning* out);
void proposal_keep_thresholds(const float* pred, int64_t rows, double rate, uint64_t* thr);
}  // namespace fsm
