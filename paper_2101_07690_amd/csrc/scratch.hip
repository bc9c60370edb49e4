// scratch.hip -- device scratch of the allocation-free entry point
// (fsm_mine_noalloc): one file-scope device array, which every GPU the
// library runs on holds until the process ends, carved by a host-side
// first-fit arena for the duration of one call.
//
// In host code `scratch` names a host-side stand-in, not the device array:
// the device address is taken once per device with hipGetSymbolAddress
// (that device current) and only that address is handed to kernels, copies
// and fills.
#include <map>
#include <mutex>

#include "internal.h"

namespace fsm {
namespace {

constexpr size_t SCRATCH_BYTES = (size_t)FSM_NOALLOC_SCRATCH_MIB << 20;
constexpr size_t ALIGN = 256;
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

std::mutex g_base_mu;
uint8_t* g_base[MAX_DEVICES] = {};   // device address of each device's array
std::mutex g_call_mu[MAX_DEVICES];   // one allocation-free call per device at a time

thread_local Arena* g_active = nullptr;

}  // namespace

Arena::Arena(uint8_t* b, size_t n) : base(b), size(n) { free_[0] = n; }

void* Arena::alloc(size_t bytes) {
    const size_t need = (bytes + ALIGN - 1) / ALIGN * ALIGN;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < need) continue;
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > need) free_[off + need] = len - need;
        used_[off] = need;
        in_use += need;
        if (in_use > peak) peak = in_use;
        return base + off;
    }
    return nullptr;
}

void Arena::release(void* p) {
    const size_t off = (size_t)((uint8_t*)p - base);
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, len = u->second;
    in_use -= len;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
        len += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == start) {
            start = prev->first;
            len += prev->second;
            free_.erase(prev);
        }
    }
    free_[start] = len;
}

size_t Arena::largest_free() const {
    size_t m = 0;
    for (const auto& f : free_) m = f.second > m ? f.second : m;
    return m;
}

Arena* active_arena() { return g_active; }

ArenaScope::ArenaScope(Arena* a) : prev(g_active) { g_active = a; }
ArenaScope::~ArenaScope() { g_active = prev; }

size_t scratch_bytes() { return SCRATCH_BYTES; }

uint8_t* scratch_base(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) fail(FSM_EUNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_base_mu);
    if (!g_base[dev]) {
        void* p = nullptr;
        // the caller made `dev` current: its copy of the array
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(FSM_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                 hipGetErrorString(e));
        g_base[dev] = static_cast<uint8_t*>(p);
    }
    return g_base[dev];
}

std::mutex& scratch_lock(int dev) { return g_call_mu[dev]; }

}  // namespace fsm
