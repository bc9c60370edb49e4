// tune.cpp -- autotuning of the batch shapes (chunk size, tile height).
#include <chrono>
#include <cstring>
#include <vector>

#include "internal.h"

namespace fsm {

// Every candidate is timed twice (the faster counts): a single call can be
// slowed by first-use allocations or a rerun after a table overflow.
void tune_batch(const fsm_graph* const* gs, int32_t count, const int64_t* supports,
                int32_t max_size, fsm_tuning* out) {
    static const int64_t chunks[] = {8192, 16384, 32768};
    static const int32_t tiles[] = {4, 16, 64};
    std::vector<fsm_result> rs((size_t)count);
    std::vector<fsm_result*> rp;
    for (auto& r : rs) rp.push_back(&r);
    auto run = [&](int64_t cv, int32_t tpw) {
        fsm_batch_options bo;
        memset(&bo, 0, sizeof(bo));
        bo.max_size = max_size;
        bo.mode = FSM_BATCHED;
        bo.chunk_vertices = cv;
        bo.tiles_per_wave = tpw;
        for (auto& r : rs) r = fsm_result();
        FSM_HIP(hipStreamSynchronize(stream()));
        const auto t0 = std::chrono::steady_clock::now();
        mine_batch(gs, count, supports, bo, rp.data());
        FSM_HIP(hipStreamSynchronize(stream()));
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
            .count();
    };
    run(chunks[1], tiles[1]);   // warm-up: code objects, allocator pools
    memset(out, 0, sizeof(*out));
    double best = 0;
    for (int64_t cv : chunks)
        for (int32_t tpw : tiles) {
            const double a = run(cv, tpw), b = run(cv, tpw);
            const double ms = a < b ? a : b;
            const int c = out->configs++;
            out->cand_chunk[c] = cv;
            out->cand_tiles[c] = tpw;
            out->cand_ms[c] = ms;
            if (c == 0 || ms < best) {
                best = ms;
                out->chunk_vertices = cv;
                out->tiles_per_wave = tpw;
            }
        }
    set_tuning(out->chunk_vertices, out->tiles_per_wave);
}

}  // namespace fsm
