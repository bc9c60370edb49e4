// pieces.hip -- segmented radix sort of the join's piece lists (hipCUB).
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace fsm {

void sort_segments(const uint64_t* keys_in, uint64_t* keys_out, const uint8_t* vals_in,
                   uint8_t* vals_out, int items, int segments, const int32_t* off) {
    size_t bytes = 0;
    FSM_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(
        nullptr, bytes, keys_in, keys_out, vals_in, vals_out, items, segments, off, off + 1, 0,
        64, stream()));
    DBuf<uint8_t> tmp(bytes > 0 ? bytes : 1);
    FSM_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(
        tmp.p, bytes, keys_in, keys_out, vals_in, vals_out, items, segments, off, off + 1, 0, 64,
        stream()));
    FSM_HIP(hipStreamSynchronize(stream()));
}

}  // namespace fsm
