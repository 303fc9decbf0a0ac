// Launcher of ko_rounds.hip (internal to libko): makespans under the
// round-synchronous model.  Returns a hipError_t value as int.
#pragma once

#include <stdint.h>

#include "ko_device.h"

namespace ko {

struct RoundsArgs {
    KernelRec k[kMaxSet];     // derived records of the set, by kernel index
    uint32_t c0[kMaxSet];     // blocks of each kernel that fit one empty CU (>= 1)
    const uint8_t *orders;    // [count][n], order[j] = kernel at position j; or NULL:
                              // lexicographic ranks first .. first+count-1
    int64_t *makespans;       // [count]; -1 for an order with an index >= n
    uint64_t first;
    uint64_t count;
    uint32_t n, n_cu;
    uint32_t cap_reg, cap_lds, cap_wave, cap_blk;
    float inv_ncu;            // 1/n_cu rounded up by 3 ulps (exact quotients below 2^18)
};

int launch_rounds(const RoundsArgs &a, void *stream);

}  // namespace ko
