// Frame-sequence rules of the serving mailbox, free of HIP so that host tests
// can compile them on their own.
#pragma once

#include <stdint.h>

namespace rtc {

// The loop publishes frame q's commands into mailbox slot q % depth and reuses
// that slot for frame q + depth, which the host may start once frame q is
// published.  A copy of the slot taken after frame q was published is whole
// if, once the copy has ended, the host had started no frame beyond
// q + depth - 1 (seq_after_copy: frames started so far; the loop writes a
// frame's commands only after the host started it), as in a seqlock.
inline bool mailbox_copy_whole(uint64_t seq_after_copy, uint64_t q, uint64_t depth) {
    return seq_after_copy <= q + depth;
}

// Each of n tiles raises its flag to q + 1 once its commands of frame q are in
// the mailbox, and a tile's frames are integrated in order, so its flag only
// grows: frame q is out when every flag has reached q + 1.  Scanning from
// tile `from` (the tiles before it known to have), returns the first tile
// whose flag (flag(t), an acquire load) has not, or n.
template <class Flag>
inline int tiles_ready_from(Flag flag, int n, uint64_t q, int from) {
    int t = from;
    while (t < n && flag(t) >= q + 1) ++t;
    return t;
}

}  // namespace rtc
