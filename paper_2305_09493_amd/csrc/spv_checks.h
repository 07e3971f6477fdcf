// Argument checks that run on the device (SPV_OPT_DEBUG_CHECKS) and on the
// host alike.  They are constexpr, so HIP compiles them for both sides, and
// free of HIP, so that a host-only test can build them with g++.
//
// Batch model: module m is words[mod_off[m] .. mod_off[m+1]) of a batch of
// W words; the offsets start at 0, never decrease and end at W, and a module
// has fewer than 2^32 words (its word offsets are 32-bit).
#pragma once

#include <stdint.h>

namespace spv {

// Consecutive offsets a = mod_off[m], b = mod_off[m+1].
constexpr bool offsets_pair_ok(int64_t a, int64_t b) { return a <= b && b - a < (int64_t(1) << 32); }

// First and last offset of a batch of W words.
constexpr bool offsets_ends_ok(int64_t first, int64_t last, int64_t W) { return first == 0 && last == W; }

}  // namespace spv
