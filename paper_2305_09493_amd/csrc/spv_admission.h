// Admission rules of the validation server, free of HIP so that they can be
// built and tested on the host alone.
//
// A free slot takes arrived requests in arrival order (FIFO) while the batch
// stays within the slot: at most max_batch modules, at most cap_modules - 1
// modules (room for the padding module of a captured graph), and at most
// cap_words - 1 words (room for the padding word).  A request larger than a
// slot can ever hold (n > cap_words - 1) is rejected when it reaches the
// front of the queue; the first request that fits no more ends the batch and
// waits for the next free slot.
#pragma once

#include <stdint.h>

namespace spv {

enum AdmitAction : uint8_t { kAdmitTake = 1, kAdmitReject = 2 };

// Decide the next batch of one free slot.  size_at(i) is the word count of
// the i-th request waiting at the front of the queue (i < n_ready).  Writes
// one action per examined request (a prefix of the queue) and returns how
// many were examined; the taken ones form the batch, in order.
template <class SizeAt>
inline int64_t admit_batch(int64_t n_ready, SizeAt size_at, int64_t max_batch, int64_t cap_modules,
                           int64_t cap_words, uint8_t* action) {
  int64_t i = 0, M = 0, W = 0;
  while (i < n_ready && M < max_batch && M + 2 <= cap_modules) {
    const int64_t n = size_at(i);
    if (n > cap_words - 1) {
      action[i++] = kAdmitReject;
      continue;
    }
    if (W + n > cap_words - 1) break;
    action[i++] = kAdmitTake;
    W += n;
    ++M;
  }
  return i;
}

// Padded size of a captured graph's batch: x rounded up to a multiple of
// 2^(floor(log2 x) - 3) (at least 64), so at most 12.5% padding and few
// distinct sizes.
inline int64_t bucket_up(int64_t x) {
  if (x <= 64) return 64;
  const int lg = 63 - __builtin_clzll(uint64_t(x));
  const int64_t step = int64_t(1) << (lg - 3);
  return (x + step - 1) / step * step;
}

}  // namespace spv
