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
//
// A batch ends in one of two ways: its launch failed (a copy, the validate
// call or the graph could not be issued), or the worker saw its completion
// event.  Either way complete_batch turns every request of the batch into a
// completion record at once: status 0 with the module's result when the batch
// ran, else the error status with a zero result; the slot is free again.
#pragma once

#include <stdint.h>
#include <string.h>

#include <vector>

#include "../../include/spvgpu.h"

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

// Completion records of a finished batch.  req_at(i) gives the i-th request
// of the batch (fields id and t_arr_ns); res is the batch's result array, or
// nullptr when status != 0 (results are then zero).
template <class ReqAt>
inline void complete_batch(int64_t n, ReqAt req_at, const spv_result* res, int status, int64_t t_done_ns,
                           std::vector<spv_completion>& out) {
  for (int64_t i = 0; i < n; ++i) {
    spv_completion c;
    memset(&c, 0, sizeof(c));
    c.id = req_at(i).id;
    if (status == 0 && res) c.result = res[i];
    c.status = status;
    c.t_arrival_ns = req_at(i).t_arr_ns;
    c.t_done_ns = t_done_ns;
    c.batch_modules = n;
    out.push_back(c);
  }
}

}  // namespace spv
