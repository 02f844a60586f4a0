// Internal interface of the batched probe (plans and the serving loop build
// on it).
#pragma once

#include "lj_internal.h"

namespace lj {

constexpr uint32_t kMaxBranches = 16;

uint64_t align256(uint64_t v);
// Size class of a batch: m < 2^13, < 2^17, < 2^21, larger.
int size_class(uint64_t m);
void default_tuning(lj_batch_tuning* t);
int validate_tuning(const lj_batch_tuning& t);
int validate_descs(const lj_batch_desc* d, uint32_t k, int device);
// Probe form of a batch of m keys under tuning t (see uses_binned).
int batch_mode(const lj_batch_tuning& t, uint64_t m);
// Enqueue one batch (a probe, or zeroing the count of an empty batch) with
// workspace `ws` of at least ws_bytes(d.index, d.m, mode) bytes.
hipError_t enqueue_one(const lj_batch_desc& d, void* ws, uint32_t kpl, int mode,
                       hipStream_t st);

}  // namespace lj
