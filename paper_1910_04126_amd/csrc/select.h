// Top-k selection per row (see select.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ft {

// For each of `rows` rows of n keys (row-major), write the k smallest
// (key, doc) pairs ascending; doc = docs[row * n + c] when docs is given, else
// the column c.  minmax, when given, holds each row's smallest and largest
// key ([rows][2]).  exact_rows, when given, counts the rows of more than 4096
// keys whose sampled one-pass select fell back to the exact path.  Launches
// only.
void topk_rows(const uint64_t* keys, int64_t rows, int64_t n, const int64_t* docs, int k, uint64_t* out_key,
               int64_t* out_doc, hipStream_t s, const uint64_t* minmax = nullptr, uint32_t* exact_rows = nullptr);
// u32 keys in units of 2^shift: the selected keys are written widened,
// out_key = key << shift (tmp_key: [rows * k] scratch).
void topk_rows(const uint32_t* keys, int64_t rows, int64_t n, const int64_t* docs, int k, uint64_t* out_key, int shift,
               int64_t* out_doc, uint32_t* tmp_key, hipStream_t s, const uint64_t* minmax,
               uint32_t* exact_rows = nullptr);
void topk_rows(const float* keys, int64_t rows, int64_t n, const int64_t* docs, int k, float* out_key,
               int64_t* out_doc, hipStream_t s);

}  // namespace ft
