// Pair descriptors and bucket indices shared by the PT2 partition passes
// (k_pt2_part.hip) and the reduce (k_pt2_reduce.hip).
#pragma once
#include "dnqs_device.h"

namespace dnqs {

constexpr int kL1Threads = 1024;       // L1 workgroup
constexpr int kL1XPerGroup = 64;       // determinants per L1 workgroup
constexpr int kL1Round = 8192;         // descriptors staged in LDS per L1 round (8 per thread)
constexpr int kL2Threads = 1024;       // staged L2 workgroup
constexpr int kL2Round = 16384;        // descriptors staged per L2 round (16 per thread)
constexpr int kMaxK1 = 1024;
constexpr int kMaxK2 = 4096;
constexpr int kMaxK2Staged = 1024;     // sub-buckets per L1 bucket the staged L2 pass handles
constexpr int kRedThreads = 512;
constexpr int kRedTab = 3072;  // LDS hash-table slots per sub-bucket (a multiple of kRedThreads)
constexpr int kRedPart = 8;    // doubles of per-sub-bucket output (see k_pt2_reduce)
constexpr int kRedSingles = 256;  // single-excitation pairs a reduce workgroup queues in LDS

__device__ __forceinline__ uint32_t l1_bucket(uint64_t h, int s1) { return s1 ? (uint32_t)(h >> (64 - s1)) : 0u; }

__device__ __forceinline__ uint32_t l2_bucket(uint64_t h, int s1, int s2) {
    return s2 ? (uint32_t)((h << s1) >> (64 - s2)) : 0u;
}

constexpr int kDescXBits = 24;
constexpr int kDescHashBits = 12;

__device__ __forceinline__ uint64_t make_desc(int64_t x, uint32_t pos, uint64_t h, int s1) {
    const uint64_t l2b = (h << s1) >> (64 - kDescHashBits);
    return (uint64_t)x | ((uint64_t)pos << kDescXBits) | (l2b << (kDescXBits + 28));
}
__device__ __forceinline__ int64_t desc_x(uint64_t d) { return (int64_t)(d & ((1ull << kDescXBits) - 1)); }
__device__ __forceinline__ uint32_t desc_pos(uint64_t d) { return (uint32_t)((d >> kDescXBits) & 0xfffffffull); }
__device__ __forceinline__ uint32_t desc_sub(uint64_t d, int s2) {
    return s2 ? (uint32_t)(d >> (64 - s2)) : 0u;
}

}  // namespace dnqs
