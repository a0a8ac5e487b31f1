// Device hash set of determinants (open addressing, 64-bit CAS inserts).
// Keys: for norb <= 31 a determinant packs into one word (alpha << 32 |
// beta); otherwise alpha and beta strings are interned in their own sets
// and the key is the pair of their slot indices.  Set contents never depend
// on the order of concurrent inserts.
#pragma once

#include "common.h"

namespace hset {
namespace {  // kernels below get internal linkage in every including file

constexpr u64 EMPTY = ~0ull;
constexpr int MAX_PROBE = 1 << 12;

__device__ __forceinline__ u64 hmix(u64 x) {
    x ^= x >> 31;
    x *= 0x7fb5d329728ea185ull;
    x ^= x >> 27;
    x *= 0x81dadef4bc2dd44dull;
    x ^= x >> 33;
    return x;
}

// Insert `key` (or find it).  Returns the slot, or -1 after MAX_PROBE probes.
__device__ __forceinline__ i64 hash_insert(u64* __restrict__ table, u64 mask, u64 key, bool& fresh) {
    u64 h = hmix(key) & mask;
    for (int probe = 0; probe < MAX_PROBE; ++probe) {
        const u64 cur = table[h];
        if (cur == key) {
            fresh = false;
            return (i64)h;
        }
        if (cur == EMPTY) {
            const u64 prev = atomicCAS((unsigned long long*)&table[h], (unsigned long long)EMPTY,
                                       (unsigned long long)key);
            if (prev == EMPTY) {
                fresh = true;
                return (i64)h;
            }
            if (prev == key) {
                fresh = false;
                return (i64)h;
            }
        }
        h = (h + 1) & mask;
    }
    fresh = false;
    return -1;
}

struct HashSet {
    u64* det;       // determinant keys
    u64 det_mask;
    u64* sa;        // alpha strings (two-level keys only)
    u64 sa_mask;
    u64* sb;        // beta strings
    u64 sb_mask;
    int packed;     // 1: key = alpha << 32 | beta
    unsigned long long* overflow;  // bit 0: the determinant table, bit 1: a string table
    unsigned long long* strings;  // [0] alpha, [1] beta strings interned
};

constexpr unsigned long long OVER_DET = 1ull, OVER_STR = 2ull;

// Determinant key, interning the strings when keys are two-level.
__device__ __forceinline__ bool det_key(const HashSet& H, u64 a, u64 b, u64& key) {
    if (H.packed) {
        key = (a << 32) | b;
        return true;
    }
    bool fa, fb;
    const i64 ka = hash_insert(H.sa, H.sa_mask, a, fa);
    const i64 kb = hash_insert(H.sb, H.sb_mask, b, fb);
    if (ka < 0 || kb < 0) return false;
    if (fa) atomicAdd(&H.strings[0], 1ull);
    if (fb) atomicAdd(&H.strings[1], 1ull);
    key = ((u64)ka << 32) | (u64)kb;
    return true;
}

// t[0, n) = v, striding over a grid that may be smaller than n (tables of
// 2^32 slots would pass the 2^32 work-items of one launch)
__global__ void fill_kernel(u64* __restrict__ t, i64 n, u64 v) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) t[i] = v;
}

__global__ void insert_v_kernel(HashSet H, const u64* __restrict__ dets, i64 N) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    u64 key;
    bool fresh;
    if (!det_key(H, dets[2 * i], dets[2 * i + 1], key)) atomicOr(H.overflow, OVER_STR);
    else if (hash_insert(H.det, H.det_mask, key, fresh) < 0) atomicOr(H.overflow, OVER_DET);
}


// Look `key` up without inserting.  Returns the slot or -1.
__device__ __forceinline__ i64 hash_find(const u64* __restrict__ table, u64 mask, u64 key) {
    u64 h = hmix(key) & mask;
    for (int probe = 0; probe < MAX_PROBE; ++probe) {
        const u64 cur = table[h];
        if (cur == key) return (i64)h;
        if (cur == EMPTY) return -1;
        h = (h + 1) & mask;
    }
    return -1;
}

// Is (a, b) in the set?  (no inserts, also for two-level keys)
__device__ __forceinline__ bool det_contains(const HashSet& H, u64 a, u64 b) {
    u64 key;
    if (H.packed) {
        key = (a << 32) | b;
    } else {
        const i64 ka = hash_find(H.sa, H.sa_mask, a);
        if (ka < 0) return false;
        const i64 kb = hash_find(H.sb, H.sb_mask, b);
        if (kb < 0) return false;
        key = ((u64)ka << 32) | (u64)kb;
    }
    return hash_find(H.det, H.det_mask, key) >= 0;
}

}  // namespace
}  // namespace hset
