// Fermion phases of excitations on 64-bit occupation words (orbital p is
// bit p), shared by every kernel that evaluates a matrix element or a
// density-matrix contribution.  Written for host and device from 32-bit
// halves and shifts by less than 32 (no mask table, no 64-bit variable
// shift), so the same code can be checked exhaustively on the CPU.
#pragma once

#include <stdint.h>

#ifndef HCI_HD
#if defined(__HIPCC__) || defined(__HIP__)
#define HCI_HD __host__ __device__ __forceinline__
#else
#define HCI_HD inline
#endif
#endif

// bits [0, k) of a 32-bit word, 0 <= k <= 32
HCI_HD uint32_t phase_mask32(int k) { return k >= 32 ? 0xffffffffu : ((1u << (k & 31)) - 1u); }

// number of set bits of s below position k (0 <= k <= 64)
HCI_HD int phase_rank_below(uint64_t s, int k) {
    const uint32_t lo = (uint32_t)s, hi = (uint32_t)(s >> 32);
    const int klo = k < 32 ? k : 32, khi = k > 32 ? k - 32 : 0;
    return __builtin_popcount(lo & phase_mask32(klo)) + __builtin_popcount(hi & phase_mask32(khi));
}

// number of set bits of s strictly between orbitals p and q (p != q)
HCI_HD int phase_count_between(uint64_t s, int p, int q) {
    const int lo = p < q ? p : q, hi = p < q ? q : p;
    return phase_rank_below(s, hi) - phase_rank_below(s, lo + 1);
}

// (-1)^(number of set bits of s strictly between orbitals p and q)
HCI_HD double phase_sign_between(uint64_t s, int p, int q) {
    return (phase_count_between(s, p, q) & 1) ? -1.0 : 1.0;
}

// Phase of the same-spin double p -> r then q -> s applied to string si
// (p, q occupied; r, s empty): the second count is taken on si with p
// removed and r added, i.e. it changes by one for each of p, r that lies
// strictly between q and s.
HCI_HD double phase_sign_double(uint64_t si, int p, int r, int q, int s) {
    const int lo = q < s ? q : s, hi = q < s ? s : q;
    const int n = phase_count_between(si, p, r) + phase_count_between(si, q, s) + (p > lo && p < hi) +
                  (r > lo && r < hi);
    return (n & 1) ? -1.0 : 1.0;
}
