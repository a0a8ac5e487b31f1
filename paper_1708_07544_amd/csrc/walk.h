// Heat-bath walk over the connections of one determinant D_i (Sec.
// "Variational Stage", Fig. 1b): for every occupied pair, the pre-sorted
// list of double-excitation magnitudes is read only while
// fl(|H| * |c_i|) > eps can still hold; singles are evaluated exactly after
// an orbital-only upper bound.  fl(x * c) is monotone in x, so stopping at
// the first failing entry of a descending list is exact, not a heuristic.
#pragma once

#include "slater.h"

struct HBView {
    int n, os_len, ss_len;
    const double* os_abs;
    const u32* os_rs;
    const double* ss_abs;
    const u32* ss_rs;
    const double* single_bound;
};

inline HBView hb_view(const Integrals& I) {
    HBView v;
    v.n = I.n;
    v.os_len = I.os_len;
    v.ss_len = I.ss_len;
    v.os_abs = I.os_abs.as<double>();
    v.os_rs = I.os_rs.as<u32>();
    v.ss_abs = I.ss_abs.as<double>();
    v.ss_rs = I.ss_rs.as<u32>();
    v.single_bound = I.single_bound.as<double>();
    return v;
}

// Walk one sorted list: emit(ok, r, s) is called wave-uniformly per chunk of
// 64 entries; ok marks lanes whose entry passes the magnitude test.
template <class F>
__device__ __forceinline__ void walk_list(const double* __restrict__ mag, const u32* __restrict__ rs,
                                          int len, double ci, double eps, F&& f) {
    if (len <= 0 || !(mag[0] * ci > eps)) return;
    for (int base = 0; base < len; base += HCI_WAVE) {
        const int t = base + lane_id();
        bool pass = false;
        u32 e = 0;
        if (t < len) {
            const double prod = mag[t] * ci;
            pass = prod > eps;
            if (pass) e = rs[t];
        }
        f(pass, (int)(e & 0xffu), (int)((e >> 8) & 0xffu));
        if (!(ballot(pass) >> 63)) return;  // the last lane failed: list exhausted
    }
}

// Visit every determinant D_a connected to D_i = (A, B) with
// fl(|H_ai| * |c_i|) > eps.  visit(ok, aa, ab, is_double) is wave-uniform.
// D_a may belong to V; the caller decides what to do with it.
template <class Visit>
__device__ __forceinline__ void heat_bath_walk(const HBView& T, const IntView& I, u64 A, u64 B,
                                               double ci, double eps, Visit& visit) {
    const int n = T.n;
    // opposite-spin pairs (p alpha, q beta): p -> r, q -> s
    for (u64 ma = A; ma; ma &= ma - 1) {
        const int p = ctz64(ma);
        for (u64 mb = B; mb; mb &= mb - 1) {
            const int q = ctz64(mb);
            const i64 P = (i64)p * n + q;
            walk_list(T.os_abs + P * T.os_len, T.os_rs + P * T.os_len, T.os_len, ci, eps,
                      [&](bool pass, int r, int s) {
                          const bool ok = pass && !test_bit(A, r) && !test_bit(B, s);
                          visit(ok, A ^ bit(p) ^ bit(r), B ^ bit(q) ^ bit(s));
                      });
        }
    }
    // same-spin pairs p < q in each string: p,q -> r,s
    for (int spin = 0; spin < 2; ++spin) {
        const u64 S = spin ? B : A;
        for (u64 mq = S & (S - 1); mq; mq &= mq - 1) {
            const int q = ctz64(mq);
            for (u64 mp = S & low_mask(q); mp; mp &= mp - 1) {
                const int p = ctz64(mp);
                const i64 P = (i64)q * (q - 1) / 2 + p;
                walk_list(T.ss_abs + P * T.ss_len, T.ss_rs + P * T.ss_len, T.ss_len, ci, eps,
                          [&](bool pass, int r, int s) {
                              const bool ok = pass && !test_bit(S, r) && !test_bit(S, s);
                              const u64 S2 = S ^ bit(p) ^ bit(q) ^ bit(r) ^ bit(s);
                              visit(ok, spin ? A : S2, spin ? S2 : B);
                          });
            }
        }
    }
    // singles: lane r takes target orbital r, exact float64 element
    for (int spin = 0; spin < 2; ++spin) {
        const u64 S = spin ? B : A, O = spin ? A : B;
        for (u64 mp = S; mp; mp &= mp - 1) {
            const int p = ctz64(mp);
            const int r = lane_id();
            bool ok = false;
            u64 S2 = 0;
            if (r < n && !test_bit(S, r) && T.single_bound[p * n + r] * ci > eps) {
                const double v = sign_between(S, p, r) * single_elem_f64(I, S, O, p, r);
                const double prod = fabs(v) * ci;
                ok = prod > eps;
                S2 = S ^ bit(p) ^ bit(r);
            }
            visit(ok, spin ? A : S2, spin ? S2 : B);
        }
    }
}
