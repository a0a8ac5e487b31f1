// Hamiltonian matrix elements between determinants of excitation degree
// <= 2 (textbook Slater-Condon rules for the active-space Hamiltonian) and
// the wave-cooperative enumeration of the connections of one row of V.
#pragma once

#include "common.h"

// Single excitation p -> q in string `same` (its spin), `other` the
// opposite-spin string: h_qp + sum_{r in same} [(qp|rr) - (qr|rp)] +
// sum_{r in other} (qp|rr), summed in that order with r ascending (the
// order is part of the contract: selection compares this float64 value
// against a threshold and must match any other evaluation bit for bit).
__device__ __forceinline__ double single_elem_f64(const IntView& I, u64 same, u64 other, int p,
                                                  int q) {
    const int n = I.n;
    const i64 row = ((i64)q * n + p) * n;
    double v = I.h[(i64)q * n + p];
    for (u64 m = same; m; m &= m - 1) v += I.jk[row + ctz64(m)];
    for (u64 m = other; m; m &= m - 1) v += I.jj[row + ctz64(m)];
    return v;
}

__device__ __forceinline__ float single_elem_f32(const IntView& I, u64 same, u64 other, int p,
                                                 int q) {
    const int n = I.n;
    const i64 row = ((i64)q * n + p) * n;
    float v = I.h32[(i64)q * n + p];
    for (u64 m = same; m; m &= m - 1) v += I.jk32[row + ctz64(m)];
    for (u64 m = other; m; m &= m - 1) v += I.jj32[row + ctz64(m)];
    return v;
}

__device__ __forceinline__ i64 gidx(int n, int p, int q, int r, int s) {
    return (((i64)p * n + q) * n + r) * n + s;
}

// <D_j|H|D_i> for D_j != D_i at excitation degree 1 or 2 (float64).
__device__ __forceinline__ double hij_f64(const IntView& I, u64 ai, u64 bi, u64 aj, u64 bj) {
    const u64 xa = ai ^ aj, xb = bi ^ bj;
    const int da = popc64(xa) >> 1, db = popc64(xb) >> 1;
    const int n = I.n;
    if (db == 0 && da == 1) {
        const int p = ctz64(ai & xa), q = ctz64(aj & xa);
        return sign_between(ai, p, q) * single_elem_f64(I, ai, bi, p, q);
    }
    if (da == 0 && db == 1) {
        const int p = ctz64(bi & xb), q = ctz64(bj & xb);
        return sign_between(bi, p, q) * single_elem_f64(I, bi, ai, p, q);
    }
    if (da == 1 && db == 1) {
        const int p = ctz64(ai & xa), r = ctz64(aj & xa);
        const int q = ctz64(bi & xb), s = ctz64(bj & xb);
        return (sign_between(ai, p, r) * sign_between(bi, q, s)) * I.g[gidx(n, r, p, s, q)];
    }
    const u64 si = da == 2 ? ai : bi;
    const u64 x = da == 2 ? xa : xb;
    u64 holes = si & x, parts = x & ~si;
    const int p = ctz64(holes);
    holes &= holes - 1;
    const int q = ctz64(holes);
    const int r = ctz64(parts);
    parts &= parts - 1;
    const int s = ctz64(parts);
    const double sg = sign_double(si, p, r, q, s);
    return sg * (I.g[gidx(n, r, p, s, q)] - I.g[gidx(n, r, q, s, p)]);
}

__device__ __forceinline__ float hij_f32(const IntView& I, u64 ai, u64 bi, u64 aj, u64 bj) {
    const u64 xa = ai ^ aj, xb = bi ^ bj;
    const int da = popc64(xa) >> 1, db = popc64(xb) >> 1;
    const int n = I.n;
    if (db == 0 && da == 1) {
        const int p = ctz64(ai & xa), q = ctz64(aj & xa);
        return (float)sign_between(ai, p, q) * single_elem_f32(I, ai, bi, p, q);
    }
    if (da == 0 && db == 1) {
        const int p = ctz64(bi & xb), q = ctz64(bj & xb);
        return (float)sign_between(bi, p, q) * single_elem_f32(I, bi, ai, p, q);
    }
    if (da == 1 && db == 1) {
        const int p = ctz64(ai & xa), r = ctz64(aj & xa);
        const int q = ctz64(bi & xb), s = ctz64(bj & xb);
        return (float)(sign_between(ai, p, r) * sign_between(bi, q, s)) * I.g32[gidx(n, r, p, s, q)];
    }
    const u64 si = da == 2 ? ai : bi;
    const u64 x = da == 2 ? xa : xb;
    u64 holes = si & x, parts = x & ~si;
    const int p = ctz64(holes);
    holes &= holes - 1;
    const int q = ctz64(holes);
    const int r = ctz64(parts);
    parts &= parts - 1;
    const int s = ctz64(parts);
    const float sg = (float)sign_double(si, p, r, q, s);
    return sg * (I.g32[gidx(n, r, p, s, q)] - I.g32[gidx(n, r, q, s, p)]);
}

// Diagonal <D|H|D> (ecore excluded): occupied one-body energies plus, for
// every unordered pair of occupied spin orbitals, Coulomb minus same-spin
// exchange.
__device__ __forceinline__ double diag_f64(const IntView& I, u64 a, u64 b) {
    const int n = I.n;
    double e = 0.0;
    for (u64 m = a; m; m &= m - 1) {
        const int p = ctz64(m);
        e += I.h[(i64)p * n + p];
        for (u64 m2 = m & (m - 1); m2; m2 &= m2 - 1) {
            const int q = ctz64(m2);
            e += I.jdiag[(i64)p * n + q] - I.kdiag[(i64)p * n + q];
        }
        for (u64 m2 = b; m2; m2 &= m2 - 1) e += I.jdiag[(i64)p * n + ctz64(m2)];
    }
    for (u64 m = b; m; m &= m - 1) {
        const int p = ctz64(m);
        e += I.h[(i64)p * n + p];
        for (u64 m2 = m & (m - 1); m2; m2 &= m2 - 1) {
            const int q = ctz64(m2);
            e += I.jdiag[(i64)p * n + q] - I.kdiag[(i64)p * n + q];
        }
    }
    return e;
}

__device__ __forceinline__ u32 lower_bound_u64(const u64* __restrict__ arr, u32 len, u64 key) {
    u32 lo = 0, hi = len;
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (arr[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first index in sorted arr[0, len) whose value is >= key (u32)
__device__ __forceinline__ u32 lower_bound_u32(const u32* __restrict__ arr, u32 len, u32 key) {
    u32 lo = 0, hi = len;
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (arr[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first index in sorted arr[0, len) whose value is > key (u32)
__device__ __forceinline__ u32 upper_bound_u32(const u32* __restrict__ arr, u32 len, u32 key) {
    u32 lo = 0, hi = len;
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (arr[mid] <= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Index of the n-th (from 0) set bit of m (32-bit halves, no 64-bit
// variable shifts).
__device__ __forceinline__ int nth_set_bit(u64 m, int n) {
    u32 w = lo32(m);
    int base = 0;
    const int c = __popc(w);
    if (n >= c) {
        n -= c;
        w = hi32(m);
        base = 32;
    }
#pragma unroll
    for (int s = 16; s > 0; s >>= 1) {
        const int cl = __popc(w & ((1u << s) - 1u));
        if (n >= cl) {
            n -= cl;
            w >>= s;
            base += s;
        }
    }
    return base;
}

// Single excitations of one row, deferred.  Their element sums over every
// occupied orbital; they are a few percent of a row's connections, but
// nearly every wavefront of 64 holds one and would run that path for all
// lanes.  The wavefront queues them instead (slot l in lane l) and evaluates
// up to 64 at once.  Every lane calls push together; the caller flushes
// (lanes below n evaluate their slot) when full_for says so and at the end
// of the row.
struct SinglesQueue {
    int n = 0;  // queued, wave-uniform
    i64 k = 0;  // this lane's slot: caller's index and the determinant
    u64 a = 0, b = 0;
    __device__ __forceinline__ bool full_for(u64 m) const { return n + popc64(m) > HCI_WAVE; }
    __device__ __forceinline__ void push(u64 m, i64 kk, u64 aa, u64 bb) {
        const int cnt = popc64(m);
        const int l = lane_id();
        const bool mine = l >= n && l < n + cnt;
        const int src = mine ? nth_set_bit(m, l - n) : l;
        const i64 sk = __shfl(kk, src, HCI_WAVE);
        const u64 sa = __shfl(aa, src, HCI_WAVE);
        const u64 sb = __shfl(bb, src, HCI_WAVE);
        if (mine) {
            k = sk;
            a = sa;
            b = sb;
        }
        n += cnt;
    }
};

// Enumerate every j != i in V with excitation degree <= 2 from row i.  The
// whole wavefront calls this for one row; `vis(ok, j, aj, bj)` is invoked
// wave-uniformly, each lane carrying its own candidate (ok = it is one).
// Order of discovery (deterministic): same-alpha bucket, same-beta bucket,
// then alpha-single neighbours in adjacency order.
template <class Visitor>
__device__ __forceinline__ void enumerate_row(const SpaceView& S, u32 i, Visitor& vis) {
    const int lane = lane_id();
    const u64 A = S.alpha[i], B = S.beta[i];
    const u32 a = S.ia[i], b = S.ib[i];
    {  // same alpha string: beta differs by one or two excitations
        const u32 lo = S.aoff[a], hi = S.aoff[a + 1];
        for (u32 base = lo; base < hi; base += HCI_WAVE) {
            const u32 j = base + lane;
            bool ok = j < hi && j != i;
            u64 bj = 0;
            if (ok) {
                bj = S.beta[j];
                ok = popc64(B ^ bj) <= 4;
            }
            vis(ok, j, A, bj);
        }
    }
    {  // same beta string: alpha differs by one or two excitations
        const u32 lo = S.boff[b], hi = S.boff[b + 1];
        for (u32 base = lo; base < hi; base += HCI_WAVE) {
            const u32 k = base + lane;
            bool ok = k < hi;
            u32 j = 0;
            u64 aj = 0;
            if (ok) {
                j = S.permb[k];
                ok = j != i;
                if (ok) {
                    aj = S.alpha[j];
                    ok = popc64(A ^ aj) <= 4;
                }
            }
            vis(ok, j, aj, B);
        }
    }
    {  // one alpha and one beta excitation
        const u32 t0 = S.as_ptr[a], t1 = S.as_ptr[a + 1];
        const u32 s0 = S.bs_ptr[b], s1 = S.bs_ptr[b + 1];
        const u32 nbs = s1 - s0;
        for (u32 t = t0; t < t1; ++t) {
            const u32 a2 = S.as_idx[t];
            const u64 A2 = S.ua[a2];
            const u32 lo = S.aoff[a2], hi = S.aoff[a2 + 1];
            const u32 len = hi - lo;
            if (len <= 4u * nbs) {
                for (u32 base = lo; base < hi; base += HCI_WAVE) {
                    const u32 j = base + lane;
                    bool ok = j < hi;
                    u64 bj = 0;
                    if (ok) {
                        bj = S.beta[j];
                        ok = popc64(B ^ bj) == 2;
                    }
                    vis(ok, j, A2, bj);
                }
            } else {
                for (u32 base = s0; base < s1; base += HCI_WAVE) {
                    const u32 k = base + lane;
                    bool ok = k < s1;
                    u32 j = 0;
                    u64 bj = 0;
                    if (ok) {
                        bj = S.ub[S.bs_idx[k]];
                        const u32 pos = lower_bound_u64(S.beta + lo, len, bj);
                        ok = pos < len && S.beta[lo + pos] == bj;
                        j = lo + pos;
                    }
                    vis(ok, j, A2, bj);
                }
            }
        }
    }
}

// LDS lookup of beta strings in the alpha neighbours [tg0, tg1) of a bucket
// (alpha single x beta single connections): per neighbour a bitmap over the
// unique beta strings (W 32-bit words) with a bit for each beta string present
// in the neighbour's bucket, and per word the number of set bits before it
// (u16: buckets hold fewer than 65536 rows).  Rows of a bucket are sorted by
// beta string, so beta string b sits at position
// pre[b >> 5] + popc(word & bits below b) of the bucket.  Called by all BLOCK
// threads of the workgroup; ends with a barrier.
template <int BLOCK>
__device__ __forceinline__ void build_beta_maps(const SpaceView& S, u32 t0, u32 tg0, u32 tg1, u32 W,
                                                u32* bm, u16* pre, u32 tid) {
    const u32 nt = tg1 - tg0;
    for (u32 x = tid; x < nt * W; x += BLOCK) bm[x] = 0u;
    __syncthreads();
    for (u32 q = 0; q < nt; ++q) {
        const u32 a2 = S.as_idx[t0 + tg0 + q];
        const u32 lo = S.aoff[a2], hi = S.aoff[a2 + 1];
        u32* m = bm + q * W;
        for (u32 j = lo + tid; j < hi; j += BLOCK) {
            const u32 b = S.ib[j];
            atomicOr(&m[b >> 5], 1u << (b & 31u));
        }
    }
    __syncthreads();
    // exclusive prefix of the word popcounts, one wavefront per neighbour
    const u32 lane = (u32)lane_id();
    for (u32 q = tid / HCI_WAVE; q < nt; q += BLOCK / HCI_WAVE) {
        u32 run = 0;
        for (u32 base = 0; base < W; base += HCI_WAVE) {
            const u32 w = base + lane;
            const u32 c = w < W ? (u32)__popc(bm[q * W + w]) : 0u;
            u32 incl = c;
#pragma unroll
            for (int off = 1; off < HCI_WAVE; off <<= 1) {
                const u32 y = (u32)__shfl_up((int)incl, off, HCI_WAVE);
                if ((int)lane >= off) incl += y;
            }
            if (w < W) pre[q * W + w] = (u16)(run + incl - c);
            run += (u32)__shfl((int)incl, HCI_WAVE - 1, HCI_WAVE);
        }
    }
    __syncthreads();
}
