// Spin-traced one- and two-particle (transition) density matrices on V,
//   rdm1[p][q]       = sum_s  <bra| a+_ps a_qs |ket>,
//   rdm2[p][q][r][s] = sum_st <bra| a+_ps a+_rt a_st a_qs |ket>,
// accumulated by looping over the same single and double connections as
// the Hamiltonian product (Sec. "Computational Details").
//
// Diagonal pairs (i = j) only involve occupation numbers, so they are
// reduced without atomics: D[x][y] = sum_i bra_i ket_i n_x(i) n_y(i) over
// spin orbitals x, y, block partials then a fixed-order sum.  Each
// off-diagonal pair (row i, connection j) adds bra_i ket_j times the
// operator matrix element of the excitation D_j -> D_i to the few
// rdm entries it touches, with float64 atomics.
#include <cstdlib>

#include "slater.h"

namespace {

constexpr int ROW_BLOCK = 256;
constexpr int ROWS_PER_BLOCK = ROW_BLOCK / HCI_WAVE;
constexpr int OCC_CHUNK = 256;

__device__ __forceinline__ void add64(double* p, double v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ i64 r2idx(int n, int p, int q, int r, int s) {
    return (((i64)p * n + q) * n + r) * n + s;
}

// contributions of <D_i| ... |D_j> for a single excitation v -> u in the
// string sj (spin s) of D_j, with `other` the opposite-spin string of D_j.
// HALF adds only one entry of each pair (pq|rs), (rs|pq) of rdm2 (the two are
// equal for any bra and ket); the caller then sets rdm2 = T + T^swap.
template <bool HALF>
__device__ __forceinline__ void single_contrib(int n, double x, u64 sj, u64 other, int v, int u,
                                               double* r1, double* r2) {
    add64(&r1[(i64)u * n + v], x);
    if (!r2) return;
    for (u64 m = sj & ~bit(v); m; m &= m - 1) {  // same-spin spectators
        const int k = ctz64(m);
        add64(&r2[r2idx(n, u, v, k, k)], x);
        add64(&r2[r2idx(n, u, k, k, v)], -x);
        if (!HALF) {
            add64(&r2[r2idx(n, k, k, u, v)], x);
            add64(&r2[r2idx(n, k, v, u, k)], -x);
        }
    }
    for (u64 m = other; m; m &= m - 1) {  // opposite-spin spectators
        const int k = ctz64(m);
        add64(&r2[r2idx(n, u, v, k, k)], x);
        if (!HALF) add64(&r2[r2idx(n, k, k, u, v)], x);
    }
}

template <bool HALF>
__device__ __forceinline__ void pair_contrib(int n, double w, u64 ai, u64 bi, u64 aj, u64 bj,
                                             double* r1, double* r2) {
    const u64 xa = ai ^ aj, xb = bi ^ bj;
    const int da = popc64(xa) >> 1, db = popc64(xb) >> 1;
    if (da == 1 && db == 0) {
        const int v = ctz64(aj & xa), u = ctz64(ai & xa);
        single_contrib<HALF>(n, w * sign_between(aj, v, u), aj, bj, v, u, r1, r2);
        return;
    }
    if (da == 0 && db == 1) {
        const int v = ctz64(bj & xb), u = ctz64(bi & xb);
        single_contrib<HALF>(n, w * sign_between(bj, v, u), bj, aj, v, u, r1, r2);
        return;
    }
    if (!r2) return;
    if (da == 1 && db == 1) {
        const int v1 = ctz64(aj & xa), u1 = ctz64(ai & xa);
        const int v2 = ctz64(bj & xb), u2 = ctz64(bi & xb);
        const double x = w * (sign_between(aj, v1, u1) * sign_between(bj, v2, u2));
        add64(&r2[r2idx(n, u1, v1, u2, v2)], x);
        if (!HALF) add64(&r2[r2idx(n, u2, v2, u1, v1)], x);
        return;
    }
    const u64 sj = da == 2 ? aj : bj;
    const u64 x2 = da == 2 ? xa : xb;
    u64 holes = sj & x2, parts = x2 & ~sj;
    const int v1 = ctz64(holes);
    holes &= holes - 1;
    const int v2 = ctz64(holes);
    const int u1 = ctz64(parts);
    parts &= parts - 1;
    const int u2 = ctz64(parts);
    const double sg = sign_double(sj, v1, u1, v2, u2);
    const double x = w * sg;
    add64(&r2[r2idx(n, u1, v1, u2, v2)], x);
    add64(&r2[r2idx(n, u1, v2, u2, v1)], -x);
    if (!HALF) {
        add64(&r2[r2idx(n, u2, v2, u1, v1)], x);
        add64(&r2[r2idx(n, u2, v1, u1, v2)], -x);
    }
}

struct RdmVis {
    const double* ket;
    double bra_i;
    u64 ai, bi;
    int n;
    double* r1;
    double* r2;
    __device__ __forceinline__ void operator()(bool ok, u32 j, u64 aj, u64 bj) {
        if (!ok) return;
        const double w = bra_i * ket[j];
        if (w == 0.0) return;
        pair_contrib<true>(n, w, ai, bi, aj, bj, r1, r2);
    }
};

__global__ void __launch_bounds__(ROW_BLOCK) rdm_offdiag_kernel(SpaceView S,
                                                                const double* __restrict__ bra,
                                                                const double* __restrict__ ket,
                                                                double* __restrict__ r1,
                                                                double* __restrict__ r2) {
    const i64 i = (i64)blockIdx.x * ROWS_PER_BLOCK + threadIdx.x / HCI_WAVE;
    if (i >= S.N) return;
    const double bi_ = bra[i];
    if (bi_ == 0.0) return;  // wave-uniform
    RdmVis v{ket, bi_, S.alpha[i], S.beta[i], S.n, r1, r2};
    enumerate_row(S, (u32)i, v);
}

// Occupation correlation D[x][y] = sum_i w_i n_x(i) n_y(i) over spin
// orbitals x, y in [0, 2n) (alpha first), w_i = bra_i ket_i; one partial
// matrix per block, threads own entries, determinants staged through LDS.
constexpr int OCC_PER_THREAD = 8;
constexpr int OCC_TILE = 256 * OCC_PER_THREAD;

__global__ void __launch_bounds__(256) occ_corr_kernel(const u64* __restrict__ alpha,
                                                       const u64* __restrict__ beta,
                                                       const double* __restrict__ bra,
                                                       const double* __restrict__ ket, i64 N,
                                                       int n, i64 chunk, double* __restrict__ part) {
    __shared__ u64 sa[OCC_CHUNK], sb[OCC_CHUNK];
    __shared__ double sw[OCC_CHUNK];
    const int m = 2 * n;
    const int entries = m * m;
    const int tile0 = blockIdx.y * OCC_TILE;
    const i64 begin = (i64)blockIdx.x * chunk, end = min(begin + chunk, N);
    double acc[OCC_PER_THREAD];
#pragma unroll
    for (int e = 0; e < OCC_PER_THREAD; ++e) acc[e] = 0.0;
    for (i64 base = begin; base < end; base += OCC_CHUNK) {
        const i64 t = base + threadIdx.x;
        if (threadIdx.x < OCC_CHUNK) {
            if (t < end) {
                sa[threadIdx.x] = alpha[t];
                sb[threadIdx.x] = beta[t];
                sw[threadIdx.x] = bra[t] * ket[t];
            } else {
                sa[threadIdx.x] = 0;
                sb[threadIdx.x] = 0;
                sw[threadIdx.x] = 0.0;
            }
        }
        __syncthreads();
        const int cnt = (int)min((i64)OCC_CHUNK, end - base);
#pragma unroll
        for (int e = 0; e < OCC_PER_THREAD; ++e) {
            const int idx = tile0 + threadIdx.x + e * 256;
            if (idx < entries) {
                const int x = idx / m, y = idx % m;
                const bool xa = x < n, ya = y < n;
                const int bx = xa ? x : x - n, by = ya ? y : y - n;
                double s = 0.0;
                for (int k = 0; k < cnt; ++k) {
                    const u64 wx = xa ? sa[k] : sb[k];
                    const u64 wy = ya ? sa[k] : sb[k];
                    if (test_bit(wx, bx) && test_bit(wy, by)) s += sw[k];
                }
                acc[e] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < OCC_PER_THREAD; ++e) {
        const int idx = tile0 + threadIdx.x + e * 256;
        if (idx < entries) part[(i64)blockIdx.x * entries + idx] = acc[e];
    }
}

__global__ void occ_reduce_kernel(const double* __restrict__ part, int nblk, int entries,
                                  double* __restrict__ D) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= entries) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(i64)b * entries + idx];
    D[idx] = s;
}

// Add the diagonal-pair terms from D: rdm1[p][p] += D[pa][pa] + D[pb][pb];
// rdm2[p][p][r][r] += sum over spin pairs of D[x][y] (x != y);
// rdm2[p][r][r][p] -= same-spin D[x][y] (p != r).
__global__ void diag_terms_kernel(const double* __restrict__ D, int n, double* __restrict__ r1,
                                  double* __restrict__ r2) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    const int p = idx / n, r = idx % n;
    const int m = 2 * n;
    const double daa = D[p * m + r], dbb = D[(p + n) * m + (r + n)];
    const double dab = D[p * m + (r + n)], dba = D[(p + n) * m + r];
    if (p == r) r1[(i64)p * n + p] += daa + dbb;
    if (!r2) return;
    if (p == r) {
        r2[r2idx(n, p, p, p, p)] += dab + dba;
    } else {
        r2[r2idx(n, p, p, r, r)] += daa + dbb + dab + dba;
        r2[r2idx(n, p, r, r, p)] -= daa + dbb;
    }
}

// Gamma^{dc}: one thread per screened pair (i, a), weight d_a c_i, bra D_a,
// ket D_i (Sec. "Computational Details": the connection list of the PT2).
__global__ void pt2_pairs_kernel(const u64* __restrict__ a_hi, const u64* __restrict__ a_lo,
                                 const u32* __restrict__ idx, const double* __restrict__ dpair,
                                 const u64* __restrict__ dets, const double* __restrict__ c, i64 M,
                                 int n, double* __restrict__ r1, double* __restrict__ r2) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    const u32 i = idx[t];
    const double w = dpair[t] * c[i];
    if (w == 0.0) return;
    pair_contrib<false>(n, w, a_hi[t], a_lo[t], dets[2 * (i64)i], dets[2 * (i64)i + 1], r1, r2);
}

// rdm2 = T + T^swap in place, T^swap[p][q][r][s] = T[r][s][p][q].
__global__ void swap_sym_kernel(double* __restrict__ r2, int n) {
    const i64 n2 = (i64)n * n;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n2 * n2) return;
    const i64 P = t / n2, R = t % n2;
    if (R < P) return;
    if (R == P) {
        r2[P * n2 + P] *= 2.0;
        return;
    }
    const double v = r2[P * n2 + R] + r2[R * n2 + P];
    r2[P * n2 + R] = v;
    r2[R * n2 + P] = v;
}

// ---------------------------------------------------------------- bucket kernel
// One workgroup owns up to RDM_CHUNK rows of one alpha bucket A (all rows
// share the alpha string).  Every contribution whose orbital indices are fixed
// by A up to a small set goes to a workgroup-private float64 accumulator in
// LDS and reaches global memory once per workgroup:
//   alpha single x beta single: per alpha neighbour t of A, [t][u2][v2]
//     (processed G neighbours at a time);
//   alpha single (same beta): per neighbour, the sum and its beta-occupation
//     moments (opposite-spin spectators);
//   beta single (same alpha): [u][v] and, when it fits, [u][v][k] for the
//     same-spin spectators k;
//   alpha double (same beta): one slot per (occupied pair, empty pair) of A.
// Beta doubles (same alpha) go to global memory directly.  All rdm2 terms are
// the canonical half T (see single_contrib).
constexpr int RDM_BLOCK = 1024;
constexpr int RDM_WAVES = RDM_BLOCK / HCI_WAVE;
constexpr u32 RDM_CHUNK = 1024;

struct RdmPlan {
    int n, G;
    int npo, npv;                // occupied / empty orbital pairs of an alpha string
    int o_p11, o_s1a, o_s1b2, o_s1b3, o_d2a, total;  // offsets in doubles
    bool b3, d2;
    int W;        // beta-string bitmap words per neighbour (0: search the buckets)
    int o_bm;     // byte offset of the bitmaps (after the doubles)
    int bytes;    // LDS of the workgroup
};

__device__ __forceinline__ void lds_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// index of the unordered pair x < y
__device__ __forceinline__ int pair_index(int x, int y) { return y * (y - 1) / 2 + x; }

// position of the k-th set bit (k from 0) of s
__device__ __forceinline__ int select_bit(u64 s, int k) {
    for (int t = 0; t < k; ++t) s &= s - 1;
    return ctz64(s);
}

// 8 waves per SIMD: two workgroups share a CU (the kernel is latency bound).
// BM: alpha single x beta single pairs through the LDS beta-string maps of
// build_beta_maps; otherwise by scanning or searching each neighbour bucket.
template <bool BM>
__global__ void __launch_bounds__(RDM_BLOCK) __attribute__((amdgpu_waves_per_eu(8, 8))) rdm_bucket_kernel(SpaceView S, RdmPlan P, i64 nua,
                                                               const u32* __restrict__ cptr,
                                                               const double* __restrict__ bra,
                                                               const double* __restrict__ ket,
                                                               double* __restrict__ r1,
                                                               double* __restrict__ r2) {
    extern __shared__ double lds[];
    __shared__ u32 sh[3];
    const u32 tid = threadIdx.x;
    const int lane = lane_id();
    const u32 wave = tid / HCI_WAVE;
    const int n = P.n;
    const int nn = n * n;
    if (tid == 0) {
        // bucket of this workgroup: the last a with cptr[a] <= blockIdx.x
        const u32 w = blockIdx.x;
        u32 lo = 0, hi = (u32)nua - 1u;
        while (lo < hi) {
            const u32 mid = (lo + hi + 1u) >> 1;
            if (cptr[mid] <= w) lo = mid;
            else hi = mid - 1u;
        }
        const u32 r0 = S.aoff[lo] + (w - cptr[lo]) * RDM_CHUNK;
        sh[0] = lo;
        sh[1] = r0;
        sh[2] = min(r0 + RDM_CHUNK, S.aoff[lo + 1]);
    }
    for (int x = (int)tid; x < P.total; x += RDM_BLOCK) lds[x] = 0.0;
    __syncthreads();
    const u32 a = sh[0], row0 = sh[1], row1 = sh[2];
    const u64 A = S.ua[a];
    const u64 full = low_mask(n);
    const u64 E = ~A & full;  // empty alpha orbitals
    const u32 t0 = S.as_ptr[a];
    const u32 deg = S.as_ptr[a + 1] - t0;
    const int nocc = popc64(A), nvir = n - nocc;
    double* p11 = lds + P.o_p11;
    double* s1a = lds + P.o_s1a;
    double* s1b2 = lds + P.o_s1b2;
    double* s1b3 = lds + P.o_s1b3;
    double* d2a = lds + P.o_d2a;
    u32* bm = reinterpret_cast<u32*>(reinterpret_cast<unsigned char*>(lds) + P.o_bm);
    u16* pre = reinterpret_cast<u16*>(bm + (i64)P.G * P.W);
    const u32 ngroups = deg == 0 ? 1u : (deg + (u32)P.G - 1u) / (u32)P.G;
    for (u32 g = 0; g < ngroups; ++g) {
        const u32 tg0 = g * (u32)P.G;
        const u32 tg1 = min(tg0 + (u32)P.G, deg);
        if constexpr (BM) build_beta_maps<RDM_BLOCK>(S, t0, tg0, tg1, (u32)P.W, bm, pre, tid);
        for (u32 row = row0 + wave; row < row1; row += RDM_WAVES) {
            const double wb = bra[row];
            if (wb == 0.0) continue;  // wave-uniform
            const u64 B = S.beta[row];
            const u32 b = S.ib[row];
            if (g == 0) {
                {  // same alpha: beta single (LDS) or beta double (global)
                    const u32 lo = S.aoff[a], hi = S.aoff[a + 1];
                    for (u32 base = lo; base < hi; base += HCI_WAVE) {
                        const u32 j = base + lane;
                        if (j >= hi || j == row) continue;
                        const u64 bj = S.beta[j];
                        const u64 xb = B ^ bj;
                        const int d = popc64(xb);
                        if (d == 2) {
                            const int v = ctz64(bj & xb), u = ctz64(B & xb);
                            const double x = wb * ket[j] * sign_between(bj, v, u);
                            lds_add(&s1b2[u * n + v], x);
                            for (u64 m = B & bj; m; m &= m - 1) {  // same-spin spectators
                                const int k = ctz64(m);
                                if (P.b3) {
                                    lds_add(&s1b3[(u * n + v) * n + k], x);
                                } else {
                                    add64(&r2[r2idx(n, u, v, k, k)], x);
                                    add64(&r2[r2idx(n, u, k, k, v)], -x);
                                }
                            }
                        } else if (d == 4) {
                            u64 holes = bj & xb, parts = B & xb;
                            const int v1 = ctz64(holes);
                            holes &= holes - 1;
                            const int v2 = ctz64(holes);
                            const int u1 = ctz64(parts);
                            parts &= parts - 1;
                            const int u2 = ctz64(parts);
                            const double x = wb * ket[j] * sign_double(bj, v1, u1, v2, u2);
                            add64(&r2[r2idx(n, u1, v1, u2, v2)], x);
                            add64(&r2[r2idx(n, u1, v2, u2, v1)], -x);
                        }
                    }
                }
                {  // same beta: alpha single (LDS per neighbour) or alpha double
                    const u32 lo = S.boff[b], hi = S.boff[b + 1];
                    for (u32 base = lo; base < hi; base += HCI_WAVE) {
                        const u32 k = base + lane;
                        if (k >= hi) continue;
                        const u32 j = S.permb[k];
                        if (j == row) continue;
                        const u64 aj = S.alpha[j];
                        const u64 xa = A ^ aj;
                        const int d = popc64(xa);
                        if (d == 2) {
                            const int v = ctz64(aj & xa), u = ctz64(A & xa);
                            const double x = wb * ket[j] * sign_between(aj, v, u);
                            double* slot = s1a + (i64)(rank_below(A, u) * nvir + rank_below(E, v)) * (1 + n);
                            lds_add(&slot[0], x);
                            for (u64 m = B; m; m &= m - 1) lds_add(&slot[1 + ctz64(m)], x);
                        } else if (d == 4) {
                            u64 holes = aj & xa, parts = A & xa;
                            const int v1 = ctz64(holes);
                            holes &= holes - 1;
                            const int v2 = ctz64(holes);
                            const int u1 = ctz64(parts);
                            parts &= parts - 1;
                            const int u2 = ctz64(parts);
                            const double x = wb * ket[j] * sign_double(aj, v1, u1, v2, u2);
                            if (P.d2) {
                                const int po = pair_index(rank_below(A, u1), rank_below(A, u2));
                                const int pv = pair_index(rank_below(E, v1), rank_below(E, v2));
                                lds_add(&d2a[po * P.npv + pv], x);
                            } else {
                                add64(&r2[r2idx(n, u1, v1, u2, v2)], x);
                                add64(&r2[r2idx(n, u1, v2, u2, v1)], -x);
                            }
                        }
                    }
                }
            }
            // alpha single x beta single for neighbours [tg0, tg1)
            const u32 s0 = S.bs_ptr[b], s1 = S.bs_ptr[b + 1];
            const u32 nbs = s1 - s0;
            if constexpr (BM) {
                for (u32 base = s0; base < s1; base += HCI_WAVE) {
                    const u32 k = base + lane;
                    if (k >= s1) continue;
                    const u32 bp = S.bs_idx[k];
                    const u64 bj = S.ub[bp];
                    const u64 xb = B ^ bj;
                    const int v2 = ctz64(bj & xb), u2 = ctz64(B & xb);
                    const double wsb = wb * sign_between(bj, v2, u2);
                    const u32 w = bp >> 5, bit = bp & 31u;
                    for (u32 t = tg0; t < tg1; ++t) {
                        const u32 q = t - tg0;
                        const u32 word = bm[q * (u32)P.W + w];
                        if (((word >> bit) & 1u) == 0u) continue;
                        const u32 a2 = S.as_idx[t0 + t];
                        const u64 A2 = S.ua[a2];
                        const u64 xa = A ^ A2;
                        const double sa = sign_between(A2, ctz64(A2 & xa), ctz64(A & xa));
                        const u32 j = S.aoff[a2] + (u32)pre[q * (u32)P.W + w] +
                                      (u32)__popc(word & ((1u << bit) - 1u));
                        lds_add(&p11[(i64)q * nn + u2 * n + v2], wsb * ket[j] * sa);
                    }
                }
            }
            for (u32 t = tg0; t < (BM ? tg0 : tg1); ++t) {
                const u32 a2 = S.as_idx[t0 + t];
                const u64 A2 = S.ua[a2];
                const u64 xa = A ^ A2;
                const int v1 = ctz64(A2 & xa), u1 = ctz64(A & xa);
                const double sa = sign_between(A2, v1, u1);
                double* slot = p11 + (i64)(t - tg0) * nn;
                const u32 lo = S.aoff[a2], hi = S.aoff[a2 + 1];
                const u32 len = hi - lo;
                if (len <= 4u * nbs) {
                    for (u32 base = lo; base < hi; base += HCI_WAVE) {
                        const u32 j = base + lane;
                        if (j >= hi) continue;
                        const u64 bj = S.beta[j];
                        const u64 xb = B ^ bj;
                        if (popc64(xb) != 2) continue;
                        const int v2 = ctz64(bj & xb), u2 = ctz64(B & xb);
                        lds_add(&slot[u2 * n + v2], wb * ket[j] * sa * sign_between(bj, v2, u2));
                    }
                } else {
                    for (u32 base = s0; base < s1; base += HCI_WAVE) {
                        const u32 k = base + lane;
                        if (k >= s1) continue;
                        const u64 bj = S.ub[S.bs_idx[k]];
                        const u32 pos = lower_bound_u64(S.beta + lo, len, bj);
                        if (pos >= len || S.beta[lo + pos] != bj) continue;
                        const u32 j = lo + pos;
                        const u64 xb = B ^ bj;
                        const int v2 = ctz64(bj & xb), u2 = ctz64(B & xb);
                        lds_add(&slot[u2 * n + v2], wb * ket[j] * sa * sign_between(bj, v2, u2));
                    }
                }
            }
        }
        __syncthreads();
        // flush this group's alpha single x beta single slots
        for (int x = (int)tid; x < (int)(tg1 - tg0) * nn; x += RDM_BLOCK) {
            const double val = p11[x];
            if (val == 0.0) continue;
            p11[x] = 0.0;
            const u32 t = tg0 + (u32)(x / nn);
            const int u2 = (x % nn) / n, v2 = x % n;
            const u64 A2 = S.ua[S.as_idx[t0 + t]];
            const u64 xa = A ^ A2;
            add64(&r2[r2idx(n, ctz64(A & xa), ctz64(A2 & xa), u2, v2)], val);
        }
        __syncthreads();
    }
    // alpha singles (slot of the occupied orbital u and the empty orbital v of
    // A): r1 and same-spin spectators from the sum, opposite-spin spectators
    // from the beta-occupation moments
    for (int q = (int)tid; q < nocc * nvir; q += RDM_BLOCK) {
        const int u = select_bit(A, q / nvir), v = select_bit(E, q % nvir);
        const double* slot = s1a + (i64)q * (1 + n);
        const double X = slot[0];
        if (X != 0.0) {
            add64(&r1[u * n + v], X);
            for (u64 m = A; m; m &= m - 1) {
                const int k = ctz64(m);
                if (k == u) continue;
                add64(&r2[r2idx(n, u, v, k, k)], X);
                add64(&r2[r2idx(n, u, k, k, v)], -X);
            }
        }
        for (int k = 0; k < n; ++k) {
            const double Y = slot[1 + k];
            if (Y != 0.0) add64(&r2[r2idx(n, u, v, k, k)], Y);
        }
    }
    // beta singles: r1 and the alpha spectators from the sum
    for (int x = (int)tid; x < nn; x += RDM_BLOCK) {
        const double X = s1b2[x];
        if (X == 0.0) continue;
        const int u = x / n, v = x % n;
        add64(&r1[x], X);
        for (u64 m = A; m; m &= m - 1) add64(&r2[r2idx(n, u, v, ctz64(m), ctz64(m))], X);
    }
    if (P.b3) {
        for (int x = (int)tid; x < nn * n; x += RDM_BLOCK) {
            const double X = s1b3[x];
            if (X == 0.0) continue;
            const int u = x / nn, v = (x / n) % n, k = x % n;
            add64(&r2[r2idx(n, u, v, k, k)], X);
            add64(&r2[r2idx(n, u, k, k, v)], -X);
        }
    }
    if (P.d2) {
        for (int x = (int)tid; x < P.npo * P.npv; x += RDM_BLOCK) {
            const double X = d2a[x];
            if (X == 0.0) continue;
            const int po = x / P.npv, pv = x % P.npv;
            int y = 1;
            while ((y + 1) * y / 2 <= po) ++y;
            const int ru2 = y, ru1 = po - y * (y - 1) / 2;
            y = 1;
            while ((y + 1) * y / 2 <= pv) ++y;
            const int rv2 = y, rv1 = pv - y * (y - 1) / 2;
            const int u1 = select_bit(A, ru1), u2 = select_bit(A, ru2);
            const int v1 = select_bit(E, rv1), v2 = select_bit(E, rv2);
            add64(&r2[r2idx(n, u1, v1, u2, v2)], X);
            add64(&r2[r2idx(n, u1, v2, u2, v1)], -X);
        }
    }
}

__global__ void rdm_nchunk_kernel(const u32* __restrict__ aoff, i64 nua, u32* __restrict__ out) {
    const i64 a = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < nua) out[a] = (aoff[a + 1] - aoff[a] + RDM_CHUNK - 1) / RDM_CHUNK;
    if (a == nua) out[a] = 0;
}

// LDS layout of the bucket kernel for this context, within `budget` bytes,
// with W bitmap words per neighbour (0: no bitmaps); false when even one
// alpha neighbour per pass does not fit.
bool rdm_plan(int n, int na, int budget, int W, RdmPlan& P) {
    const int dmax = na * (n - na);
    const int nn = n * n;
    P.n = n;
    P.npo = na * (na - 1) / 2;
    P.npv = (n - na) * (n - na - 1) / 2;
    for (int variant = 0; variant < 3; ++variant) {
        P.b3 = variant == 0;
        P.d2 = variant <= 1;
        const int s1a = dmax * (1 + n);
        const int s1b3 = P.b3 ? nn * n : 0;
        const int d2 = P.d2 ? P.npo * P.npv : 0;
        const int rest = s1a + nn + s1b3 + d2;
        int G = (budget - 8 * rest) / (8 * nn + 6 * W);
        if (G < 1) continue;
        if (G > dmax) G = dmax > 0 ? dmax : 1;
        P.G = G;
        P.o_p11 = 0;
        P.o_s1a = G * nn;
        P.o_s1b2 = P.o_s1a + s1a;
        P.o_s1b3 = P.o_s1b2 + nn;
        P.o_d2a = P.o_s1b3 + s1b3;
        P.total = P.o_d2a + d2;
        P.W = W;
        P.o_bm = 8 * P.total;
        P.bytes = P.o_bm + ((6 * G * W + 15) & ~15);
        return true;
    }
    return false;
}

}  // namespace

// Diagonal-pair terms of sum_k wa_k wb_k <D_k| ops |D_k> added to rdm1/rdm2.
void rdm_add_diag(hci_ctx_s* ctx, const u64* alpha, const u64* beta, const double* wa,
                  const double* wb, i64 M, double* rdm1, double* rdm2, hipStream_t s) {
    if (M <= 0) return;
    const int n = ctx->n;
    const i64 n2 = (i64)n * n;
    const int entries = 4 * n * n;
    const i64 chunk = std::max<i64>(OCC_CHUNK, ceil_div(M, 512));
    const int nblk = (int)ceil_div(M, chunk);
    DevMem part = dev_alloc(ctx, sizeof(double) * (i64)nblk * entries, s);
    DevMem D = dev_alloc(ctx, sizeof(double) * entries, s);
    HCI_LAUNCH(ctx, "rdm_occ", s, occ_corr_kernel, dim3(nblk, (unsigned)ceil_div(entries, OCC_TILE)),
               256, 0, alpha, beta, wa, wb, M, n, chunk, part.as<double>());
    HCI_LAUNCH(ctx, "rdm_occ_reduce", s, occ_reduce_kernel, ceil_div(entries, 256), 256, 0,
               part.as<double>(), nblk, entries, D.as<double>());
    HCI_LAUNCH(ctx, "rdm_diag_terms", s, diag_terms_kernel, ceil_div(n2, 256), 256, 0,
               D.as<double>(), n, rdm1, rdm2);
}

void rdm_compute(hci_ctx_s* ctx, Space* sp, const double* bra, const double* ket, double* rdm1,
                 double* rdm2, hipStream_t s) {
    const int n = ctx->n;
    const i64 N = sp->N;
    const i64 n2 = (i64)n * n;
    HIP_CHECK(hipMemsetAsync(rdm1, 0, sizeof(double) * n2, s));
    if (rdm2) HIP_CHECK(hipMemsetAsync(rdm2, 0, sizeof(double) * n2 * n2, s));
    SpaceView S = space_view(*sp, n);
    // two workgroups per CU: up to 79 KB of LDS each
    int dev = 0, max_shared = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&max_shared, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int budget = std::min(79 * 1024, max_shared);
    const char* force_search = std::getenv("HCI_AB_SEARCH");  // "1": always search (tests)
    const int W = sp->nub <= 65535 && !(force_search && force_search[0] == '1') ? (int)ceil_div(sp->nub, 32) : 0;
    RdmPlan P;
    bool planned = false;
    if (rdm2) planned = (W > 0 && rdm_plan(n, ctx->na, budget, W, P)) || rdm_plan(n, ctx->na, budget, 0, P);
    if (planned) {
        if (!sp->rdm_cptr.ptr) {
            DevMem cnt = dev_alloc(ctx, sizeof(u32) * (sp->nua + 1), s);
            HCI_LAUNCH(ctx, "rdm_nchunk", s, rdm_nchunk_kernel, ceil_div(sp->nua + 1, 256), 256, 0,
                       sp->aoff.as<u32>(), sp->nua, cnt.as<u32>());
            sp->rdm_cptr = dev_alloc(ctx, sizeof(u32) * (sp->nua + 1), s);
            scan_u32_to_u32(ctx, cnt.as<u32>(), sp->rdm_cptr.as<u32>(), sp->nua + 1, s);
            sp->rdm_nchunk = read_scalar(sp->rdm_cptr.as<u32>() + sp->nua, s);
        }
        auto kern = P.W ? rdm_bucket_kernel<true> : rdm_bucket_kernel<false>;
        HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, P.bytes));
        HCI_LAUNCH(ctx, "rdm_offdiag", s, kern, sp->rdm_nchunk, RDM_BLOCK, (size_t)P.bytes, S, P, sp->nua,
                   sp->rdm_cptr.as<u32>(), bra, ket, rdm1, rdm2);
    } else {
        HCI_LAUNCH(ctx, "rdm_offdiag", s, rdm_offdiag_kernel, ceil_div(N, ROWS_PER_BLOCK), ROW_BLOCK,
                   0, S, bra, ket, rdm1, rdm2);
    }
    // the off-diagonal passes accumulate one entry of each (pq|rs), (rs|pq) pair
    if (rdm2) {
        HCI_LAUNCH(ctx, "rdm_swap_sym", s, swap_sym_kernel, ceil_div(n2 * n2, 256), 256, 0, rdm2, n);
    }
    rdm_add_diag(ctx, sp->alpha.as<u64>(), sp->beta.as<u64>(), bra, ket, N, rdm1, rdm2, s);
}

void rdm_add_pairs(hci_ctx_s* ctx, const u64* a_hi, const u64* a_lo, const u32* idx, const double* wa, i64 M,
                   const u64* dets, const double* c, double* rdm1, double* rdm2, hipStream_t s) {
    if (M <= 0) return;
    HCI_LAUNCH(ctx, "rdm_pt2_pairs", s, pt2_pairs_kernel, ceil_div(M, 256), 256, 0, a_hi, a_lo, idx, wa, dets,
               c, M, ctx->n, rdm1, rdm2);
}
