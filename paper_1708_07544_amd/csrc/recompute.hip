// sigma = H c without a stored Hamiltonian (the product inside the Davidson
// solver, Sec. "Variational Stage", over every single and double connection
// between members of V, Sec. "Computational Details"), for spaces whose
// Hamiltonian does not fit in memory.
//
// The connections of a row D_i = (A, B) fall in three classes, and each is
// found by comparing occupation words staged on chip rather than by reading
// candidates from global memory once per row:
//   * same alpha string (beta single or double): the rows of bucket A;
//   * alpha single x beta single: the rows of the buckets A' one alpha
//     single away (the alpha adjacency of the space), whose beta string is
//     one single from B;
//   * same beta string (alpha single or double): the rows of beta bucket B
//     (beta-major order).
// A workgroup owns a chunk of up to RC_ROWS consecutive rows of one bucket.
// The candidate columns of the chunk -- its own bucket, then (alpha-major)
// every bucket one alpha single away, concatenated -- are staged in LDS a
// tile at a time (occupation word, c_j, and the link each column came
// from), and each wavefront scans them for its rows with a popcount test.
// Hits are compacted into two queues per wavefront (singles; doubles and
// alpha x beta) and evaluated 64 at a time, so the element code runs with
// full wavefronts instead of the few lanes that hit in each 64-column step.
// An alpha-single link A -> A' fixes the orbital pair (p -> r) and its phase
// (kept per link in LDS), so its elements are sign * (rp|sq) with (s, q) from
// the beta strings.  Single excitations sum over the occupied orbitals; the
// part that depends on the chunk's fixed string is summed once per chunk.
//
// Every row is owned by one wavefront of one workgroup in each of the two
// kernels: the alpha-major kernel writes sigma_i = H_ii c_i + (its classes),
// the beta-major kernel then adds the same-beta class.  No atomics; the
// order of every sum is fixed by the data.
#include <cstdlib>

#include "slater.h"

namespace {

constexpr int RC_BLOCK = 512;
constexpr int RC_WAVES = RC_BLOCK / HCI_WAVE;
constexpr u32 RC_ROWS = 256;    // rows per chunk (workgroup)
constexpr u32 RC_TILE = 2048;   // candidate columns staged at a time
constexpr u32 RC_UNROLL = 4;    // 64-column steps whose loads are in flight together
constexpr u32 RC_OWN = 0xffffu; // column from the chunk's own bucket
constexpr u32 RC_BM_BYTES = 28 * 1024;  // bitmaps of a neighbour group (aliases the column tile)

// Neighbour lookup through LDS bitmaps of the beta strings present in each
// neighbour bucket (when the space has at most 65535 unique beta strings):
// W words per neighbour, G neighbours per group, nbs_avg the mean number of
// beta singles of a beta string (to choose between lookup and scan per chunk).
struct RcBitmaps {
    u32 W, G;
    float nbs_avg;
};

// Element arithmetic of one precision: float32 elements (rounded integrals,
// float32 sums) for the mixed product, float64 otherwise.
template <class VT>
struct RcInts {
    int n;
    const VT* h;   // [n][n]
    const VT* g;   // [n]^4
    const VT* jk;  // [n][n][n]: (qp|rr) - (qr|rp)
    const VT* jj;  // [n][n][n]: (qp|rr)
};

inline RcInts<float> rc_ints_f32(const IntView& I) { return {I.n, I.h32, I.g32, I.jk32, I.jj32}; }
inline RcInts<double> rc_ints_f64(const IntView& I) { return {I.n, I.h, I.g, I.jk, I.jj}; }

template <class VT>
struct RcLds {
    u64* colw;     // [RC_TILE] varying string of each staged column
    VT* colc;      // [RC_TILE] its coefficient
    u16* colk;     // [RC_TILE] its link (RC_OWN: the chunk's own bucket)
    u32* loff;     // [maxl + 1] first concatenated column of each link
    u32* lstart;   // [maxl] first row of each link's bucket
    u32* linfo;    // [maxl] p | r << 8 | (sign < 0) << 16 of each alpha-single link
    double* racc;  // [RC_ROWS]
    u16* queue;    // [RC_WAVES][3][128] singles / same-string doubles / alpha x beta queues
    VT* ftab;      // [n*n]
};

// maxl: links of a chunk at most (its own bucket + the largest alpha degree).
// colw, colc, colk are contiguous (the tile region, at least RC_BM_BYTES,
// which the neighbour bitmaps reuse).
template <class VT>
__device__ __forceinline__ RcLds<VT> rc_lds(char* smem, int n, u32 maxl) {
    RcLds<VT> L;
    L.colw = reinterpret_cast<u64*>(smem);
    L.colc = reinterpret_cast<VT*>(L.colw + RC_TILE);
    L.colk = reinterpret_cast<u16*>(L.colc + RC_TILE);
    L.ftab = reinterpret_cast<VT*>(L.colk + RC_TILE);
    L.loff = reinterpret_cast<u32*>(L.ftab + n * n);
    L.lstart = L.loff + maxl + 1;
    L.linfo = L.lstart + maxl;
    L.racc = reinterpret_cast<double*>(smem + ((reinterpret_cast<char*>(L.linfo + maxl) - smem + 7) & ~(size_t)7));
    L.queue = reinterpret_cast<u16*>(L.racc + RC_ROWS);
    return L;
}

template <class VT>
size_t rc_lds_bytes(int n, u32 maxl) {
    const size_t head = (sizeof(u64) + sizeof(VT) + sizeof(u16)) * RC_TILE + sizeof(VT) * (size_t)n * n +
                        sizeof(u32) * (3 * (size_t)maxl + 1);
    return ((head + 7) & ~(size_t)7) + sizeof(double) * RC_ROWS + sizeof(u16) * RC_WAVES * 384;
}
static_assert((sizeof(u64) + sizeof(float) + sizeof(u16)) * RC_TILE >= RC_BM_BYTES, "bitmaps fit the tile region");

// Ftab[q][p] = sum over the occupied orbitals r of the chunk's fixed string F of (qp|rr)
template <class VT>
__device__ __forceinline__ void rc_fixed_table(const RcInts<VT>& T, u64 F, VT* Ftab) {
    const int n = T.n;
    for (int e = (int)threadIdx.x; e < n * n; e += RC_BLOCK) {
        const int row = e * n;  // e = q * n + p
        VT v = (VT)0;
        for (u64 m = F; m; m &= m - 1) v += T.jj[row + ctz64(m)];
        Ftab[e] = v;
    }
}

// Single excitation within the varying strings: X (row) -> Y (column), the
// other spin's string fixed (Ftab); h_qp + sum_{r in X} [(qp|rr) - (qr|rp)]
// + sum_{r in F} (qp|rr) with the phase of X.
template <class VT>
__device__ __forceinline__ double rc_single(const RcInts<VT>& T, const VT* Ftab, u64 X, u64 Y) {
    const int n = T.n;
    const u64 x = X ^ Y;
    const int p = ctz64(X & x), q = ctz64(Y & x);
    const int row = (q * n + p) * n;  // n <= 64: every index below 2^31
    VT v = T.h[q * n + p];
    for (u64 m = X; m; m &= m - 1) v += T.jk[row + ctz64(m)];
    v += Ftab[q * n + p];
    return (double)((VT)sign_between(X, p, q) * v);
}

// Double excitation within the varying strings: (rp|sq) - (rq|sp) with the
// phase of X (holes p < q of X, particles r < s of Y).
template <class VT>
__device__ __forceinline__ double rc_double(const RcInts<VT>& T, u64 X, u64 Y) {
    const int n = T.n;
    const u64 x = X ^ Y;
    u64 holes = X & x, parts = x & ~X;
    const int p = ctz64(holes);
    holes &= holes - 1;
    const int q = ctz64(holes);
    const int r = ctz64(parts);
    parts &= parts - 1;
    const int s = ctz64(parts);
    const int rn = r * n;
    return (double)((VT)sign_double(X, p, r, q, s) *
                    (T.g[((rn + p) * n + s) * n + q] - T.g[((rn + q) * n + s) * n + p]));
}

// Alpha single (link: p -> r with its phase) times beta single X (row) ->
// Y (column): sign * (rp|sq) with q in X, s in Y.
template <class VT>
__device__ __forceinline__ double rc_cross(const RcInts<VT>& T, u32 info, u64 X, u64 Y) {
    const int n = T.n;
    const u64 x = X ^ Y;
    const int q = ctz64(X & x), s = ctz64(Y & x);
    const int p = (int)(info & 0xffu), r = (int)((info >> 8) & 0xffu);
    const VT sa = (info >> 16) ? (VT)-1 : (VT)1;
    return (double)((sa * (VT)sign_between(X, q, s)) * T.g[((r * n + p) * n + s) * n + q]);
}

// Stage columns [P0, P0 + tlen) of the chunk's concatenated links: link t
// holds rows [lstart[t], lstart[t] + loff[t+1] - loff[t]).  ALPHA_MAJOR:
// the varying string is beta, rows are determinant indices; else alpha, rows
// are beta-major positions.
template <class VT, bool ALPHA_MAJOR>
__device__ __forceinline__ void rc_stage(const SpaceView& S, const VT* __restrict__ cx, const RcLds<VT>& L,
                                         u32 nlinks, u32 P0, u32 tlen) {
    for (u32 k = threadIdx.x; k < tlen; k += RC_BLOCK) {
        const u32 P = P0 + k;
        u32 lo = 0, hi = nlinks - 1;  // last link with loff[t] <= P
        while (lo < hi) {
            const u32 mid = (lo + hi + 1) >> 1;
            if (L.loff[mid] <= P) lo = mid;
            else hi = mid - 1;
        }
        const u32 row = L.lstart[lo] + (P - L.loff[lo]);
        if (ALPHA_MAJOR) {
            L.colw[k] = S.beta[row];
            L.colc[k] = cx[row];
        } else {
            const u32 j = S.permb[row];
            L.colw[k] = S.alpha[j];
            L.colc[k] = cx[j];
        }
        L.colk[k] = lo == 0 ? (u16)RC_OWN : (u16)(lo - 1);
    }
}

// One row X against the staged tile: hits are compacted into the wavefront's
// two queues (singles; doubles and alpha x beta) and evaluated 64 at a time.
template <class VT>
__device__ __forceinline__ void rc_flush_d(const RcInts<VT>& T, const RcLds<VT>& L, const u16* qd, u32 cnt, u64 X,
                                           double& acc) {
    if ((u32)lane_id() < cnt) {
        const u32 kk = qd[lane_id()];
        acc += rc_double<VT>(T, X, L.colw[kk]) * (double)L.colc[kk];
    }
}

template <class VT>
__device__ __forceinline__ void rc_flush_x(const RcInts<VT>& T, const RcLds<VT>& L, const u16* qx, u32 cnt, u64 X,
                                           double& acc) {
    if ((u32)lane_id() < cnt) {
        const u32 kk = qx[lane_id()];
        acc += rc_cross<VT>(T, L.linfo[L.colk[kk]], X, L.colw[kk]) * (double)L.colc[kk];
    }
}

template <class VT>
__device__ __forceinline__ void rc_flush_s(const RcInts<VT>& T, const RcLds<VT>& L, const u16* qs, u32 cnt, u64 X,
                                           double& acc) {
    if ((u32)lane_id() < cnt) {
        const u32 kk = qs[lane_id()];
        acc += rc_single<VT>(T, L.ftab, X, L.colw[kk]) * (double)L.colc[kk];
    }
}

// drop the 64 evaluated entries of a queue holding cnt >= 64
__device__ __forceinline__ void rc_shift(u16* q, u32 cnt) {
    const u32 lane = (u32)lane_id();
    const u32 rest = cnt - HCI_WAVE;
    const u16 mv = lane < rest ? q[HCI_WAVE + lane] : (u16)0;
    __builtin_amdgcn_wave_barrier();
    if (lane < rest) q[lane] = mv;
    __builtin_amdgcn_wave_barrier();
}

// One row X against the staged tile (columns [0, own) are the chunk's own
// bucket): hits are compacted into the wavefront's three queues (singles,
// same-string doubles, alpha x beta) and evaluated 64 at a time.
template <class VT>
__device__ __forceinline__ double rc_row(const RcInts<VT>& T, const RcLds<VT>& L, u16* qs, u16* qd, u16* qx,
                                         u32 tlen, u32 own, u64 X) {
    const u32 lane = (u32)lane_id();
    double acc = 0.0;
    u32 ns = 0, nd = 0, nx = 0;  // queued (wave-uniform)
    for (u32 k0 = 0; k0 < tlen; k0 += RC_UNROLL * HCI_WAVE) {
        int d[RC_UNROLL];
#pragma unroll
        for (u32 u = 0; u < RC_UNROLL; ++u) {
            const u32 k = k0 + u * HCI_WAVE + lane;
            d[u] = k < tlen ? popc64(X ^ L.colw[k]) : 0;
        }
#pragma unroll
        for (u32 u = 0; u < RC_UNROLL; ++u) {
            const u32 kb = k0 + u * HCI_WAVE;  // wave-uniform
            const u32 k = kb + lane;
            // a step wholly past the chunk's own bucket can only hold alpha x
            // beta hits, one wholly inside it only singles and doubles
            const bool any_own = kb < own, all_own = kb + HCI_WAVE <= own;
            if (!all_own) {
                const bool crs = k >= own && d[u] == 2;
                const u64 mx = ballot(crs);
                if (crs) qx[nx + rank_in(mx)] = (u16)k;
                nx += (u32)popc64(mx);
            }
            if (any_own) {
                const bool in_own = k < own;
                const bool sgl = in_own && d[u] == 2;
                const bool dbl = in_own && d[u] == 4;
                const u64 ms = ballot(sgl), md = ballot(dbl);
                if (sgl) qs[ns + rank_in(ms)] = (u16)k;
                if (dbl) qd[nd + rank_in(md)] = (u16)k;
                ns += (u32)popc64(ms);
                nd += (u32)popc64(md);
            }
            __builtin_amdgcn_wave_barrier();
            if (nx >= HCI_WAVE) {
                rc_flush_x<VT>(T, L, qx, HCI_WAVE, X, acc);
                rc_shift(qx, nx);
                nx -= HCI_WAVE;
            }
            if (any_own) {
                if (nd >= HCI_WAVE) {
                    rc_flush_d<VT>(T, L, qd, HCI_WAVE, X, acc);
                    rc_shift(qd, nd);
                    nd -= HCI_WAVE;
                }
                if (ns >= HCI_WAVE) {
                    rc_flush_s<VT>(T, L, qs, HCI_WAVE, X, acc);
                    rc_shift(qs, ns);
                    ns -= HCI_WAVE;
                }
            }
        }
    }
    rc_flush_x<VT>(T, L, qx, nx, X, acc);
    rc_flush_d<VT>(T, L, qd, nd, X, acc);
    rc_flush_s<VT>(T, L, qs, ns, X, acc);
    __builtin_amdgcn_wave_barrier();
    return wave_sum_f64(acc);
}

// Alpha single x beta single connections of rows [r0, r1) of bucket A by
// lookup: for a group of neighbours A' (links 1.. of the chunk), LDS bitmaps
// of the beta strings present in each bucket A' (build_beta_maps); each row
// probes its beta singles (the beta adjacency) in every bitmap of the group.
// Hits are queued as (neighbour, single) and evaluated 64 at a time; c_j is
// read from global memory at its position in bucket A'.  The bitmaps alias
// the column tile.  Adds to racc; ends with a barrier.
template <class VT>
__device__ __forceinline__ void rc_cross_lookup(const SpaceView& S, const RcInts<VT>& T, const VT* __restrict__ cx,
                                                const RcLds<VT>& L, u32 t_beg, u32 deg, u32 r0, u32 r1,
                                                RcBitmaps M, u16* qx) {
    const u32 tid = threadIdx.x;
    const u32 wave = tid / HCI_WAVE;
    const u32 lane = (u32)lane_id();
    u32* bm = reinterpret_cast<u32*>(L.colw);
    u16* pre = reinterpret_cast<u16*>(bm + (size_t)M.G * M.W);
    for (u32 g0 = 0; g0 < deg; g0 += M.G) {
        const u32 g1 = min(g0 + M.G, deg);
        const u32 ng = g1 - g0;
        build_beta_maps<RC_BLOCK>(S, t_beg, g0, g1, M.W, bm, pre, tid);
        for (u32 r = r0 + wave; r < r1; r += RC_WAVES) {
            const u64 X = S.beta[r];
            const u32 bs = S.ib[r];
            const u32 s0 = S.bs_ptr[bs], s1 = S.bs_ptr[bs + 1];
            double acc = 0.0;
            u32 nx = 0;
            auto flush = [&](u32 cnt) {
                if (lane < cnt) {
                    const u32 e = qx[lane];
                    const u32 q = e >> 10, kk = e & 1023u;
                    const u32 bp = S.bs_idx[s0 + kk];
                    const u32 w = bp >> 5, bt = bp & 31u;
                    const u32 word = bm[q * M.W + w];
                    const u32 j = L.lstart[1 + g0 + q] + (u32)pre[q * M.W + w] +
                                  (u32)__builtin_popcount(word & ((1u << bt) - 1u));
                    acc += rc_cross<VT>(T, L.linfo[g0 + q], X, S.ub[bp]) * (double)cx[j];
                }
            };
            for (u32 k0 = s0; k0 < s1; k0 += HCI_WAVE) {
                const u32 k = k0 + lane;
                const bool valid = k < s1;
                const u32 bp = valid ? S.bs_idx[k] : 0u;
                const u32 w = bp >> 5, bt = bp & 31u;
                for (u32 q = 0; q < ng; ++q) {
                    const bool hit = valid && ((bm[q * M.W + w] >> bt) & 1u);
                    const u64 m = ballot(hit);
                    if (hit) qx[nx + rank_in(m)] = (u16)((q << 10) | (k - s0));
                    nx += (u32)popc64(m);
                    __builtin_amdgcn_wave_barrier();
                    if (nx >= HCI_WAVE) {
                        flush(HCI_WAVE);
                        rc_shift(qx, nx);
                        nx -= HCI_WAVE;
                    }
                }
            }
            flush(nx);
            __builtin_amdgcn_wave_barrier();
            acc = wave_sum_f64(acc);
            if (lane == 0) L.racc[r - r0] += acc;
        }
        __syncthreads();  // the bitmaps are rebuilt for the next group
    }
}

// One chunk: rows [r0, r1) of bucket `b` (alpha-major: determinant indices of
// alpha bucket b; beta-major: positions of beta bucket b).  Link 0 is the
// bucket itself; alpha-major chunks add the buckets one alpha single away.
// Returns with racc[0, r1 - r0) holding the rows' sums (last barrier done).
template <class VT, bool ALPHA_MAJOR>
__device__ __forceinline__ void rc_chunk(const SpaceView& S, const RcInts<VT>& T, const VT* __restrict__ cx,
                                         const RcLds<VT>& L, u32 b, u32 r0, u32 r1, RcBitmaps M) {
    const u32 tid = threadIdx.x;
    const u32 wave = tid / HCI_WAVE;
    const u32 lane = (u32)lane_id();
    const u32 nr = r1 - r0;
    const u64 F = ALPHA_MAJOR ? S.ua[b] : S.ub[b];
    const u32* off = ALPHA_MAJOR ? S.aoff : S.boff;
    const u32 t_beg = ALPHA_MAJOR ? S.as_ptr[b] : 0u;
    const u32 deg = ALPHA_MAJOR ? S.as_ptr[b + 1] - t_beg : 0u;
    const u32 nlinks = 1 + deg;
    for (u32 x = tid; x < nr; x += RC_BLOCK) L.racc[x] = 0.0;
    rc_fixed_table<VT>(T, F, L.ftab);
    // link table: own bucket, then the alpha neighbours in adjacency order
    // neighbour buckets by lookup when scanning them would cost more than
    // probing every row's beta singles in them (uniform decision)
    bool lookup = false;
    if (ALPHA_MAJOR && M.W > 0 && deg > 0) {
        const u32 own_len = off[b + 1] - off[b];
        (void)own_len;
        lookup = true;  // refined below once the link lengths are known
    }
    if (wave == 0) {
        u32 run = 0;
        for (u32 base = 0; base < nlinks; base += HCI_WAVE) {
            const u32 t = base + lane;
            u32 len = 0;
            if (t < nlinks) {
                u32 bb = b;
                if (t > 0) {
                    bb = S.as_idx[t_beg + t - 1];
                    const u64 x = F ^ S.ua[bb];
                    const int p = ctz64(F & x), r = ctz64(S.ua[bb] & x);
                    L.linfo[t - 1] = (u32)p | ((u32)r << 8) | ((count_between(F, p, r) & 1) ? (1u << 16) : 0u);
                }
                L.lstart[t] = off[bb];
                len = off[bb + 1] - off[bb];
            }
            u32 incl = len;
#pragma unroll
            for (int o = 1; o < HCI_WAVE; o <<= 1) {
                const u32 y = (u32)__shfl_up((int)incl, o, HCI_WAVE);
                if ((int)lane >= o) incl += y;
            }
            if (t < nlinks) L.loff[t] = run + incl - len;
            run += (u32)__shfl((int)incl, HCI_WAVE - 1, HCI_WAVE);
        }
        if (lane == 0) L.loff[nlinks] = run;
    }
    __syncthreads();
    u32 total = L.loff[nlinks];
    if (lookup) {
        const u32 scan_cols = total - L.loff[1];
        lookup = (float)scan_cols > 2.0f * (float)deg * M.nbs_avg;
        if (lookup) total = L.loff[1];  // scan only the own bucket
    }
    u16* qs = L.queue + wave * 384;
    u16* qd = qs + 128;
    u16* qx = qd + 128;
    if (lookup) rc_cross_lookup<VT>(S, T, cx, L, t_beg, deg, r0, r1, M, qx);
    for (u32 P0 = 0; P0 < total; P0 += RC_TILE) {
        const u32 tlen = min(RC_TILE, total - P0);
        rc_stage<VT, ALPHA_MAJOR>(S, cx, L, nlinks, P0, tlen);
        __syncthreads();
        const u32 own = L.loff[1] > P0 ? min(L.loff[1] - P0, tlen) : 0u;  // own-bucket columns of this tile
        for (u32 r = r0 + wave; r < r1; r += RC_WAVES) {
            const u64 X = ALPHA_MAJOR ? S.beta[r] : S.alpha[S.permb[r]];
            const double v = rc_row<VT>(T, L, qs, qd, qx, tlen, own, X);
            if (lane == 0) L.racc[r - r0] += v;
        }
        __syncthreads();
    }
}

// Alpha-major kernel: same-alpha and alpha single x beta single classes, the
// diagonal, and the write of sigma.  chunks: [nch][3] = bucket, first row,
// end row.
template <class VT>
__global__ void __launch_bounds__(RC_BLOCK) rc_alpha_kernel(SpaceView S, RcInts<VT> T, const u32* __restrict__ chunks,
                                                            i64 nch, const VT* __restrict__ cx,
                                                            const double* __restrict__ c,
                                                            const double* __restrict__ hd,
                                                            double* __restrict__ sigma, u32 maxl, RcBitmaps M) {
    extern __shared__ __align__(16) char smem[];
    const RcLds<VT> L = rc_lds<VT>(smem, T.n, maxl);
    for (i64 ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const u32 a = chunks[3 * ch], r0 = chunks[3 * ch + 1], r1 = chunks[3 * ch + 2];
        rc_chunk<VT, true>(S, T, cx, L, a, r0, r1, M);
        for (u32 r = r0 + threadIdx.x; r < r1; r += RC_BLOCK) sigma[r] = hd[r] * c[r] + L.racc[r - r0];
        __syncthreads();
    }
}

// Beta-major kernel: same-beta class (alpha single or double), added to
// sigma.  chunks: [nch][3] = beta bucket, first position, end position in
// beta-major order (positions k, determinants permb[k]).
template <class VT>
__global__ void __launch_bounds__(RC_BLOCK) rc_beta_kernel(SpaceView S, RcInts<VT> T, const u32* __restrict__ chunks,
                                                           i64 nch, const VT* __restrict__ cx,
                                                           double* __restrict__ sigma) {
    extern __shared__ __align__(16) char smem[];
    const RcLds<VT> L = rc_lds<VT>(smem, T.n, 1);
    for (i64 ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const u32 b = chunks[3 * ch], k0 = chunks[3 * ch + 1], k1 = chunks[3 * ch + 2];
        if (S.boff[b + 1] - S.boff[b] < 2) continue;  // a lone determinant (uniform)
        rc_chunk<VT, false>(S, T, cx, L, b, k0, k1, RcBitmaps{0u, 0u, 0.0f});
        for (u32 k = k0 + threadIdx.x; k < k1; k += RC_BLOCK) sigma[S.permb[k]] += L.racc[k - k0];
        __syncthreads();
    }
}

// Chunks of up to RC_ROWS rows of each bucket: count, scan, fill.
__global__ void rc_count_kernel(const u32* __restrict__ off, i64 m, u32* __restrict__ cnt) {
    const i64 a = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < m) cnt[a] = (off[a + 1] - off[a] + RC_ROWS - 1) / RC_ROWS;
    if (a == m) cnt[a] = 0;
}

__global__ void rc_fill_kernel(const u32* __restrict__ off, i64 m, const u32* __restrict__ cptr,
                               u32* __restrict__ chunks) {
    const i64 a = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= m) return;
    const u32 lo = off[a], hi = off[a + 1];
    u32 k = cptr[a];
    for (u32 r = lo; r < hi; r += RC_ROWS, ++k) {
        chunks[3 * (i64)k] = (u32)a;
        chunks[3 * (i64)k + 1] = r;
        chunks[3 * (i64)k + 2] = min(r + RC_ROWS, hi);
    }
}

void rc_chunks(hci_ctx_s* ctx, const DevMem& off, i64 m, DevMem& chunks, i64& nch, hipStream_t s) {
    DevMem cnt = dev_alloc(ctx, sizeof(u32) * (m + 1), s);
    DevMem cptr = dev_alloc(ctx, sizeof(u32) * (m + 1), s);
    HCI_LAUNCH(ctx, "rc_chunks", s, rc_count_kernel, ceil_div(m + 1, 256), 256, 0, off.as<u32>(), m, cnt.as<u32>());
    scan_u32_to_u32(ctx, cnt.as<u32>(), cptr.as<u32>(), m + 1, s);
    nch = read_scalar(cptr.as<u32>() + m, s);
    chunks = dev_alloc(ctx, sizeof(u32) * 3 * (nch > 0 ? nch : 1), s);
    HCI_LAUNCH(ctx, "rc_chunks", s, rc_fill_kernel, ceil_div(m, 256), 256, 0, off.as<u32>(), m, cptr.as<u32>(),
               chunks.as<u32>());
}

template <class VT>
void rc_launch(hci_ctx_s* ctx, Space* sp, RcInts<VT> T, const VT* cx, const double* c, double* sigma,
               hipStream_t s, const char* na, const char* nb) {
    const SpaceView S = space_view(*sp, ctx->n);
    const u32 maxl = (u32)sp->rc_maxdeg + 1;
    const size_t lds_a = rc_lds_bytes<VT>(ctx->n, maxl), lds_b = rc_lds_bytes<VT>(ctx->n, 1);
    HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(rc_alpha_kernel<VT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_a));
    HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(rc_beta_kernel<VT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_b));
    const i64 ga = row_grid(sp->rc_nch_a * RC_BLOCK, RC_BLOCK, RC_BLOCK);
    const i64 gb = row_grid(sp->rc_nch_b * RC_BLOCK, RC_BLOCK, RC_BLOCK);
    // beta-string bitmaps of neighbour groups (as the stored build), within the tile's LDS
    RcBitmaps M{0u, 0u, 0.0f};
    const char* force_search = std::getenv("HCI_AB_SEARCH");  // "1": always scan (tests)
    if (sp->nub <= 65535 && !(force_search && force_search[0] == '1')) {
        const u32 W = (u32)ceil_div(sp->nub, 32);
        const u32 G = (u32)std::min<i64>(64, RC_BM_BYTES / (6 * (i64)W));
        if (G >= 1) M = RcBitmaps{W, G, (float)sp->n_bs / (float)sp->nub};
        // "1": look every neighbour bucket up, whatever scanning it would cost (tests)
        const char* force_lookup = std::getenv("HCI_RC_LOOKUP");
        if (G >= 1 && force_lookup && force_lookup[0] == '1') M.nbs_avg = 0.0f;
    }
    HCI_LAUNCH(ctx, na, s, rc_alpha_kernel<VT>, ga, RC_BLOCK, lds_a, S, T, sp->rc_chunk_a.as<u32>(), sp->rc_nch_a, cx,
               c, sp->hdiag.as<double>(), sigma, maxl, M);
    HCI_LAUNCH(ctx, nb, s, rc_beta_kernel<VT>, gb, RC_BLOCK, lds_b, S, T, sp->rc_chunk_b.as<u32>(), sp->rc_nch_b, cx,
               sigma);
}

// largest alpha-single degree among the unique alpha strings
__global__ void rc_maxdeg_kernel(const u32* __restrict__ ptr, i64 m, unsigned int* __restrict__ out) {
    const i64 a = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    u32 v = a < m ? ptr[a + 1] - ptr[a] : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const u32 w = (u32)__shfl_xor((int)v, o, HCI_WAVE);
        v = w > v ? w : v;
    }
    if (lane_id() == 0 && v) atomicMax(out, v);
}

__global__ void rc_to_f32(const double* __restrict__ x, float* __restrict__ y, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

}  // namespace

void recompute_apply(hci_ctx_s* ctx, Space* sp, const double* c, double* sigma, int precision, hipStream_t s) {
    ensure_diag(ctx, sp, s);
    if (!sp->rc_chunk_a.ptr) {
        rc_chunks(ctx, sp->aoff, sp->nua, sp->rc_chunk_a, sp->rc_nch_a, s);
        rc_chunks(ctx, sp->boff, sp->nub, sp->rc_chunk_b, sp->rc_nch_b, s);
        DevMem mx = dev_alloc(ctx, sizeof(u32), s);
        HIP_CHECK(hipMemsetAsync(mx.ptr, 0, sizeof(u32), s));
        HCI_LAUNCH(ctx, "rc_chunks", s, rc_maxdeg_kernel, ceil_div(sp->nua, 256), 256, 0, sp->as_ptr.as<u32>(),
                   sp->nua, (unsigned int*)mx.as<u32>());
        sp->rc_maxdeg = read_scalar(mx.as<u32>(), s);
        HCI_REQUIRE(sp->rc_maxdeg < 0xffffu, HCI_E_UNSUPPORTED, "recomputed product: alpha degree above 65534");
    }
    const IntView I = int_view(ctx->ints);
    const i64 N = sp->N;
    if (precision == HCI_FP32_MIXED) {
        if (!sp->c32.ptr) sp->c32 = dev_alloc(ctx, sizeof(float) * N, s);
        HCI_LAUNCH(ctx, "c_to_f32", s, rc_to_f32, ceil_div(N, 256), 256, 0, c, sp->c32.as<float>(), N);
        rc_launch<float>(ctx, sp, rc_ints_f32(I), sp->c32.as<float>(), c, sigma, s, "sigma_recompute_f32",
                         "sigma_recompute_f32_beta");
    } else {
        rc_launch<double>(ctx, sp, rc_ints_f64(I), c, c, sigma, s, "sigma_recompute_f64",
                          "sigma_recompute_f64_beta");
    }
}
