// Spin-traced one- and two-particle (transition) density matrices on V,
//   rdm1[p][q]       = sum_s  <bra| a+_ps a_qs |ket>,
//   rdm2[p][q][r][s] = sum_st <bra| a+_ps a+_rt a_st a_qs |ket>,
// accumulated by looping over the same single and double connections as
// the Hamiltonian product (Sec. "Computational Details").
//
// Diagonal pairs (i = j) only involve occupation numbers, so they are
// reduced as an occupation-correlation product: D[x][y] = sum_i bra_i ket_i
// n_x(i) n_y(i) over spin orbitals x, y, block partials then a fixed-order
// sum.  Off-diagonal pairs go through rdm_det_kernel (below): per-chunk
// owners, private copies per workgroup, fixed-order sums.  The screened PT2
// pairs of the relaxed gradient (Gamma^{dc}) are sorted by excitation class
// and reduced class by class.  No floating-point atomics anywhere, so the
// result is the same bit for bit from run to run.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <queue>
#include <vector>

#include "slater.h"

namespace {

constexpr int OCC_CHUNK = 256;

__device__ __forceinline__ i64 r2idx(int n, int p, int q, int r, int s) {
    return (((i64)p * n + q) * n + r) * n + s;
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

// ---------------------------------------------------- screened pairs
// Gamma^{dc} of the PT2 pieces: bra D_a (weight d_a), ket D_i (weight c_i)
// over the screened connection list (Sec. "Computational Details").  Each
// pair is one excitation class: a single v -> u of one spin, an
// opposite-spin double, or a same-spin double with holes v1 < v2 and
// particles u1 < u2.  The class and its orbitals form a 27-bit key
// (type << 24 | four 6-bit orbitals); the pairs are sorted by key (stable, so
// pairs of one class keep their list order) and each class is reduced by one
// wavefront in a fixed order:
//   doubles: X = sum of the signed weights, added to its table entry;
//   singles: g = sum of x, A_k = sum x [k occupied in the ket's string of the
//   excited spin, k != v], B_k = sum x [k occupied in the other string].
// pair_table_kernel then gives every rdm entry one owner that adds the
// entries of the tables it receives (the same terms an operator application
// per pair gives: see the comments there).
constexpr u32 PK_SKIP = 7u;  // type of a pair with zero weight (sorted last, ignored)

struct PairClass {
    u32 key;    // type << 24 | o0 << 18 | o1 << 12 | o2 << 6 | o3
    double x;   // signed weight
    u64 same;   // singles: ket string of the excited spin
    u64 other;  // singles: ket string of the other spin
};

__device__ __forceinline__ u32 pk_pack(u32 type, int o0, int o1, int o2, int o3) {
    return type << 24 | (u32)o0 << 18 | (u32)o1 << 12 | (u32)o2 << 6 | (u32)o3;
}

__device__ __forceinline__ PairClass pair_class(double w, u64 ai, u64 bi, u64 aj, u64 bj) {
    PairClass P{pk_pack(PK_SKIP, 0, 0, 0, 0), 0.0, 0, 0};
    if (w == 0.0) return P;
    const u64 xa = ai ^ aj, xb = bi ^ bj;
    const int da = popc64(xa) >> 1, db = popc64(xb) >> 1;
    if (da + db == 1) {  // single v -> u (type 0 alpha, 1 beta)
        const bool al = da == 1;
        const u64 sj = al ? aj : bj, x = al ? xa : xb;
        const int v = ctz64(sj & x), u = ctz64(x & ~sj);
        P.key = pk_pack(al ? 0u : 1u, u, v, 0, 0);
        P.x = w * sign_between(sj, v, u);
        P.same = sj;
        P.other = al ? bj : aj;
        return P;
    }
    if (da == 1 && db == 1) {  // type 2: alpha v1 -> u1 with beta v2 -> u2
        const int v1 = ctz64(aj & xa), u1 = ctz64(ai & xa);
        const int v2 = ctz64(bj & xb), u2 = ctz64(bi & xb);
        P.key = pk_pack(2u, u1, v1, u2, v2);
        P.x = w * (sign_between(aj, v1, u1) * sign_between(bj, v2, u2));
        return P;
    }
    // same-spin double (type 3 alpha, 4 beta); ctz order gives v1 < v2, u1 < u2
    const bool al = da == 2;
    const u64 sj = al ? aj : bj, x2 = al ? xa : xb;
    u64 holes = sj & x2, parts = x2 & ~sj;
    const int v1 = ctz64(holes);
    holes &= holes - 1;
    const int v2 = ctz64(holes);
    const int u1 = ctz64(parts);
    parts &= parts - 1;
    const int u2 = ctz64(parts);
    P.key = pk_pack(al ? 3u : 4u, u1, v1, u2, v2);
    P.x = w * sign_double(sj, v1, u1, v2, u2);
    return P;
}

__device__ __forceinline__ PairClass pair_class_at(i64 t, const u64* __restrict__ a_hi,
                                                   const u64* __restrict__ a_lo, const u32* __restrict__ idx,
                                                   const double* __restrict__ wa, const u64* __restrict__ dets,
                                                   const double* __restrict__ c) {
    const u32 i = idx[t];
    return pair_class(wa[t] * c[i], a_hi[t], a_lo[t], dets[2 * (i64)i], dets[2 * (i64)i + 1]);
}

// key << 32 | t for every pair of the pass
__global__ void pair_keys_kernel(const u64* __restrict__ a_hi, const u64* __restrict__ a_lo,
                                 const u32* __restrict__ idx, const double* __restrict__ wa,
                                 const u64* __restrict__ dets, const double* __restrict__ c, i64 M,
                                 u64* __restrict__ keyed) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    keyed[t] = (u64)pair_class_at(t, a_hi, a_lo, idx, wa, dets, c).key << 32 | (u64)t;
}

__global__ void pair_heads_kernel(const u64* __restrict__ keyed, i64 M, u32* __restrict__ flags) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    flags[t] = (t == 0 || (keyed[t] >> 32) != (keyed[t - 1] >> 32)) ? 1u : 0u;
}

__global__ void pair_starts_kernel(const u32* __restrict__ flags, const u32* __restrict__ pos, i64 M,
                                   i64* __restrict__ start) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < M && flags[t]) start[pos[t]] = t;
}

// one wavefront per class segment [start[g], start[g + 1]) of the sorted pairs
__global__ void __launch_bounds__(256) pair_segments_kernel(
    const u64* __restrict__ keyed, const i64* __restrict__ start, i64 nseg, i64 M, const u64* __restrict__ a_hi,
    const u64* __restrict__ a_lo, const u32* __restrict__ idx, const double* __restrict__ wa,
    const u64* __restrict__ dets, const double* __restrict__ c, int n, double* __restrict__ dtab,
    double* __restrict__ stab) {
    const int lane = lane_id();
    const i64 nw = (i64)gridDim.x * (blockDim.x / 64);
    const i64 n4 = (i64)n * n * n * n;
    for (i64 g = (i64)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; g < nseg; g += nw) {
        const i64 b = start[g], e = g + 1 < nseg ? start[g + 1] : M;
        const u32 key = (u32)(keyed[b] >> 32);
        const u32 type = key >> 24;
        if (type == PK_SKIP) continue;
        const int o0 = (key >> 18) & 63, o1 = (key >> 12) & 63, o2 = (key >> 6) & 63, o3 = key & 63;
        if (type >= 2) {
            // lane-strided partial sums in list order, then a fixed butterfly
            double acc = 0.0;
            for (i64 t = b + lane; t < e; t += 64)
                acc += pair_class_at((i64)(u32)keyed[t], a_hi, a_lo, idx, wa, dets, c).x;
            acc = wave_sum_f64(acc);
            if (lane == 0) dtab[(i64)(type - 2) * n4 + (((i64)o0 * n + o1) * n + o2) * n + o3] += acc;
            continue;
        }
        // singles: lane k keeps A_k, B_k; the pairs go 64 at a time, each
        // broadcast to every lane in list order
        const int v = o1;
        double A = 0.0, B = 0.0, gsum = 0.0;
        for (i64 base = b; base < e; base += 64) {
            PairClass mine{0u, 0.0, 0, 0};
            if (base + lane < e) mine = pair_class_at((i64)(u32)keyed[base + lane], a_hi, a_lo, idx, wa, dets, c);
            const int cnt = (int)min((i64)64, e - base);
            for (int j = 0; j < cnt; ++j) {
                const double xj = __shfl(mine.x, j, HCI_WAVE);
                const u64 sj = __shfl(mine.same, j, HCI_WAVE), oj = __shfl(mine.other, j, HCI_WAVE);
                gsum += xj;
                if (lane < n) {
                    if (lane != v && test_bit(sj, lane)) A += xj;
                    if (test_bit(oj, lane)) B += xj;
                }
            }
        }
        double* row = stab + (((i64)type * n + o0) * n + v) * (2 * n + 1);
        if (lane < n) {
            row[lane] += A;
            row[n + lane] += B;
        }
        if (lane == 0) row[2 * n] += gsum;
    }
}

// Every rdm entry adds what the class tables give it:
//   alpha-beta double (u1 v1 | u2 v2) with sum X: [u1 v1 u2 v2] and [u2 v2 u1 v1] += X;
//   same-spin double (u1 < u2, v1 < v2), X: [u1 v1 u2 v2], [u2 v2 u1 v1] += X and
//     [u1 v2 u2 v1], [u2 v1 u1 v2] -= X, so entry (p q r s) with p != r, q != s
//     receives +-X(min(p,r), min(q,s), max(p,r), max(q,s)), + when p < r and
//     q < s agree;
//   single v -> u (spectator k): [u v k k] and [k k u v] += A_k + B_k,
//     [u k k v] and [k v u k] -= A_k; rdm1[u][v] += g.
__global__ void pair_table_kernel(const double* __restrict__ dtab, const double* __restrict__ stab, int n,
                                  double* __restrict__ r1, double* __restrict__ r2) {
    const i64 n2 = (i64)n * n, n4 = n2 * n2;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n4 + n2) return;
    const int w = 2 * n + 1;
    auto S = [&](int sp, int u, int v, int k) { return stab[(((i64)sp * n + u) * n + v) * w + k]; };
    if (t >= n4) {  // rdm1
        const int p = (int)((t - n4) / n), q = (int)((t - n4) % n);
        if (p != q) r1[(i64)p * n + q] += S(0, p, q, 2 * n) + S(1, p, q, 2 * n);
        return;
    }
    const int p = (int)(t / (n2 * n)), q = (int)(t / n2 % n), r = (int)(t / n % n), s = (int)(t % n);
    auto D = [&](int type, int a, int b2, int c2, int d) {
        return dtab[(i64)type * n4 + (((i64)a * n + b2) * n + c2) * n + d];
    };
    double v = D(0, p, q, r, s) + D(0, r, s, p, q);
    if (p != r && q != s) {
        const double X = D(1, min(p, r), min(q, s), max(p, r), max(q, s)) +
                         D(2, min(p, r), min(q, s), max(p, r), max(q, s));
        v += ((p < r) == (q < s)) ? X : -X;
    }
    for (int sp = 0; sp < 2; ++sp) {
        if (r == s && p != q) v += S(sp, p, q, r) + S(sp, p, q, n + r);
        if (p == q && r != s) v += S(sp, r, s, p) + S(sp, r, s, n + p);
        if (q == r && p != s) v -= S(sp, p, s, q);
        if (p == s && r != q) v -= S(sp, r, q, p);
    }
    r2[t] += v;
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

// ---------------------------------------------------------------- off-diagonal kernels
// Off-diagonal pairs (row i = bra determinant, j = ket determinant) without
// atomics.  Every kernel below runs a persistent grid of P workgroups over a
// list of row chunks (up to RDM_CHUNK rows of one bucket each) that assigns
// each chunk to one workgroup and balances an estimated cost (RdmChunks).
// Workgroup p adds into its own private copy of the output in global memory
// -- the canonical half T of rdm2 (one entry of each (pq|rs), (rs|pq) pair;
// rdm2 = T + T^swap at the end) and rdm1 -- and the copies are summed in a
// fixed order.  Inside a workgroup every entry has one writer at a time:
//   * rdm_same_kernel, once over the alpha buckets (connections with the same
//     alpha string: beta singles and doubles) and once over the beta buckets
//     in beta-major order (the same beta string: alpha singles and doubles).
//     The chunk's rows are staged in LDS and the bucket's candidates are read
//     a piece at a time, up to SS_PER_THREAD per thread; the rows are taken
//     one after another, with a barrier after each row (one row's
//     contributions fall on distinct entries, two rows' may not), and each
//     wavefront gathers a row's connections among its candidates into a
//     queue so the contribution code runs once per row.  A single v -> u
//     adds x to S2[u][v] (later rdm1[u][v] and the opposite-spin spectators,
//     which the bucket's fixed string gives) and to S3[u][v][k] for the
//     same-spin spectators k (in LDS when it fits, else straight into the
//     copy); a double goes into an LDS table of the particle and hole pairs
//     when it fits (small n), else straight into the copy.
//   * rdm_nb_kernel, over the alpha buckets: alpha single x beta single
//     connections.  For a group of alpha neighbours A' of the chunk's bucket A
//     the kernel keeps bitmaps of the beta strings present in each A'
//     (build_beta_maps) and a tile [u2][v2] per A' (in LDS when it fits, else
//     the entries of the copy that A' fixes); neighbour q is owned by
//     wavefront q mod RDM_WAVES, whose memory operations take effect in
//     program order.  The beta singles of a few rows at a time are staged in
//     LDS, so the owner only tests its bitmap, gathers ket and adds.
constexpr int RDM_BLOCK = 1024;
constexpr int RDM_WAVES = RDM_BLOCK / HCI_WAVE;
// two workgroups of 16 wavefronts per CU: 8 per SIMD, which caps the kernels at 64 VGPRs
constexpr int RDM_WAVES_PER_SIMD = 8;
constexpr u32 RDM_CHUNK = 1024;
constexpr int SS_PER_THREAD = 4;     // bucket candidates held per thread
constexpr u32 SS_PIECE = SS_PER_THREAD * RDM_BLOCK;  // candidates of the bucket taken at a time

// non-atomic update of an entry this thread (or wavefront) alone writes at this moment
__device__ __forceinline__ void own_add(double* p, double v) { *p += v; }

// Candidates of one row gathered per wavefront: slot l in lane l (the
// candidate's string and ket coefficient), filled from a ballot mask by
// shuffles; every lane calls push together.
struct HitQueue {
    int n = 0;  // queued, wave-uniform
    u64 y = 0;
    double w = 0.0;
    __device__ __forceinline__ bool full_for(u64 m) const { return n + popc64(m) > HCI_WAVE; }
    __device__ __forceinline__ void push(u64 m, u64 yy, double ww) {
        const int cnt = popc64(m);
        const int l = lane_id();
        const bool mine = l >= n && l < n + cnt;
        const int src = mine ? nth_set_bit(m, l - n) : l;
        const u64 sy = __shfl(yy, src, HCI_WAVE);
        const double sw = __shfl(ww, src, HCI_WAVE);
        if (mine) {
            y = sy;
            w = sw;
        }
        n += cnt;
    }
};

struct SameArgs {
    int n;
    const u32* list;    // chunks of this workgroup: list[wptr[p] .. wptr[p + 1])
    const u32* wptr;
    const u32* off;     // [nbuck + 1] first position of each bucket
    const u64* xs;      // [nbuck] the fixed string of each bucket
    const u64* ys;      // [N] the string of the excited spin at each position
    const double* bra;  // [N] in the same order
    const double* ket;
    double* priv;
    i64 stride;
};

// LDS: rows (string, bra) | S2 [n][n] | S3 [n][n][n] | XD [P][P] | pair table; a piece of
// candidates sits in registers, up to SS_PER_THREAD per thread.  With DX (small
// n: the whole table fits on chip, one workgroup per CU) the doubles add into
// XD, indexed by the particle pair u1 < u2 and the hole pair v1 < v2 (P = n(n-1)/2
// pairs), instead of the private copy, so no row waits for global memory.
template <bool S3, bool DX>
__global__ void __launch_bounds__(RDM_BLOCK, DX ? RDM_WAVES_PER_SIMD / 2 : RDM_WAVES_PER_SIMD) rdm_same_kernel(SameArgs G) {
    extern __shared__ double lds[];
    constexpr u32 RS = DX ? RDM_CHUNK / 2 : RDM_CHUNK;  // rows staged at a time
    const u32 tid = threadIdx.x;
    const int n = G.n;
    const int nn = n * n;
    const int np2 = n * (n - 1) / 2;
    const i64 n4 = (i64)nn * nn;
    u64* ry = reinterpret_cast<u64*>(lds);
    double* rw = lds + RS;
    double* s2 = lds + 2 * RS;
    double* s3 = s2 + nn;
    double* xd = s3 + (S3 ? nn * n : 0);
    u16* pairs = reinterpret_cast<u16*>(xd + (DX ? np2 * np2 : 0));  // pair index -> a | b << 8
    double* r2 = G.priv + (i64)blockIdx.x * G.stride;
    double* r1 = r2 + n4;
    const int nacc = nn + (S3 ? nn * n : 0);
    if constexpr (DX) {
        for (int x = (int)tid; x < np2 * np2; x += RDM_BLOCK) xd[x] = 0.0;
        for (int b = 1; b < n; ++b)
            for (int a = (int)tid; a < b; a += RDM_BLOCK) pairs[b * (b - 1) / 2 + a] = (u16)(a | b << 8);
    }
    for (u32 t = G.wptr[blockIdx.x]; t < G.wptr[blockIdx.x + 1]; ++t) {
        const u32 bk = G.list[3 * (i64)t], row0 = G.list[3 * (i64)t + 1], row1 = G.list[3 * (i64)t + 2];
        const u32 lo = G.off[bk], hi = G.off[bk + 1];
        const u64 X = G.xs[bk];
        const u32 nrow = row1 - row0;
        for (int x = (int)tid; x < nacc; x += RDM_BLOCK) s2[x] = 0.0;
        for (u32 p0 = lo; p0 < hi; p0 += SS_PIECE) {
            const u32 np = min(SS_PIECE, hi - p0);
            u64 Yc[SS_PER_THREAD];
            double kc[SS_PER_THREAD];
#pragma unroll
            for (int t = 0; t < SS_PER_THREAD; ++t) {
                const u32 j = tid + (u32)t * RDM_BLOCK;
                Yc[t] = j < np ? G.ys[p0 + j] : 0ull;
                kc[t] = j < np ? G.ket[p0 + j] : 0.0;
            }
            for (u32 rs0 = 0; rs0 < nrow; rs0 += RS) {
                const u32 nr = min(RS, nrow - rs0);
                __syncthreads();  // the previous rows are done (and the accumulators cleared)
                for (u32 i = tid; i < nr; i += RDM_BLOCK) {
                    ry[i] = G.ys[row0 + rs0 + i];
                    rw[i] = G.bra[row0 + rs0 + i];
                }
                __syncthreads();
                for (u32 i = 0; i < nr; ++i) {
                    const double wb = rw[i];
                    if (wb == 0.0) continue;  // uniform
                    const u64 Yi = ry[i];
                    // the row's connections among this thread's candidates, gathered per
                    // wavefront (slot l in lane l) so the contribution code runs once for
                    // up to 64 of them; they are distinct excitations, so distinct entries
                    HitQueue q;
                    auto contribute = [&]() {
                        // a single's same-spin spectators when S3 is not on chip:
                        // (hit, spectator) pairs spread over the lanes below
                        u64 sm = 0;
                        int su = 0, sv = 0;
                        double sx = 0.0;
                        if (lane_id() < q.n) {
                            const u64 Yj = q.y;
                            const u64 xy = Yi ^ Yj;
                            if (popc64(xy) == 2) {
                                const int u = ctz64(Yi & xy), v = ctz64(Yj & xy);
                                const double x = wb * q.w * sign_between(Yj, v, u);
                                own_add(&s2[u * n + v], x);
                                if constexpr (S3) {
                                    for (u64 m = Yi & Yj; m; m &= m - 1)  // same-spin spectators
                                        own_add(&s3[(u * n + v) * n + ctz64(m)], x);
                                } else {
                                    sm = Yi & Yj;
                                    su = u;
                                    sv = v;
                                    sx = x;
                                }
                            } else {
                                u64 parts = Yi & xy, holes = Yj & xy;
                                const int u1 = ctz64(parts);
                                parts &= parts - 1;
                                const int u2 = ctz64(parts);
                                const int v1 = ctz64(holes);
                                holes &= holes - 1;
                                const int v2 = ctz64(holes);
                                const double x = wb * q.w * sign_double(Yj, v1, u1, v2, u2);
                                if constexpr (DX) {
                                    own_add(&xd[(u2 * (u2 - 1) / 2 + u1) * np2 + v2 * (v2 - 1) / 2 + v1], x);
                                } else {
                                    own_add(&r2[r2idx(n, u1, v1, u2, v2)], x);
                                    own_add(&r2[r2idx(n, u1, v2, u2, v1)], -x);
                                }
                            }
                        }
                        if constexpr (!S3) {
                            // lane l takes pair base + l: the hit is the last lane whose
                            // exclusive offset is <= it, the spectator its rank in sm
                            // (distinct (u, v, k) within a row, so distinct entries)
                            const int cnt = popc64(sm);
                            int incl = cnt;
#pragma unroll
                            for (int off = 1; off < HCI_WAVE; off <<= 1) {
                                const int y = __shfl_up(incl, off, HCI_WAVE);
                                if (lane_id() >= off) incl += y;
                            }
                            const int excl = incl - cnt;
                            const int total = __shfl(incl, HCI_WAVE - 1, HCI_WAVE);
                            for (int base = 0; base < total; base += HCI_WAVE) {
                                const int p = base + lane_id();
                                int lo = 0, hi = HCI_WAVE - 1;
                                while (lo < hi) {  // uniform trip count: every lane shuffles
                                    const int mid = (lo + hi + 1) >> 1;
                                    if (__shfl(excl, mid, HCI_WAVE) <= p) lo = mid;
                                    else hi = mid - 1;
                                }
                                const u64 hm = __shfl(sm, lo, HCI_WAVE);
                                const int hu = __shfl(su, lo, HCI_WAVE), hv = __shfl(sv, lo, HCI_WAVE);
                                const double hx = __shfl(sx, lo, HCI_WAVE);
                                const int r = p - __shfl(excl, lo, HCI_WAVE);
                                if (p < total) {
                                    const int k = nth_set_bit(hm, r);
                                    own_add(&r2[r2idx(n, hu, hv, k, k)], hx);
                                    own_add(&r2[r2idx(n, hu, k, k, hv)], -hx);
                                }
                            }
                        }
                        q.n = 0;
                    };
#pragma unroll
                    for (int t = 0; t < SS_PER_THREAD; ++t) {
                        const int d = tid + (u32)t * RDM_BLOCK < np ? popc64(Yi ^ Yc[t]) : 0;  // 0 for the row itself
                        const u64 m = ballot(d == 2 || d == 4);
                        if (m) {
                            if (q.full_for(m)) contribute();
                            q.push(m, Yc[t], kc[t]);
                        }
                    }
                    if (q.n) contribute();
                    __syncthreads();  // the next row may add to the same entries
                }
            }
        }
        // S2: rdm1 and the opposite-spin spectators (the bucket's fixed string)
        for (int x = (int)tid; x < nn; x += RDM_BLOCK) {
            const double val = s2[x];
            if (val == 0.0) continue;
            const int u = x / n, v = x % n;
            own_add(&r1[x], val);
            for (u64 m = X; m; m &= m - 1) own_add(&r2[r2idx(n, u, v, ctz64(m), ctz64(m))], val);
        }
        __syncthreads();  // S2 and S3 can meet on an entry
        if constexpr (S3) {
            for (int x = (int)tid; x < nn * n; x += RDM_BLOCK) {
                const double val = s3[x];
                if (val == 0.0) continue;  // (also every k = v entry)
                const int u = x / nn, v = (x / n) % n, k = x % n;
                own_add(&r2[r2idx(n, u, v, k, k)], val);
                own_add(&r2[r2idx(n, u, k, k, v)], -val);
            }
        }
        if constexpr (DX) {
            // doubles: [u1 v1 u2 v2] += X and [u1 v2 u2 v1] -= X, distinct entries for distinct pairs
            for (int x = (int)tid; x < np2 * np2; x += RDM_BLOCK) {
                const double val = xd[x];
                if (val == 0.0) continue;
                xd[x] = 0.0;
                const u32 pu = pairs[x / np2], pv = pairs[x % np2];
                const int u1 = (int)(pu & 0xffu), u2 = (int)(pu >> 8), v1 = (int)(pv & 0xffu), v2 = (int)(pv >> 8);
                own_add(&r2[r2idx(n, u1, v1, u2, v2)], val);
                own_add(&r2[r2idx(n, u1, v2, u2, v1)], -val);
            }
        }
        __syncthreads();  // LDS is reused by the next chunk
    }
}

struct NbPlan {
    int n, G;      // G: alpha neighbours per group (bitmaps and tiles rebuilt per group)
    int W;         // beta-string bitmap words per neighbour (0: scan the neighbour buckets)
    int R;         // rows whose beta singles are staged at a time
    int ds;        // staged beta singles per row (the most a string has)
    bool tile;     // tiles [u2][v2] in LDS (else straight into the copy)
    int o_sing, o_row, o_nb, o_bm;  // byte offsets: singles, rows, neighbour info, bitmaps
    int bytes;
};

constexpr u32 NB_NONE = 0xffffffffu;
constexpr int NB_ROWS = 2;  // rows whose gathers one wavefront keeps in flight
constexpr u32 NB_SCAN = 4;  // without bitmaps: scan a neighbour bucket of at most NB_SCAN beta singles per row

template <bool BM, bool TILE>
__global__ void __launch_bounds__(RDM_BLOCK, RDM_WAVES_PER_SIMD) rdm_nb_kernel(SpaceView S, NbPlan P, const u32* __restrict__ list,
                                                           const u32* __restrict__ wptr,
                                                           const double* __restrict__ bra,
                                                           const double* __restrict__ ket, double* __restrict__ priv,
                                                           i64 stride) {
    extern __shared__ double lds[];
    const u32 tid = threadIdx.x;
    const int lane = lane_id();
    const u32 wave = tid / HCI_WAVE;
    const int n = P.n;
    const int nn = n * n;
    const i64 n4 = (i64)nn * nn;
    unsigned char* base = reinterpret_cast<unsigned char*>(lds);
    double* tiles = lds;  // [G][n][n] when TILE
    uint2* sing = reinterpret_cast<uint2*>(base + P.o_sing);    // [R][ds]: (beta string, u2 * n + v2 | sign bit)
    u64* rB = reinterpret_cast<u64*>(base + P.o_row);           // [R] beta string of the row
    double* rW = reinterpret_cast<double*>(rB + P.R);            // [R] bra of the row
    u32* nbl = reinterpret_cast<u32*>(base + P.o_nb);            // [G] first row of the neighbour bucket
    u32* nbh = nbl + P.G;                                        // [G] end of it
    u32* nbt = nbh + P.G;                                        // [G] u1 * n + v1
    double* nbs = reinterpret_cast<double*>(nbt + ((P.G + 1) & ~1));  // [G] sign of the alpha single
    u32* bm = reinterpret_cast<u32*>(base + P.o_bm);
    u16* pre = reinterpret_cast<u16*>(bm + (i64)P.G * P.W);
    double* r2 = priv + (i64)blockIdx.x * stride;
    if constexpr (TILE)
        for (int x = (int)tid; x < P.G * nn; x += RDM_BLOCK) tiles[x] = 0.0;
    for (u32 ct = wptr[blockIdx.x]; ct < wptr[blockIdx.x + 1]; ++ct) {
        const u32 a = list[3 * (i64)ct], row0 = list[3 * (i64)ct + 1], row1 = list[3 * (i64)ct + 2];
        const u64 A = S.ua[a];
        const u32 t0 = S.as_ptr[a];
        const u32 deg = S.as_ptr[a + 1] - t0;
        for (u32 tg0 = 0; tg0 < deg; tg0 += (u32)P.G) {
            const u32 tg1 = min(tg0 + (u32)P.G, deg);
            const u32 nt = tg1 - tg0;
            if constexpr (BM) build_beta_maps<RDM_BLOCK>(S, t0, tg0, tg1, (u32)P.W, bm, pre, tid);
            for (u32 q = tid; q < nt; q += RDM_BLOCK) {
                const u32 a2 = S.as_idx[t0 + tg0 + q];
                const u64 A2 = S.ua[a2];
                const u64 xa = A ^ A2;
                const int u1 = ctz64(A & xa), v1 = ctz64(A2 & xa);
                nbl[q] = S.aoff[a2];
                nbh[q] = S.aoff[a2 + 1];
                nbt[q] = (u32)(u1 * n + v1);
                nbs[q] = sign_between(A2, v1, u1);
            }
            for (u32 s0 = row0; s0 < row1; s0 += (u32)P.R) {
                const u32 nr = min((u32)P.R, row1 - s0);
                __syncthreads();  // neighbour info written; the previous rows are done
                for (u32 i = tid; i < nr; i += RDM_BLOCK) {
                    rB[i] = S.beta[s0 + i];
                    rW[i] = bra[s0 + i];
                }
                {
                    for (u32 x = tid; x < nr * (u32)P.ds; x += RDM_BLOCK) {
                        const u32 i = x / (u32)P.ds, e = x % (u32)P.ds;
                        const u32 b = S.ib[s0 + i];
                        const u32 k = S.bs_ptr[b] + e;
                        uint2 val = make_uint2(NB_NONE, 0u);
                        if (k < S.bs_ptr[b + 1]) {
                            const u32 bp = S.bs_idx[k];
                            const u64 B = S.beta[s0 + i];
                            const u64 bj = S.ub[bp];
                            const u64 xb = B ^ bj;
                            const int v2 = ctz64(bj & xb), u2 = ctz64(B & xb);
                            const double sg = sign_between(bj, v2, u2);
                            val = make_uint2(bp, (u32)(u2 * n + v2) | (sg < 0.0 ? 0x80000000u : 0u));
                        }
                        sing[x] = val;
                    }
                }
                __syncthreads();
                for (u32 q = wave; q < nt; q += RDM_WAVES) {
                    const u32 lo2 = nbl[q];
                    const double sa = nbs[q];
                    const u32 t = nbt[q];
                    double* tile = TILE ? tiles + (i64)q * nn : r2 + r2idx(n, (int)(t / (u32)n), (int)(t % (u32)n), 0, 0);
                    if constexpr (BM) {
                        const u32* bmq = bm + q * (u32)P.W;
                        const u16* preq = pre + q * (u32)P.W;
                        // NB_ROWS rows at a time: their ket gathers are in flight
                        // together, then the tile additions follow in row order
                        for (u32 i0 = 0; i0 < nr; i0 += NB_ROWS) {
                            for (u32 e = (u32)lane; e < (u32)P.ds; e += HCI_WAVE) {
                                double x[NB_ROWS];
                                u32 slot[NB_ROWS];
#pragma unroll
                                for (int r = 0; r < NB_ROWS; ++r) {
                                    x[r] = 0.0;
                                    slot[r] = 0u;
                                    const u32 i = i0 + (u32)r;
                                    if (i >= nr) continue;
                                    const uint2 sv = sing[i * (u32)P.ds + e];
                                    if (sv.x == NB_NONE) continue;
                                    const u32 word = bmq[sv.x >> 5], bit = sv.x & 31u;
                                    if (((word >> bit) & 1u) == 0u) continue;
                                    const u32 j = lo2 + (u32)preq[sv.x >> 5] + (u32)__popc(word & ((1u << bit) - 1u));
                                    const double w = rW[i] * sa;
                                    x[r] = ((sv.y >> 31) ? -w : w) * ket[j];
                                    slot[r] = sv.y & 0x7fffffffu;
                                }
#pragma unroll
                                for (int r = 0; r < NB_ROWS; ++r)
                                    if (x[r] != 0.0) own_add(&tile[slot[r]], x[r]);
                            }
                        }
                    } else if (nbh[q] - lo2 <= NB_SCAN * (u32)P.ds) {  // scan a small neighbour bucket
                        const u32 hi2 = nbh[q];
                        for (u32 i = 0; i < nr; ++i) {
                            const double w = rW[i] * sa;
                            if (w == 0.0) continue;  // uniform
                            const u64 B = rB[i];
                            for (u32 j = lo2 + (u32)lane; j < hi2; j += HCI_WAVE) {
                                const u64 bj = S.beta[j];
                                const u64 xb = B ^ bj;
                                if (popc64(xb) != 2) continue;
                                const int v2 = ctz64(bj & xb), u2 = ctz64(B & xb);
                                own_add(&tile[u2 * n + v2], w * ket[j] * sign_between(bj, v2, u2));
                            }
                        }
                    } else {  // look each beta single of the row up in a large one (sorted by beta)
                        const u32 len2 = nbh[q] - lo2;
                        for (u32 i = 0; i < nr; ++i) {
                            const double w = rW[i] * sa;
                            if (w == 0.0) continue;  // uniform
                            for (u32 e = (u32)lane; e < (u32)P.ds; e += HCI_WAVE) {
                                const uint2 sv = sing[i * (u32)P.ds + e];
                                if (sv.x == NB_NONE) continue;
                                const u64 bj = S.ub[sv.x];
                                const u32 pos = lower_bound_u64(S.beta + lo2, len2, bj);
                                if (pos >= len2 || S.beta[lo2 + pos] != bj) continue;
                                const double x = w * ket[lo2 + pos];
                                own_add(&tile[sv.y & 0x7fffffffu], (sv.y >> 31) ? -x : x);
                            }
                        }
                    }
                }
            }
            __syncthreads();
            // flush this group's tiles: neighbour q fixes (u1, v1)
            if constexpr (TILE) {
                for (int x = (int)tid; x < (int)nt * nn; x += RDM_BLOCK) {
                    const double val = tiles[x];
                    if (val == 0.0) continue;
                    tiles[x] = 0.0;
                    const u32 t = nbt[x / nn];
                    own_add(&r2[r2idx(n, (int)(t / (u32)n), (int)(t % (u32)n), 0, 0) + x % nn], val);
                }
                __syncthreads();
            }
        }
    }
}

// Estimated time of one row of bucket a in the alpha single x beta single
// kernel: a pass per alpha neighbour, plus (without bitmaps) the scan of a
// small neighbour bucket or a binary search per beta single of a large one.
__global__ void nb_cost_kernel(SpaceView S, i64 nua, int W, int ds, float* __restrict__ out) {
    const i64 a = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nua) return;
    float c = 1.0f;
    for (u32 t = S.as_ptr[a]; t < S.as_ptr[a + 1]; ++t) {
        const u32 a2 = S.as_idx[t];
        const u32 len = S.aoff[a2 + 1] - S.aoff[a2];
        if (W > 0) c += 1.0f;
        else if (len <= NB_SCAN * (u32)ds) c += 1.0f + (float)len / HCI_WAVE;
        else c += 1.0f + (float)ds / HCI_WAVE * (float)(32 - __clz(len));
    }
    out[a] = c;
}

// beta-major copies: out[k] = in[permb[k]]
template <class T>
__global__ void rdm_permute_kernel(const T* __restrict__ in, const u32* __restrict__ permb, i64 N,
                                   T* __restrict__ out) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < N) out[k] = in[permb[k]];
}

__global__ void rdm_zero_kernel(double* __restrict__ x, i64 m) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (i64)gridDim.x * blockDim.x) x[i] = 0.0;
}

// out[e] = sum over the P private copies of entry e, in copy order
__global__ void rdm_sum_copies_kernel(const double* __restrict__ priv, int P, i64 stride, i64 m,
                                      double* __restrict__ out) {
    const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += priv[(i64)p * stride + e];
    out[e] = s;
}

// LDS layout of rdm_nb_kernel within `budget` bytes, with W bitmap words per
// neighbour (0: scan the neighbour buckets).  Groups should keep every
// wavefront busy (G >= RDM_WAVES): tiles stay in LDS only when that holds,
// else they go straight into the private copy (each entry still has one
// owner, the neighbour's wavefront).  False when W > 0 and no group of
// RDM_WAVES bitmaps fits (the caller retries with W = 0).
bool nb_plan(int n, int na, int nb, int budget, int W, NbPlan& P) {
    const int gmax = std::max(1, na * (n - na));  // alpha singles of a string
    const int ds = std::max(1, nb * (n - nb));    // beta singles of a string
    const int nn = n * n;
    P.n = n;
    P.W = W;
    P.ds = ds;
    P.R = std::max(1, std::min<int>(RDM_CHUNK, 16384 / (8 * ds)));
    const int fixed_sing = 8 * P.R * ds;
    const int fixed_rows = 16 * P.R;
    for (int tile = 1; tile >= 0; --tile) {
        const int per = (tile ? 8 * nn : 0) + 6 * W + 24;
        const int room = budget - fixed_sing - fixed_rows - 64;
        int G = room / per;
        if (G < RDM_WAVES && !(tile == 0 && W == 0)) continue;
        if (G < 1) return false;
        G = std::min(G, gmax);
        P.G = G;
        P.tile = tile != 0;
        int off = P.tile ? 8 * G * nn : 0;
        P.o_sing = off;
        off += fixed_sing;
        P.o_row = off;
        off += fixed_rows;
        P.o_nb = off;
        off += 12 * G + 8 + 8 * G;
        off = (off + 15) & ~15;
        P.o_bm = off;
        off += (6 * G * W + 15) & ~15;
        P.bytes = off;
        return P.bytes <= budget;
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

namespace {
// Row chunks of the buckets (off: nbuck + 1 offsets) assigned to P
// workgroups: largest estimated cost first, each to the least loaded
// workgroup (ties: lowest index), so the assignment depends only on the
// space.  cost(bucket, rows) estimates a chunk's time.
template <class Cost>
void plan_chunks(const u32* off, i64 nbuck, int P, Cost cost, std::vector<u32>& list, std::vector<u32>& wptr) {
    struct Ch {
        u32 b, r0, r1;
        double cost;
    };
    std::vector<Ch> ch;
    for (i64 b = 0; b < nbuck; ++b)
        for (u32 r0 = off[b]; r0 < off[b + 1]; r0 += RDM_CHUNK) {
            const u32 r1 = std::min(r0 + RDM_CHUNK, off[b + 1]);
            ch.push_back({(u32)b, r0, r1, cost((u32)b, off[b + 1] - off[b], r1 - r0)});
        }
    std::vector<u32> order(ch.size());
    for (size_t i = 0; i < ch.size(); ++i) order[i] = (u32)i;
    std::stable_sort(order.begin(), order.end(), [&](u32 x, u32 y) { return ch[x].cost > ch[y].cost; });
    using Load = std::pair<double, int>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int p = 0; p < P; ++p) heap.push({0.0, p});
    std::vector<u32> owner(ch.size());
    std::vector<u32> count(P, 0);
    for (u32 i : order) {
        Load l = heap.top();
        heap.pop();
        owner[i] = (u32)l.second;
        ++count[l.second];
        l.first += ch[i].cost;
        heap.push(l);
    }
    // workgroup p's chunks in the order it received them
    wptr.assign(P + 1, 0);
    for (int p = 0; p < P; ++p) wptr[p + 1] = wptr[p] + count[p];
    std::vector<u32> cur(wptr.begin(), wptr.end() - 1);
    list.assign(3 * ch.size(), 0);
    for (u32 i : order) {
        const u32 at = cur[owner[i]]++;
        list[3 * at] = ch[i].b;
        list[3 * at + 1] = ch[i].r0;
        list[3 * at + 2] = ch[i].r1;
    }
}
}  // namespace

void rdm_compute(hci_ctx_s* ctx, Space* sp, const double* bra, const double* ket, double* rdm1,
                 double* rdm2, hipStream_t s) {
    const int n = ctx->n;
    const i64 N = sp->N;
    const i64 n2 = (i64)n * n, n4 = n2 * n2;
    SpaceView S = space_view(*sp, n);
    int dev = 0, max_shared = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&max_shared, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int budget = std::min(79 * 1024, max_shared);  // two workgroups per CU
    // same-string kernel: rows (16 B each), S2, S3 when it fits; for small n the
    // table of doubles too (then one workgroup per CU, half the rows staged)
    const int np2 = n * (n - 1) / 2;
    const int dx_bytes = 8 * (int)RDM_CHUNK + 8 * (int)(n2 + n2 * n) + 8 * np2 * np2 + ((2 * np2 + 15) & ~15);
    const bool dx = dx_bytes <= max_shared;
    const int same_base = 16 * (int)RDM_CHUNK + 8 * (int)n2;
    const bool s3 = dx || same_base + 8 * (int)(n2 * n) <= budget;
    HCI_REQUIRE(same_base <= budget, HCI_E_UNSUPPORTED, "density matrices: no on-chip plan fits this orbital count");
    const int same_bytes = dx ? dx_bytes : same_base + (s3 ? 8 * (int)(n2 * n) : 0);
    const char* force_search = std::getenv("HCI_AB_SEARCH");  // "1": always search (tests)
    const int W = sp->nub <= 65535 && !(force_search && force_search[0] == '1') ? (int)ceil_div(sp->nub, 32) : 0;
    NbPlan P;
    const bool planned = (W > 0 && nb_plan(n, ctx->na, ctx->nb, budget, W, P)) ||
                         nb_plan(n, ctx->na, ctx->nb, budget, 0, P);
    HCI_REQUIRE(planned, HCI_E_UNSUPPORTED, "density matrices: no on-chip plan fits this orbital count");
    // private copies of T and rdm1, one per workgroup of the persistent grids:
    // two workgroups per CU, within 8 GiB of copies
    int cus = 0;
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const i64 stride = n4 + n2;
    const i64 by_mem = std::max<i64>(1, ((i64)8 << 30) / (stride * (i64)sizeof(double)));
    const int Pw = (int)std::max<i64>(1, std::min<i64>({(i64)2 * cus, by_mem, N}));
    // the same-string kernel with the table of doubles holds a CU alone: as many
    // workgroups as CUs, each with a longer list
    const int Ps = dx ? std::min(Pw, cus) : Pw;
    if (sp->rdm_sa.P != Ps || sp->rdm_nb.P != Pw || sp->rdm_nb.key != (P.W > 0)) {
        // bucket offsets and the alpha single x beta single cost per bucket
        // in one read-back through pinned memory
        const i64 nua = sp->nua, nub = sp->nub;
        DevMem bc = dev_alloc(ctx, sizeof(float) * nua, s);
        HCI_LAUNCH(ctx, "rdm_plan", s, nb_cost_kernel, ceil_div(nua, 256), 256, 0, S, nua, P.W, P.ds,
                   bc.as<float>());
        u32* hs = static_cast<u32*>(host_staging(ctx, sizeof(u32) * (size_t)(2 * nua + nub + 2)));
        HIP_CHECK(hipMemcpyAsync(hs, sp->aoff.ptr, sizeof(u32) * (nua + 1), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(hs + nua + 1, sp->boff.ptr, sizeof(u32) * (nub + 1), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(hs + nua + nub + 2, bc.ptr, sizeof(float) * nua, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        const std::vector<u32> aoff(hs, hs + nua + 1), boff(hs + nua + 1, hs + nua + nub + 2);
        std::vector<float> bcost(nua);
        std::memcpy(bcost.data(), hs + nua + nub + 2, sizeof(float) * nua);
        // a row of a same-string chunk costs a barrier per piece of its bucket
        // (and a chunk about two rows for its flush); an alpha single x beta
        // single chunk one pass per alpha neighbour
        const u32 piece = SS_PIECE;
        auto same_cost = [&](u32, u32 size, u32 rows) { return (double)rows * (double)ceil_div(size, piece) + 2.0; };
        auto nb_cost = [&](u32 b, u32, u32 rows) { return (double)rows * (double)bcost[b]; };
        std::vector<u32> list[3], wptr[3];
        plan_chunks(aoff.data(), nua, Ps, same_cost, list[0], wptr[0]);
        plan_chunks(boff.data(), nub, Ps, same_cost, list[1], wptr[1]);
        plan_chunks(aoff.data(), nua, Pw, nb_cost, list[2], wptr[2]);
        // all three plans up through the staging area, one wait
        size_t words = 0;
        for (int q = 0; q < 3; ++q) words += list[q].size() + wptr[q].size();
        u32* up = static_cast<u32*>(host_staging(ctx, sizeof(u32) * words));
        RdmChunks* dst[3] = {&sp->rdm_sa, &sp->rdm_sb, &sp->rdm_nb};
        const int Pq[3] = {Ps, Ps, Pw};
        size_t at = 0;
        for (int q = 0; q < 3; ++q) {
            RdmChunks& C = *dst[q];
            C.list = dev_alloc(ctx, sizeof(u32) * std::max<size_t>(list[q].size(), 3), s);
            C.wptr = dev_alloc(ctx, sizeof(u32) * wptr[q].size(), s);
            std::memcpy(up + at, list[q].data(), sizeof(u32) * list[q].size());
            HIP_CHECK(hipMemcpyAsync(C.list.ptr, up + at, sizeof(u32) * list[q].size(), hipMemcpyHostToDevice, s));
            at += list[q].size();
            std::memcpy(up + at, wptr[q].data(), sizeof(u32) * wptr[q].size());
            HIP_CHECK(hipMemcpyAsync(C.wptr.ptr, up + at, sizeof(u32) * wptr[q].size(), hipMemcpyHostToDevice, s));
            at += wptr[q].size();
            C.P = Pq[q];
        }
        HIP_CHECK(hipStreamSynchronize(s));  // the staging area is free again
        sp->rdm_nb.key = P.W > 0;
    }
    ensure_alpha_b(ctx, sp, s);
    DevMem ket_b = dev_alloc(ctx, sizeof(double) * N, s), bra_b = dev_alloc(ctx, sizeof(double) * N, s);
    HCI_LAUNCH(ctx, "rdm_permute", s, rdm_permute_kernel<double>, ceil_div(N, 256), 256, 0, ket, sp->permb.as<u32>(),
               N, ket_b.as<double>());
    HCI_LAUNCH(ctx, "rdm_permute", s, rdm_permute_kernel<double>, ceil_div(N, 256), 256, 0, bra, sp->permb.as<u32>(),
               N, bra_b.as<double>());
    DevMem priv = dev_alloc(ctx, sizeof(double) * Pw * stride, s);
    HCI_LAUNCH(ctx, "rdm_zero", s, rdm_zero_kernel, std::min<i64>(ceil_div(Pw * stride, 256), 65536), 256, 0,
               priv.as<double>(), Pw * stride);
    auto same = dx ? rdm_same_kernel<true, true> : s3 ? rdm_same_kernel<true, false> : rdm_same_kernel<false, false>;
    HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(same), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  same_bytes));
    // same alpha string (beta singles and doubles), then same beta string in beta-major order
    SameArgs ga{n, sp->rdm_sa.list.as<u32>(), sp->rdm_sa.wptr.as<u32>(), sp->aoff.as<u32>(), sp->ua.as<u64>(),
                sp->beta.as<u64>(), bra, ket, priv.as<double>(), stride};
    SameArgs gb{n, sp->rdm_sb.list.as<u32>(), sp->rdm_sb.wptr.as<u32>(), sp->boff.as<u32>(), sp->ub.as<u64>(),
                sp->alpha_b.as<u64>(), bra_b.as<double>(), ket_b.as<double>(), priv.as<double>(), stride};
    HCI_LAUNCH(ctx, "rdm_same", s, same, Ps, RDM_BLOCK, (size_t)same_bytes, ga);
    HCI_LAUNCH(ctx, "rdm_same", s, same, Ps, RDM_BLOCK, (size_t)same_bytes, gb);
    // alpha single x beta single
    auto nbk = P.W ? (P.tile ? rdm_nb_kernel<true, true> : rdm_nb_kernel<true, false>)
                   : (P.tile ? rdm_nb_kernel<false, true> : rdm_nb_kernel<false, false>);
    HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(nbk), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  P.bytes));
    HCI_LAUNCH(ctx, "rdm_nb", s, nbk, Pw, RDM_BLOCK, (size_t)P.bytes, S, P, sp->rdm_nb.list.as<u32>(),
               sp->rdm_nb.wptr.as<u32>(), bra, ket, priv.as<double>(), stride);
    HCI_LAUNCH(ctx, "rdm_sum", s, rdm_sum_copies_kernel, ceil_div(n2, 256), 256, 0, priv.as<double>() + n4, (int)Pw,
               stride, n2, rdm1);
    if (rdm2) {
        HCI_LAUNCH(ctx, "rdm_sum", s, rdm_sum_copies_kernel, ceil_div(n4, 256), 256, 0, priv.as<double>(), (int)Pw,
                   stride, n4, rdm2);
        // the off-diagonal passes accumulate one entry of each (pq|rs), (rs|pq) pair
        HCI_LAUNCH(ctx, "rdm_swap_sym", s, swap_sym_kernel, ceil_div(n4, 256), 256, 0, rdm2, n);
    }
    rdm_add_diag(ctx, sp->alpha.as<u64>(), sp->beta.as<u64>(), bra, ket, N, rdm1, rdm2, s);
}

void pair_rdm_init(hci_ctx_s* ctx, PairRdm& A, hipStream_t s) {
    const i64 n = ctx->n, n4 = n * n * n * n;
    A.dtab = dev_alloc(ctx, sizeof(double) * 3 * n4, s);
    A.stab = dev_alloc(ctx, sizeof(double) * 2 * n * n * (2 * n + 1), s);
    HCI_LAUNCH(ctx, "rdm_zero", s, rdm_zero_kernel, std::min<i64>(ceil_div(3 * n4, 256), 65536), 256, 0,
               A.dtab.as<double>(), 3 * n4);
    HCI_LAUNCH(ctx, "rdm_zero", s, rdm_zero_kernel, ceil_div(2 * n * n * (2 * n + 1), 256), 256, 0,
               A.stab.as<double>(), 2 * n * n * (2 * n + 1));
}

void pair_rdm_add(hci_ctx_s* ctx, PairRdm& A, const u64* a_hi, const u64* a_lo, const u32* idx, const double* wa,
                  i64 M, const u64* dets, const double* c, hipStream_t s) {
    if (M <= 0) return;
    HCI_REQUIRE(M < ((i64)1 << 32), HCI_E_UNSUPPORTED, "pt2 pairs: more than 2^32 pairs in one pass");
    DevMem keyed = dev_alloc(ctx, sizeof(u64) * M, s);
    HCI_LAUNCH(ctx, "rdm_pair_keys", s, pair_keys_kernel, ceil_div(M, 256), 256, 0, a_hi, a_lo, idx, wa, dets, c,
               M, keyed.as<u64>());
    {
        DevMem tmp = dev_alloc(ctx, sizeof(u64) * M, s);
        radix_sort64_bytes(ctx, keyed.as<u64>(), tmp.as<u64>(), M, 4, 8, s);  // by the key, bits 32..63
    }
    DevMem flags = dev_alloc(ctx, sizeof(u32) * (M + 1), s), pos = dev_alloc(ctx, sizeof(u32) * (M + 1), s);
    HCI_LAUNCH(ctx, "rdm_pair_heads", s, pair_heads_kernel, ceil_div(M, 256), 256, 0, keyed.as<u64>(), M,
               flags.as<u32>());
    HIP_CHECK(hipMemsetAsync(flags.as<u32>() + M, 0, sizeof(u32), s));
    scan_u32_to_u32(ctx, flags.as<u32>(), pos.as<u32>(), M + 1, s);
    const i64 nseg = read_scalar(pos.as<u32>() + M, s);
    DevMem start = dev_alloc(ctx, sizeof(i64) * nseg, s);
    HCI_LAUNCH(ctx, "rdm_pair_starts", s, pair_starts_kernel, ceil_div(M, 256), 256, 0, flags.as<u32>(),
               pos.as<u32>(), M, start.as<i64>());
    const i64 blocks = std::min<i64>(ceil_div(nseg, 4), 16384);
    HCI_LAUNCH(ctx, "rdm_pair_segments", s, pair_segments_kernel, blocks, 256, 0, keyed.as<u64>(),
               start.as<i64>(), nseg, M, a_hi, a_lo, idx, wa, dets, c, ctx->n, A.dtab.as<double>(),
               A.stab.as<double>());
}

void pair_rdm_finish(hci_ctx_s* ctx, PairRdm& A, double* rdm1, double* rdm2, hipStream_t s) {
    const i64 n = ctx->n, n2 = n * n, n4 = n2 * n2;
    HCI_LAUNCH(ctx, "rdm_pair_tables", s, pair_table_kernel, ceil_div(n4 + n2, 256), 256, 0, A.dtab.as<double>(),
               A.stab.as<double>(), (int)n, rdm1, rdm2);
}
