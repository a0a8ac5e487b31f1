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
#include <cstdlib>

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

// ---------------------------------------------------------------- off-diagonal kernel
// Off-diagonal pairs (row i = bra determinant, j = ket determinant) without
// atomics.  A persistent grid of P workgroups: workgroup p takes the chunks
// c = p, p + P, ... (up to RDM_CHUNK rows of one alpha bucket A each) in that
// order and owns a private copy of the output in global memory -- the
// canonical half T of rdm2 (one entry of each (pq|rs), (rs|pq) pair, see
// single_contrib) and rdm1; the P copies are then summed in a fixed order.
// Inside a workgroup every accumulator has one writer at a time:
//   * the chunk's rows are taken one after another for their same-alpha
//     connections (beta single or double: the rows of bucket A) and then
//     their same-beta connections (alpha single or double: the rows of the
//     row's beta bucket), each row's candidates spread over all threads of
//     the workgroup, with a barrier between the two classes and after each
//     row.  One row's contributions of one class fall on distinct entries
//     (distinct excitations), so each thread adds to its own: beta singles
//     into the chunk's LDS sums [u][v] (and [u][v][k] for the same-spin
//     spectators when they fit), alpha singles into one LDS slot per alpha
//     neighbour of A with the beta-occupation moments (when they fit), the
//     rest straight into the private copy;
//   * then the wavefronts own the alpha neighbours A' of A (neighbour q goes
//     to wavefront q mod waves) and accumulate the alpha single x beta single
//     pairs of every row of the chunk with A' in an LDS tile [u2][v2] per
//     neighbour, found through bitmaps of the beta strings present in each
//     neighbour bucket (build_beta_maps) or by scanning the bucket;
//   * the LDS sums reach the private copy class by class, separated by
//     barriers (different classes can share an entry of the spin-traced
//     output).
constexpr int RDM_BLOCK = 1024;
constexpr int RDM_WAVES = RDM_BLOCK / HCI_WAVE;
constexpr u32 RDM_CHUNK = 1024;

struct RdmPlan {
    int n, G;               // G: alpha neighbours per group (bitmaps and tiles rebuilt per group)
    bool tile;              // alpha single x beta single tiles in LDS (else straight into the copy)
    bool s1a, b3;           // alpha-single slots / beta-single spectator block in LDS
    int o_p11, o_s1a, o_s1b2, o_s1b3, total;  // offsets in doubles
    int W;                  // beta-string bitmap words per neighbour (0: scan the buckets)
    int o_bm;               // byte offset of the bitmaps (after the doubles)
    int bytes;              // LDS of the workgroup
};

// position of the k-th set bit (k from 0) of s
__device__ __forceinline__ int select_bit(u64 s, int k) {
    for (int t = 0; t < k; ++t) s &= s - 1;
    return ctz64(s);
}

// non-atomic update of an entry this thread alone writes at this moment
__device__ __forceinline__ void own_add(double* p, double v) { *p += v; }

template <bool BM>
__global__ void __launch_bounds__(RDM_BLOCK) rdm_det_kernel(SpaceView S, RdmPlan P, i64 nua, i64 nchunk,
                                                            const u32* __restrict__ cptr,
                                                            const double* __restrict__ bra,
                                                            const double* __restrict__ ket,
                                                            const u64* __restrict__ alpha_b,
                                                            const double* __restrict__ ket_b,
                                                            double* __restrict__ priv) {
    extern __shared__ double lds[];
    __shared__ u32 sh[3];
    const u32 tid = threadIdx.x;
    const int lane = lane_id();
    const u32 wave = tid / HCI_WAVE;
    const int n = P.n;
    const int nn = n * n;
    const i64 n4 = (i64)nn * nn;
    double* r2 = priv + (i64)blockIdx.x * (n4 + nn);  // this workgroup's copy: T, then rdm1
    double* r1 = r2 + n4;
    double* p11 = lds + P.o_p11;
    double* s1a = lds + P.o_s1a;
    double* s1b2 = lds + P.o_s1b2;
    double* s1b3 = lds + P.o_s1b3;
    u32* bm = reinterpret_cast<u32*>(reinterpret_cast<unsigned char*>(lds) + P.o_bm);
    u16* pre = reinterpret_cast<u16*>(bm + (i64)P.G * P.W);
    for (i64 ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        if (tid == 0) {
            // bucket of this chunk: the last a with cptr[a] <= ch
            u32 lo = 0, hi = (u32)nua - 1u;
            while (lo < hi) {
                const u32 mid = (lo + hi + 1u) >> 1;
                if (cptr[mid] <= (u32)ch) lo = mid;
                else hi = mid - 1u;
            }
            const u32 r0 = S.aoff[lo] + ((u32)ch - cptr[lo]) * RDM_CHUNK;
            sh[0] = lo;
            sh[1] = r0;
            sh[2] = min(r0 + RDM_CHUNK, S.aoff[lo + 1]);
        }
        for (int x = (int)tid; x < P.total; x += RDM_BLOCK) lds[x] = 0.0;
        __syncthreads();
        const u32 a = sh[0], row0 = sh[1], row1 = sh[2];
        const u64 A = S.ua[a];
        const u64 E = ~A & low_mask(n);  // empty alpha orbitals
        const u32 t0 = S.as_ptr[a];
        const u32 deg = S.as_ptr[a + 1] - t0;
        const int nocc = popc64(A), nvir = n - nocc;
        // same-string classes: one row at a time, its candidates spread over
        // the whole workgroup (one row's contributions fall on distinct entries)
        for (u32 row = row0; row < row1; ++row) {
            const double wb = bra[row];
            if (wb == 0.0) continue;  // wave-uniform
            const u64 B = S.beta[row];
            const u32 b = S.ib[row];
            {  // same alpha: beta single or double
                const u32 lo = S.aoff[a], hi = S.aoff[a + 1];
                for (u32 j = lo + tid; j < hi; j += RDM_BLOCK) {
                    const u64 bj = S.beta[j];
                    const double kj = ket[j];
                    const u64 xb = B ^ bj;  // 0 for the row itself
                    const int d = popc64(xb);
                    if (d == 2) {
                        const int v = ctz64(bj & xb), u = ctz64(B & xb);
                        const double x = wb * kj * sign_between(bj, v, u);
                        own_add(&s1b2[u * n + v], x);
                        for (u64 m = B & bj; m; m &= m - 1) {  // same-spin spectators
                            const int k = ctz64(m);
                            if (P.b3) {
                                own_add(&s1b3[(u * n + v) * n + k], x);
                            } else {
                                own_add(&r2[r2idx(n, u, v, k, k)], x);
                                own_add(&r2[r2idx(n, u, k, k, v)], -x);
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
                        const double x = wb * kj * sign_double(bj, v1, u1, v2, u2);
                        own_add(&r2[r2idx(n, u1, v1, u2, v2)], x);
                        own_add(&r2[r2idx(n, u1, v2, u2, v1)], -x);
                    }
                }
            }
            __syncthreads();  // alpha and beta classes can meet on an entry
            {  // same beta: alpha single or double
                const u32 lo = S.boff[b], hi = S.boff[b + 1];
                for (u32 k = lo + tid; k < hi; k += RDM_BLOCK) {
                    // beta-major copies: the candidate's alpha word and ket coefficient
                    const u64 aj = alpha_b[k];
                    const double kj = ket_b[k];
                    const u64 xa = A ^ aj;  // 0 for the row itself
                    const int d = popc64(xa);
                    if (d == 2) {
                        const int v = ctz64(aj & xa), u = ctz64(A & xa);
                        const double x = wb * kj * sign_between(aj, v, u);
                        if (P.s1a) {
                            double* slot = s1a + (i64)(rank_below(A, u) * nvir + rank_below(E, v)) * (1 + n);
                            own_add(&slot[0], x);
                            for (u64 m = B; m; m &= m - 1) own_add(&slot[1 + ctz64(m)], x);
                        } else {
                            own_add(&r1[u * n + v], x);
                            for (u64 m = A & aj; m; m &= m - 1) {  // same-spin spectators
                                const int kk = ctz64(m);
                                own_add(&r2[r2idx(n, u, v, kk, kk)], x);
                                own_add(&r2[r2idx(n, u, kk, kk, v)], -x);
                            }
                            for (u64 m = B; m; m &= m - 1) own_add(&r2[r2idx(n, u, v, ctz64(m), ctz64(m))], x);
                        }
                    } else if (d == 4) {
                        u64 holes = aj & xa, parts = A & xa;
                        const int v1 = ctz64(holes);
                        holes &= holes - 1;
                        const int v2 = ctz64(holes);
                        const int u1 = ctz64(parts);
                        parts &= parts - 1;
                        const int u2 = ctz64(parts);
                        const double x = wb * kj * sign_double(aj, v1, u1, v2, u2);
                        own_add(&r2[r2idx(n, u1, v1, u2, v2)], x);
                        own_add(&r2[r2idx(n, u1, v2, u2, v1)], -x);
                    }
                }
            }
            __syncthreads();  // the next row may add to the same entries
        }
        const u32 ngroups = deg == 0 ? 1u : (deg + (u32)P.G - 1u) / (u32)P.G;
        for (u32 gi = 0; gi < ngroups; ++gi) {
            const u32 tg0 = gi * (u32)P.G;
            const u32 tg1 = min(tg0 + (u32)P.G, deg);
            if constexpr (BM) build_beta_maps<RDM_BLOCK>(S, t0, tg0, tg1, (u32)P.W, bm, pre, tid);
            {
                // alpha single x beta single for the neighbours of this group owned by this wavefront
                for (u32 t = tg0 + wave; t < tg1; t += RDM_WAVES) {
                    const u32 q = t - tg0;
                    const u32 a2 = S.as_idx[t0 + t];
                    const u64 A2 = S.ua[a2];
                    const u64 xa = A ^ A2;
                    const int u1 = ctz64(A & xa), v1 = ctz64(A2 & xa);
                    const double sa = sign_between(A2, v1, u1);
                    // the tile [u2][v2] of this neighbour: in LDS, or its entries of the copy
                    double* tile = P.tile ? p11 + (i64)q * nn : r2 + r2idx(n, u1, v1, 0, 0);
                    const u32 lo2 = S.aoff[a2], hi2 = S.aoff[a2 + 1];
                    for (u32 row = row0; row < row1; ++row) {
                        const double wb = bra[row];
                        if (wb == 0.0) continue;  // wave-uniform
                        const u64 B = S.beta[row];
                        if constexpr (BM) {
                            const u32 b = S.ib[row];
                            const u32 s0 = S.bs_ptr[b], s1 = S.bs_ptr[b + 1];
                            for (u32 base = s0; base < s1; base += HCI_WAVE) {
                                const u32 k = base + lane;
                                if (k >= s1) continue;
                                const u32 bp = S.bs_idx[k];
                                const u32 w = bp >> 5, bit = bp & 31u;
                                const u32 word = bm[q * (u32)P.W + w];
                                if (((word >> bit) & 1u) == 0u) continue;
                                const u64 bj = S.ub[bp];
                                const u64 xb = B ^ bj;
                                const int v2 = ctz64(bj & xb), u2 = ctz64(B & xb);
                                const u32 j = lo2 + (u32)pre[q * (u32)P.W + w] + (u32)__popc(word & ((1u << bit) - 1u));
                                own_add(&tile[u2 * n + v2], wb * ket[j] * sa * sign_between(bj, v2, u2));
                            }
                        } else {
                            for (u32 base = lo2; base < hi2; base += HCI_WAVE) {
                                const u32 j = base + lane;
                                if (j >= hi2) continue;
                                const u64 bj = S.beta[j];
                                const u64 xb = B ^ bj;
                                if (popc64(xb) != 2) continue;
                                const int v2 = ctz64(bj & xb), u2 = ctz64(B & xb);
                                own_add(&tile[u2 * n + v2], wb * ket[j] * sa * sign_between(bj, v2, u2));
                            }
                        }
                    }
                }
            }
            __syncthreads();
            // flush this group's tiles: neighbour q fixes (u1, v1)
            for (int x = (int)tid; P.tile && x < (int)(tg1 - tg0) * nn; x += RDM_BLOCK) {
                const double val = p11[x];
                if (val == 0.0) continue;
                p11[x] = 0.0;
                const u32 t = tg0 + (u32)(x / nn);
                const int u2 = (x % nn) / n, v2 = x % n;
                const u64 A2 = S.ua[S.as_idx[t0 + t]];
                const u64 xa = A ^ A2;
                own_add(&r2[r2idx(n, ctz64(A & xa), ctz64(A2 & xa), u2, v2)], val);
            }
            __syncthreads();
        }
        // alpha singles (slot of the occupied orbital u and the empty orbital v
        // of A): rdm1 and same-spin spectators from the sum, opposite-spin
        // spectators from the beta-occupation moments
        if (P.s1a) {
            for (int q = (int)tid; q < nocc * nvir; q += RDM_BLOCK) {
                const int u = select_bit(A, q / nvir), v = select_bit(E, q % nvir);
                const double* slot = s1a + (i64)q * (1 + n);
                const double X = slot[0];
                if (X != 0.0) {
                    own_add(&r1[u * n + v], X);
                    for (u64 m = A; m; m &= m - 1) {
                        const int k = ctz64(m);
                        if (k == u) continue;
                        own_add(&r2[r2idx(n, u, v, k, k)], X);
                        own_add(&r2[r2idx(n, u, k, k, v)], -X);
                    }
                }
                for (int k = 0; k < n; ++k) {
                    const double Y = slot[1 + k];
                    if (Y != 0.0) own_add(&r2[r2idx(n, u, v, k, k)], Y);
                }
            }
            __syncthreads();
        }
        // beta singles: rdm1 and the alpha spectators from the sum
        for (int x = (int)tid; x < nn; x += RDM_BLOCK) {
            const double X = s1b2[x];
            if (X == 0.0) continue;
            const int u = x / n, v = x % n;
            own_add(&r1[x], X);
            for (u64 m = A; m; m &= m - 1) own_add(&r2[r2idx(n, u, v, ctz64(m), ctz64(m))], X);
        }
        __syncthreads();
        if (P.b3) {
            for (int x = (int)tid; x < nn * n; x += RDM_BLOCK) {
                const double X = s1b3[x];
                if (X == 0.0) continue;
                const int u = x / nn, v = (x / n) % n, k = x % n;
                own_add(&r2[r2idx(n, u, v, k, k)], X);
                own_add(&r2[r2idx(n, u, k, k, v)], -X);
            }
        }
        __syncthreads();
    }
}

__global__ void rdm_nchunk_kernel(const u32* __restrict__ aoff, i64 nua, u32* __restrict__ out) {
    const i64 a = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < nua) out[a] = (aoff[a + 1] - aoff[a] + RDM_CHUNK - 1) / RDM_CHUNK;
    if (a == nua) out[a] = 0;
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

// LDS layout of the kernel for this context within `budget` bytes, with W
// bitmap words per neighbour (0: scan the neighbour buckets).  Neighbour
// groups should keep every wavefront busy (G >= RDM_WAVES): the tiles stay
// in LDS only when they allow that, else they go straight into the private
// copy (each entry still has one owner, the neighbour's wavefront); bitmaps
// only when at least RDM_WAVES of them fit (else the buckets are scanned and
// one group holds every neighbour).  False when W > 0 and the bitmaps do not
// fit (the caller retries with W = 0).
bool rdm_plan(int n, int na, int budget, int W, RdmPlan& P) {
    const int dmax = na * (n - na);
    const int nn = n * n;
    P.n = n;
    P.W = W;
    int want = std::min(RDM_WAVES / 2, std::max(dmax, 1));
    if (const char* e = std::getenv("HCI_RDM_GROUP_MIN")) {  // smallest acceptable group (tuning)
        const int k = std::atoi(e);
        if (k >= 1) want = std::min(k, std::max(dmax, 1));
    }
    auto place = [&](bool tile, bool s1a_lds, bool b3) -> bool {
        const int s1a = s1a_lds ? dmax * (1 + n) : 0;
        const int s1b3 = b3 ? nn * n : 0;
        const int rest = s1a + nn + s1b3;
        const int per = (tile ? 8 * nn : 0) + 6 * W;
        int G = per > 0 ? (budget - 8 * rest) / per : (1 << 20);
        if (G < want) return false;
        if (G > dmax) G = dmax > 0 ? dmax : 1;
        P.G = G;
        P.tile = tile;
        P.s1a = s1a_lds;
        P.b3 = b3;
        P.o_p11 = 0;
        P.o_s1a = tile ? G * nn : 0;
        P.o_s1b2 = P.o_s1a + s1a;
        P.o_s1b3 = P.o_s1b2 + nn;
        P.total = P.o_s1b3 + s1b3;
        P.o_bm = 8 * P.total;
        P.bytes = P.o_bm + ((6 * G * W + 15) & ~15);
        return 8 * rest <= budget;
    };
    for (int tile = 1; tile >= 0; --tile)
        for (int variant = 0; variant < 3; ++variant)
            if (place(tile != 0, variant <= 1, variant == 0)) return true;
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
    const i64 n2 = (i64)n * n, n4 = n2 * n2;
    SpaceView S = space_view(*sp, n);
    int dev = 0, max_shared = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&max_shared, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int budget = std::min(79 * 1024, max_shared);  // two workgroups per CU
    const char* force_search = std::getenv("HCI_AB_SEARCH");  // "1": always search (tests)
    const int W = sp->nub <= 65535 && !(force_search && force_search[0] == '1') ? (int)ceil_div(sp->nub, 32) : 0;
    RdmPlan P;
    const bool planned = (W > 0 && rdm_plan(n, ctx->na, budget, W, P)) || rdm_plan(n, ctx->na, budget, 0, P);
    HCI_REQUIRE(planned, HCI_E_UNSUPPORTED, "density matrices: no on-chip plan fits this orbital count");
    if (!sp->rdm_cptr.ptr) {
        DevMem cnt = dev_alloc(ctx, sizeof(u32) * (sp->nua + 1), s);
        HCI_LAUNCH(ctx, "rdm_nchunk", s, rdm_nchunk_kernel, ceil_div(sp->nua + 1, 256), 256, 0, sp->aoff.as<u32>(),
                   sp->nua, cnt.as<u32>());
        sp->rdm_cptr = dev_alloc(ctx, sizeof(u32) * (sp->nua + 1), s);
        scan_u32_to_u32(ctx, cnt.as<u32>(), sp->rdm_cptr.as<u32>(), sp->nua + 1, s);
        sp->rdm_nchunk = read_scalar(sp->rdm_cptr.as<u32>() + sp->nua, s);
    }
    // private copies of T and rdm1, one per workgroup of the persistent grid:
    // two workgroups per CU, within 8 GiB of copies
    int cus = 0;
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const i64 stride = n4 + n2;
    const i64 by_mem = std::max<i64>(1, ((i64)8 << 30) / (stride * (i64)sizeof(double)));
    const i64 Pw = std::max<i64>(1, std::min<i64>({(i64)2 * cus, by_mem, sp->rdm_nchunk}));
    if (!sp->alpha_b.ptr) {  // alpha word of each beta-major position (cached with the space)
        sp->alpha_b = dev_alloc(ctx, sizeof(u64) * N, s);
        HCI_LAUNCH(ctx, "rdm_permute", s, rdm_permute_kernel<u64>, ceil_div(N, 256), 256, 0, sp->alpha.as<u64>(),
                   sp->permb.as<u32>(), N, sp->alpha_b.as<u64>());
    }
    DevMem ket_b = dev_alloc(ctx, sizeof(double) * N, s);
    HCI_LAUNCH(ctx, "rdm_permute", s, rdm_permute_kernel<double>, ceil_div(N, 256), 256, 0, ket, sp->permb.as<u32>(),
               N, ket_b.as<double>());
    DevMem priv = dev_alloc(ctx, sizeof(double) * Pw * stride, s);
    HCI_LAUNCH(ctx, "rdm_zero", s, rdm_zero_kernel, std::min<i64>(ceil_div(Pw * stride, 256), 65536), 256, 0,
               priv.as<double>(), Pw * stride);
    auto kern = P.W ? rdm_det_kernel<true> : rdm_det_kernel<false>;
    HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  P.bytes));
    HCI_LAUNCH(ctx, "rdm_offdiag", s, kern, Pw, RDM_BLOCK, (size_t)P.bytes, S, P, sp->nua, sp->rdm_nchunk,
               sp->rdm_cptr.as<u32>(), bra, ket, sp->alpha_b.as<u64>(), ket_b.as<double>(), priv.as<double>());
    HCI_LAUNCH(ctx, "rdm_sum", s, rdm_sum_copies_kernel, ceil_div(n2, 256), 256, 0, priv.as<double>() + n4, (int)Pw,
               stride, n2, rdm1);
    if (rdm2) {
        HCI_LAUNCH(ctx, "rdm_sum", s, rdm_sum_copies_kernel, ceil_div(n4, 256), 256, 0, priv.as<double>(), (int)Pw,
                   stride, n4, rdm2);
        // the off-diagonal pass accumulates one entry of each (pq|rs), (rs|pq) pair
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
