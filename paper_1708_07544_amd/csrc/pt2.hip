// eps2-screened second-order pieces on a frozen V, c, E0 (Sec. "Perturbative
// stage"): the Epstein-Nesbet partition (eq. h0), the screened sum of
// eq. pt_hci and the Hylleraas minimiser d_a = N_a / (E0 - H_aa).
//
//   pairs  M = {(i, a): D_a outside V, one excitation from D_i,
//               fl(|H_ai| |c_i|) > eps2}            (heat-bath walk at eps2)
//   N_a  = sum_{i:(i,a) in M} H_ai c_i,  E2 = sum_a N_a d_a,
//   r_i  = dE2/dc_i at fixed E0 = 2 sum_{a:(i,a) in M} H_ai d_a.
//
// The pairs are produced in i order (count pass, scan, fill pass), then
// stably radix-sorted by a: every N_a is summed in ascending i, and r is
// summed back in the original i order, so all sums have a fixed order.
#include "hashset.h"
#include "walk.h"

using namespace hset;

namespace {

constexpr int PT_BLOCK = 256;
constexpr int PT_ROWS = PT_BLOCK / HCI_WAVE;

__global__ void pt_fill_u64(u64* __restrict__ t, i64 n, u64 v) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) t[i] = v;
}

__global__ void pt_insert_v(HashSet H, const u64* __restrict__ dets, i64 N) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    u64 key;
    bool fresh;
    if (!det_key(H, dets[2 * i], dets[2 * i + 1], key) || hash_insert(H.det, H.det_mask, key, fresh) < 0)
        atomicOr(H.overflow, 1ull);
}

// Pass of a connected determinant when the pairs are taken in nparts passes
// (hash partition of D_a; nparts = 1: a single pass).
__device__ __forceinline__ bool pt_in_part(u64 aa, u64 ab, u32 nparts, u32 part) {
    if (nparts <= 1) return true;
    u64 x = (aa * 0x9E3779B97F4A7C15ull) ^ ((ab + 0x632BE59BD9B4E019ull) * 0xC2B2AE3D27D4EB4Full);
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    return (u32)(x >> 32) % nparts == part;
}

struct CountHits {
    const HashSet* H;
    u32 nparts, part;
    u32 cnt = 0;
    __device__ __forceinline__ void operator()(bool ok, u64 aa, u64 ab) {
        const bool hit = ok && pt_in_part(aa, ab, nparts, part) && !det_contains(*H, aa, ab);
        cnt += (u32)__popcll(ballot(hit));
    }
};

struct FillHits {
    const HashSet* H;
    const IntView* I;
    u32 nparts, part;
    u64 ai, bi;
    u32 row;
    i64 pos;
    u64* a_hi;
    u64* a_lo;
    u32* idx;
    double* hai;
    __device__ __forceinline__ void operator()(bool ok, u64 aa, u64 ab) {
        const bool hit = ok && pt_in_part(aa, ab, nparts, part) && !det_contains(*H, aa, ab);
        const u64 m = ballot(hit);
        if (hit) {
            const i64 at = pos + rank_in(m);
            a_hi[at] = aa;
            a_lo[at] = ab;
            idx[at] = row;
            hai[at] = hij_f64(*I, ai, bi, aa, ab);
        }
        pos += __popcll(m);
    }
};

__global__ void __launch_bounds__(PT_BLOCK) pt_count_kernel(HBView T, IntView I, HashSet H,
                                                            const u64* __restrict__ dets,
                                                            const double* __restrict__ c, i64 N,
                                                            double eps, double hb_max, u32 nparts,
                                                            u32 part, u32* __restrict__ counts) {
    const i64 i = (i64)blockIdx.x * PT_ROWS + threadIdx.x / HCI_WAVE;
    if (i >= N) return;
    const double ci = fabs(c[i]);
    CountHits v{&H, nparts, part};
    if (hb_max * ci > eps) heat_bath_walk(T, I, dets[2 * i], dets[2 * i + 1], ci, eps, v);
    if (lane_id() == 0) counts[i] = v.cnt;
}

__global__ void __launch_bounds__(PT_BLOCK) pt_fill_kernel(HBView T, IntView I, HashSet H,
                                                           const u64* __restrict__ dets,
                                                           const double* __restrict__ c, i64 N,
                                                           double eps, double hb_max, u32 nparts,
                                                           u32 part, const i64* __restrict__ off,
                                                           u64* __restrict__ a_hi,
                                                           u64* __restrict__ a_lo,
                                                           u32* __restrict__ idx,
                                                           double* __restrict__ hai,
                                                           unsigned long long* __restrict__ bad) {
    const i64 i = (i64)blockIdx.x * PT_ROWS + threadIdx.x / HCI_WAVE;
    if (i >= N) return;
    const double ci = fabs(c[i]);
    const u64 A = dets[2 * i], B = dets[2 * i + 1];
    FillHits v{&H, &I, nparts, part, A, B, (u32)i, off[i], a_hi, a_lo, idx, hai};
    if (hb_max * ci > eps) heat_bath_walk(T, I, A, B, ci, eps, v);
    if (lane_id() == 0 && v.pos != off[i + 1]) atomicAdd(bad, 1ull);
}

// H_ai of stored pairs with the current integrals
__global__ void pair_elems(IntView I, const u64* __restrict__ dets, const u32* __restrict__ idx,
                           const u64* __restrict__ a_hi, const u64* __restrict__ a_lo, i64 M,
                           double* __restrict__ hai) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    const i64 i = idx[t];
    hai[t] = hij_f64(I, dets[2 * i], dets[2 * i + 1], a_hi[t], a_lo[t]);
}

__global__ void iota_u32(u32* __restrict__ x, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (u32)i;
}

__global__ void seg_flags(const u64* __restrict__ hi, const u64* __restrict__ lo, i64 n,
                          u32* __restrict__ flags) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = (i == 0 || hi[i] != hi[i - 1] || lo[i] != lo[i - 1]) ? 1u : 0u;
}

__global__ void seg_starts(const u32* __restrict__ flags, const u32* __restrict__ excl, i64 n,
                           i64* __restrict__ start, const u64* __restrict__ hi,
                           const u64* __restrict__ lo, u64* __restrict__ ca, u64* __restrict__ cb) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flags[i]) {
        const u32 s = excl[i];
        start[s] = i;
        ca[s] = hi[i];
        cb[s] = lo[i];
    }
}

// One thread per connected determinant a: N_a over its pairs in ascending
// i, H_aa, d_a, the E2 term, and d_a copied back to every pair.
__global__ void seg_reduce(IntView I, const i64* __restrict__ start, i64 nseg, i64 M,
                           const u32* __restrict__ perm, const double* __restrict__ hai,
                           const u32* __restrict__ idx, const double* __restrict__ c,
                           const u64* __restrict__ ca, const u64* __restrict__ cb, double e0,
                           double* __restrict__ d, double* __restrict__ term,
                           double* __restrict__ dpair) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const i64 t0 = start[s], t1 = s + 1 < nseg ? start[s + 1] : M;
    double na = 0.0;
    for (i64 t = t0; t < t1; ++t) {
        const u32 p = perm[t];
        na += hai[p] * c[idx[p]];
    }
    const double haa = diag_f64(I, ca[s], cb[s]);
    const double da = na / (e0 - haa);
    d[s] = da;
    term[s] = na * da;
    for (i64 t = t0; t < t1; ++t) dpair[perm[t]] = da;
}

// r_i = 2 sum over the pairs of row i (contiguous, i order) of H_ai d_a
// (ADD: added to r, one pass of several)
template <bool ADD>
__global__ void r_rows(const i64* __restrict__ off, i64 N, const double* __restrict__ hai,
                       const double* __restrict__ dpair, double* __restrict__ r) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (i64 t = off[i]; t < off[i + 1]; ++t) acc += hai[t] * dpair[t];
    if constexpr (ADD) r[i] += 2.0 * acc;
    else r[i] = 2.0 * acc;
}

// ---------------------------------------------------------- sampled estimate
// Integer draw weights q_i = max(1, round(2^31 |c_i| / max|c|)) for c_i != 0
// (0 otherwise): their prefix sums are exact in any order.
__global__ void abs_max_bits(const double* __restrict__ c, i64 N, unsigned long long* __restrict__ out) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    // |x| as bits is monotone in |x| for finite doubles
    u64 v = i < N ? (u64)__double_as_longlong(fabs(c[i])) : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const u64 o = (u64)__shfl_xor((long long)v, off, HCI_WAVE);
        v = o > v ? o : v;
    }
    if (lane_id() == 0 && v) atomicMax(out, (unsigned long long)v);
}

__global__ void draw_weights(const double* __restrict__ c, i64 N, const unsigned long long* __restrict__ cmax_bits,
                             u32* __restrict__ q) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    if (i == N) {
        q[N] = 0u;
        return;
    }
    const double cmax = __longlong_as_double((long long)*cmax_bits);
    const double a = fabs(c[i]);
    u32 v = 0u;
    if (a > 0.0) {
        const double x = floor(ldexp(a / cmax, 31) + 0.5);
        v = x < 1.0 ? 1u : (u32)x;
    }
    q[i] = v;
}

// Draw k picks the row whose cumulative weight range holds
// min(Q - 1, floor(u_k Q)); multiplicities by integer atomics.
__global__ void draw_rows(const double* __restrict__ u, i64 nd, const i64* __restrict__ qex, i64 N,
                          u32* __restrict__ w, unsigned long long* __restrict__ bad) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nd) return;
    const double uk = u[k];
    if (!(uk >= 0.0 && uk < 1.0)) {
        atomicAdd(bad, 1ull);
        return;
    }
    const i64 Q = qex[N];
    i64 t = (i64)floor(uk * (double)Q);
    if (t > Q - 1) t = Q - 1;
    // last row with qex[row] <= t
    i64 lo = 0, hi = N - 1;
    while (lo < hi) {
        const i64 mid = (lo + hi + 1) >> 1;
        if (qex[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    atomicAdd(&w[lo], 1u);
}

__global__ void drawn_flags(const u32* __restrict__ w, i64 N, u32* __restrict__ f) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) f[i] = w[i] > 0u ? 1u : 0u;
    if (i == N) f[N] = 0u;
}

// Compact the drawn rows (ascending): determinants, coefficients and the
// weight w_i / p_i with p_i = q_i / Q.
__global__ void drawn_gather(const u32* __restrict__ w, const u32* __restrict__ q, const i64* __restrict__ qex,
                             const u32* __restrict__ ex, i64 N, const u64* __restrict__ dets,
                             const double* __restrict__ c, u64* __restrict__ sdets, double* __restrict__ sc,
                             double* __restrict__ swp) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || w[i] == 0u) return;
    const u32 k = ex[i];
    sdets[2 * (i64)k] = dets[2 * i];
    sdets[2 * (i64)k + 1] = dets[2 * i + 1];
    sc[k] = c[i];
    const double p = (double)q[i] / (double)qex[N];
    swp[k] = (double)w[i] / p;
}

// One thread per connected determinant a: the estimator sums over its pairs
// (ascending drawn row), x = H_ai c_i, at eps2 (all pairs) and at eps2_d
// (pairs with fl(|H_ai| |c_i|) > eps2_d):
//   T_a = [S1^2 - S2 + (nd - 1) S3] / (nd (nd - 1)),
//   S1 = sum w x / p, S2 = sum (w x / p)^2, S3 = sum w x^2 / p,
// term = T_a / (E0 - H_aa).
__global__ void stoch_reduce(IntView I, const i64* __restrict__ start, i64 nseg, i64 M,
                             const u32* __restrict__ perm, const double* __restrict__ hai,
                             const u32* __restrict__ idx, const double* __restrict__ sc,
                             const double* __restrict__ swp, const u64* __restrict__ ca,
                             const u64* __restrict__ cb, double e0, double eps_d, double nd,
                             double* __restrict__ term, double* __restrict__ term_d) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const i64 t0 = start[s], t1 = s + 1 < nseg ? start[s + 1] : M;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
    for (i64 t = t0; t < t1; ++t) {
        const u32 pr = perm[t];
        const u32 k = idx[pr];
        const double h = hai[pr], ck = sc[k];
        const double x = h * ck;
        const double wx = swp[k] * x;
        s1 += wx;
        s2 += wx * wx;
        s3 += wx * x;
        if (fabs(h) * fabs(ck) > eps_d) {
            d1 += wx;
            d2 += wx * wx;
            d3 += wx * x;
        }
    }
    const double den = e0 - diag_f64(I, ca[s], cb[s]);
    const double norm = nd * (nd - 1.0);
    term[s] = ((s1 * s1 - s2 + (nd - 1.0) * s3) / norm) / den;
    term_d[s] = ((d1 * d1 - d2 + (nd - 1.0) * d3) / norm) / den;
}

__global__ void sum_fixed(const double* __restrict__ x, i64 n, double* __restrict__ out) {
    // one block, fixed-order: strided partials then a tree
    __shared__ double red[256];
    double acc = 0.0;
    for (i64 k = threadIdx.x; k < n; k += 256) acc += x[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// First level of a fixed-order sum: block b adds x[k] for k = b*256 + t + j*nb*256
// (strided per thread, then a tree), part[b] = its total.
__global__ void sum_partials(const double* __restrict__ x, i64 n, double* __restrict__ part) {
    __shared__ double red[256];
    const i64 stride = (i64)gridDim.x * 256;
    double acc = 0.0;
    for (i64 k = (i64)blockIdx.x * 256 + threadIdx.x; k < n; k += stride) acc += x[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sq_kernel_pt(const double* __restrict__ d, i64 n, double* __restrict__ out) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = d[i] * d[i];
}

i64 p2(i64 x) {
    i64 p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

namespace {

// Hash set of V for the "outside V" test of the walk.
struct VSet {
    DevMem flags;  // [1] overflow, [2..3] interned alpha / beta strings, [4] fill mismatch
    DevMem table, sa, sb;
    HashSet H;
};

void vset_build(hci_ctx_s* ctx, const u64* dets, i64 N, VSet& v, hipStream_t s) {
    const bool packed = ctx->n <= 31;
    v.flags = dev_alloc(ctx, sizeof(u64) * 5, s);
    unsigned long long* fl = (unsigned long long*)v.flags.as<u64>();
    HIP_CHECK(hipMemsetAsync(v.flags.ptr, 0, sizeof(u64) * 5, s));
    const i64 slots = p2(std::max<i64>(4 * N, 1 << 16));
    v.table = dev_alloc(ctx, sizeof(u64) * slots, s);
    HCI_LAUNCH(ctx, "pt2_fill", s, pt_fill_u64, ceil_div(slots, 256), 256, 0, v.table.as<u64>(), slots,
               EMPTY);
    v.H = HashSet{v.table.as<u64>(), (u64)(slots - 1), nullptr, 0, nullptr, 0, packed ? 1 : 0, fl + 1, fl + 2};
    if (!packed) {
        v.sa = dev_alloc(ctx, sizeof(u64) * slots, s);
        v.sb = dev_alloc(ctx, sizeof(u64) * slots, s);
        HCI_LAUNCH(ctx, "pt2_fill", s, pt_fill_u64, ceil_div(slots, 256), 256, 0, v.sa.as<u64>(), slots,
                   EMPTY);
        HCI_LAUNCH(ctx, "pt2_fill", s, pt_fill_u64, ceil_div(slots, 256), 256, 0, v.sb.as<u64>(), slots,
                   EMPTY);
        v.H.sa = v.sa.as<u64>();
        v.H.sb = v.sb.as<u64>();
        v.H.sa_mask = v.H.sb_mask = (u64)(slots - 1);
    }
    HCI_LAUNCH(ctx, "pt2_insert_v", s, pt_insert_v, ceil_div(N, 256), 256, 0, v.H, dets, N);
    HCI_REQUIRE(read_scalar(v.flags.as<u64>() + 1, s) == 0, HCI_E_NOMEM, "pt2: hash set of V overflowed");
}

// Screened pairs (i, a) of rows [0, N) of `dets` (coefficients c), a outside
// V and in hash partition `part` of `nparts`: count, scan, fill in i order.
struct Pairs {
    DevMem off, a_hi, a_lo, idx, hai;
    i64 M = -1;  // not counted yet
};

i64 count_pairs(hci_ctx_s* ctx, const VSet& v, const u64* dets, const double* c, i64 N, double eps,
                double hbm, u32 nparts, u32 part, DevMem& off, hipStream_t s) {
    HBView T = hb_view(ctx->ints);
    IntView I = int_view(ctx->ints);
    DevMem counts = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    HCI_LAUNCH(ctx, "pt2_count", s, pt_count_kernel, ceil_div(N, PT_ROWS), PT_BLOCK, 0, T, I, v.H, dets, c,
               N, eps, hbm, nparts, part, counts.as<u32>());
    HIP_CHECK(hipMemsetAsync(counts.as<u32>() + N, 0, sizeof(u32), s));
    off = dev_alloc(ctx, sizeof(i64) * (N + 1), s);
    scan_u32_to_i64(ctx, counts.as<u32>(), off.as<i64>(), N + 1, s);
    return read_scalar(off.as<i64>() + N, s);
}

// (P.off and P.M already hold the count of this pass when P.M >= 0 on entry)
void walk_pairs(hci_ctx_s* ctx, const VSet& v, const u64* dets, const double* c, i64 N, double eps,
                double hbm, u32 nparts, u32 part, Pairs& P, hipStream_t s) {
    if (P.M < 0) P.M = count_pairs(ctx, v, dets, c, N, eps, hbm, nparts, part, P.off, s);
    HCI_REQUIRE(P.M < ((i64)1 << 32) - 1, HCI_E_UNSUPPORTED, "pt2: more than 2^32 screened pairs in one pass");
    const i64 Ma = P.M > 0 ? P.M : 1;
    P.a_hi = dev_alloc(ctx, sizeof(u64) * Ma, s);
    P.a_lo = dev_alloc(ctx, sizeof(u64) * Ma, s);
    P.idx = dev_alloc(ctx, sizeof(u32) * Ma, s);
    P.hai = dev_alloc(ctx, sizeof(double) * Ma, s);
    if (P.M == 0) return;
    HBView T = hb_view(ctx->ints);
    IntView I = int_view(ctx->ints);
    unsigned long long* fl = (unsigned long long*)v.flags.as<u64>();
    HCI_LAUNCH(ctx, "pt2_fill_pairs", s, pt_fill_kernel, ceil_div(N, PT_ROWS), PT_BLOCK, 0, T, I, v.H, dets,
               c, N, eps, hbm, nparts, part, P.off.as<i64>(), P.a_hi.as<u64>(), P.a_lo.as<u64>(),
               P.idx.as<u32>(), P.hai.as<double>(), fl + 4);
    HCI_REQUIRE(read_scalar(v.flags.as<u64>() + 4, s) == 0, HCI_E_HIP,
                "internal: pt2 fill disagrees with the count pass");
}

// Stable sort of the pairs by a (payload: pair position) and the segments of
// equal a: start, and the determinant of each.
struct Segs {
    DevMem perm, start, ca, cb;
    i64 nseg = 0;
};

void sort_segments(hci_ctx_s* ctx, const u64* a_hi, const u64* a_lo, i64 M, Segs& G, hipStream_t s) {
    const int n = ctx->n;
    DevMem khi = dev_alloc(ctx, sizeof(u64) * M, s), klo = dev_alloc(ctx, sizeof(u64) * M, s);
    G.perm = dev_alloc(ctx, sizeof(u32) * M, s);
    HIP_CHECK(hipMemcpyAsync(khi.ptr, a_hi, sizeof(u64) * M, hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipMemcpyAsync(klo.ptr, a_lo, sizeof(u64) * M, hipMemcpyDeviceToDevice, s));
    HCI_LAUNCH(ctx, "pt2_iota", s, iota_u32, ceil_div(M, 256), 256, 0, G.perm.as<u32>(), M);
    {
        DevMem thi = dev_alloc(ctx, sizeof(u64) * M, s), tlo = dev_alloc(ctx, sizeof(u64) * M, s);
        DevMem tv = dev_alloc(ctx, sizeof(u32) * M, s);
        radix_sort128(ctx, khi.as<u64>(), klo.as<u64>(), G.perm.as<u32>(), thi.as<u64>(), tlo.as<u64>(),
                      tv.as<u32>(), M, n, n, s);
    }
    DevMem fl2 = dev_alloc(ctx, sizeof(u32) * (M + 1), s), ex = dev_alloc(ctx, sizeof(u32) * (M + 1), s);
    HCI_LAUNCH(ctx, "pt2_segflags", s, seg_flags, ceil_div(M, 256), 256, 0, khi.as<u64>(), klo.as<u64>(),
               M, fl2.as<u32>());
    HIP_CHECK(hipMemsetAsync(fl2.as<u32>() + M, 0, sizeof(u32), s));
    scan_u32_to_u32(ctx, fl2.as<u32>(), ex.as<u32>(), M + 1, s);
    G.nseg = read_scalar(ex.as<u32>() + M, s);
    G.start = dev_alloc(ctx, sizeof(i64) * G.nseg, s);
    G.ca = dev_alloc(ctx, sizeof(u64) * G.nseg, s);
    G.cb = dev_alloc(ctx, sizeof(u64) * G.nseg, s);
    HCI_LAUNCH(ctx, "pt2_segstarts", s, seg_starts, ceil_div(M, 256), 256, 0, fl2.as<u32>(), ex.as<u32>(),
               M, G.start.as<i64>(), khi.as<u64>(), klo.as<u64>(), G.ca.as<u64>(), G.cb.as<u64>());
}

// fixed-order sum of x[0, n): block partials, then one block over them
double sum_to_host(hci_ctx_s* ctx, const double* x, i64 n, hipStream_t s) {
    const i64 nb = std::max<i64>(1, std::min<i64>(1024, ceil_div(n, 256 * 8)));
    DevMem part = dev_alloc(ctx, sizeof(double) * (nb + 1), s);
    HCI_LAUNCH(ctx, "pt2_sum", s, sum_partials, nb, 256, 0, x, n, part.as<double>());
    HCI_LAUNCH(ctx, "pt2_sum", s, sum_fixed, 1, 256, 0, part.as<double>(), nb, part.as<double>() + nb);
    return read_scalar(part.as<double>() + nb, s);
}

}  // namespace

namespace {

// One pass of the screened pairs: the pairs (i, a) with D_a in hash
// partition `part` of `nparts`, sorted into segments of equal a, with the
// first-order amplitudes d_a of the segments and their copy on every pair.
struct Pt2Pass {
    Pairs P;
    Segs G;
    DevMem d, term, dpair;
};

// Run the screened pairs in passes over hash partitions of D_a sized to the
// pt2 memory budget: a count pass over all rows comes first (it allocates
// only the row offsets), so the number of passes is fixed before any pair
// is stored.  `each(Pt2Pass&)` sees every nonempty pass in order; the
// passes' sums are added in that order (fixed).
template <class F>
void pt2_passes(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, double e0, double eps2,
                int* npasses, hipStream_t s, F&& each) {
    const double hbm = heat_bath_max(ctx, s);
    IntView I = int_view(ctx->ints);
    VSet v;
    vset_build(ctx, dets, N, v, s);
    DevMem off_all;
    const i64 Mall = count_pairs(ctx, v, dets, c, N, eps2, hbm, 1, 0, off_all, s);
    const i64 budget = std::max<i64>(ctx->pt2_budget, PT2_BYTES_PER_PAIR);
    const i64 nparts = std::max<i64>(1, ceil_div(Mall * PT2_BYTES_PER_PAIR, budget));
    HCI_REQUIRE(nparts <= 65536, HCI_E_NOMEM, "pt2: more than 65536 passes needed for the memory budget");
    if (nparts > 1) off_all = DevMem();
    if (npasses) *npasses = (int)nparts;
    for (i64 part = 0; part < nparts; ++part) {
        Pt2Pass X;
        if (nparts == 1) {  // the sizing count is this pass's count
            X.P.M = Mall;
            X.P.off = std::move(off_all);
        }
        walk_pairs(ctx, v, dets, c, N, eps2, hbm, (u32)nparts, (u32)part, X.P, s);
        if (X.P.M == 0) continue;
        sort_segments(ctx, X.P.a_hi.as<u64>(), X.P.a_lo.as<u64>(), X.P.M, X.G, s);
        X.d = dev_alloc(ctx, sizeof(double) * X.G.nseg, s);
        X.term = dev_alloc(ctx, sizeof(double) * X.G.nseg, s);
        X.dpair = dev_alloc(ctx, sizeof(double) * X.P.M, s);
        HCI_LAUNCH(ctx, "pt2_reduce", s, seg_reduce, ceil_div(X.G.nseg, 256), 256, 0, I, X.G.start.as<i64>(),
                   X.G.nseg, X.P.M, X.G.perm.as<u32>(), X.P.hai.as<double>(), X.P.idx.as<u32>(), c,
                   X.G.ca.as<u64>(), X.G.cb.as<u64>(), e0, X.d.as<double>(), X.term.as<double>(),
                   X.dpair.as<double>());
        each(X);
    }
}

}  // namespace

// The screened pairs frozen at some integrals: the set M (pairs and their
// segments of equal a) is kept, the elements are recomputed at every use.
struct Pt2Frozen {
    i64 N = 0;
    u64 hash = 0;
    Pairs P;
    Segs G;
};

i64 pt2_freeze(hci_ctx_s* ctx, const u64* dets, i64 N, u64 hash, const double* c, double eps2, hipStream_t s) {
    drop_frozen(ctx);
    auto F = std::make_unique<Pt2Frozen>();
    F->N = N;
    F->hash = hash;
    const double hbm = heat_bath_max(ctx, s);
    VSet v;
    vset_build(ctx, dets, N, v, s);
    F->P.M = count_pairs(ctx, v, dets, c, N, eps2, hbm, 1, 0, F->P.off, s);
    HCI_REQUIRE(F->P.M * PT2_BYTES_PER_PAIR <= std::max<i64>(ctx->pt2_budget, PT2_BYTES_PER_PAIR), HCI_E_NOMEM,
                "pt2: the screened pairs to freeze (" + std::to_string(F->P.M) +
                    ") exceed the pt2 memory budget; a frozen set is held in one pass");
    walk_pairs(ctx, v, dets, c, N, eps2, hbm, 1, 0, F->P, s);
    if (F->P.M > 0) sort_segments(ctx, F->P.a_hi.as<u64>(), F->P.a_lo.as<u64>(), F->P.M, F->G, s);
    const i64 M = F->P.M;
    ctx->frozen = F.release();
    return M;
}

double pt2_frozen_energy(hci_ctx_s* ctx, const u64* dets, i64 N, u64 hash, const double* c, double e0,
                         hipStream_t s) {
    Pt2Frozen* F = ctx->frozen;
    HCI_REQUIRE(F != nullptr, HCI_E_ARG, "no frozen pt2 pair set (call hci_pt2_freeze first)");
    HCI_REQUIRE(F->N == N && F->hash == hash, HCI_E_ARG, "the frozen pt2 pair set belongs to another list");
    const i64 M = F->P.M;
    if (M == 0) return 0.0;
    IntView I = int_view(ctx->ints);
    HCI_LAUNCH(ctx, "pt2_frozen_elems", s, pair_elems, ceil_div(M, 256), 256, 0, I, dets, F->P.idx.as<u32>(),
               F->P.a_hi.as<u64>(), F->P.a_lo.as<u64>(), M, F->P.hai.as<double>());
    const i64 nseg = F->G.nseg;
    DevMem d = dev_alloc(ctx, sizeof(double) * nseg, s), term = dev_alloc(ctx, sizeof(double) * nseg, s);
    DevMem dpair = dev_alloc(ctx, sizeof(double) * M, s);
    HCI_LAUNCH(ctx, "pt2_reduce", s, seg_reduce, ceil_div(nseg, 256), 256, 0, I, F->G.start.as<i64>(), nseg, M,
               F->G.perm.as<u32>(), F->P.hai.as<double>(), F->P.idx.as<u32>(), c, F->G.ca.as<u64>(),
               F->G.cb.as<u64>(), e0, d.as<double>(), term.as<double>(), dpair.as<double>());
    return sum_to_host(ctx, term.as<double>(), nseg, s);
}

void drop_frozen(hci_ctx_s* ctx) {
    delete ctx->frozen;
    ctx->frozen = nullptr;
}

void pt2_relaxed_pieces(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, double e0, double eps2,
                        double* r, double* dc1, double* dc2, double* dd1, double* dd2, double* e2_out,
                        double* dd_out, i64* nconn, int* npasses, hipStream_t s) {
    HIP_CHECK(hipMemsetAsync(r, 0, sizeof(double) * N, s));
    double e2 = 0.0, dd = 0.0;
    i64 nc = 0;
    PairRdm acc;
    pair_rdm_init(ctx, acc, s);
    pt2_passes(ctx, dets, N, c, e0, eps2, npasses, s, [&](Pt2Pass& X) {
        HCI_LAUNCH(ctx, "pt2_r", s, r_rows<true>, ceil_div(N, 256), 256, 0, X.P.off.as<i64>(), N,
                   X.P.hai.as<double>(), X.dpair.as<double>(), r);
        e2 += sum_to_host(ctx, X.term.as<double>(), X.G.nseg, s);
        HCI_LAUNCH(ctx, "pt2_dd_sq", s, sq_kernel_pt, ceil_div(X.G.nseg, 256), 256, 0, X.d.as<double>(),
                   X.G.nseg, X.term.as<double>());
        dd += sum_to_host(ctx, X.term.as<double>(), X.G.nseg, s);
        nc += X.G.nseg;
        // Gamma^{dc}: bra D_a (weight d_a), ket D_i (weight c_i) over the pass's pairs
        pair_rdm_add(ctx, acc, X.P.a_hi.as<u64>(), X.P.a_lo.as<u64>(), X.P.idx.as<u32>(), X.dpair.as<double>(),
                     X.P.M, dets, c, s);
        // Gamma^{dd}: the diagonal of the connected determinants, weights d_a^2
        rdm_add_diag(ctx, X.G.ca.as<u64>(), X.G.cb.as<u64>(), X.d.as<double>(), X.d.as<double>(), X.G.nseg,
                     dd1, dd2, s);
    });
    pair_rdm_finish(ctx, acc, dc1, dc2, s);
    *e2_out = e2;
    *dd_out = dd;
    if (nconn) *nconn = nc;
}

double pt2_energy(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, double e0, double eps2,
                  double* r, i64* nconn, int* npasses, hipStream_t s) {
    if (r) HIP_CHECK(hipMemsetAsync(r, 0, sizeof(double) * N, s));
    double e2 = 0.0;
    i64 nc = 0;
    pt2_passes(ctx, dets, N, c, e0, eps2, npasses, s, [&](Pt2Pass& X) {
        if (r)
            HCI_LAUNCH(ctx, "pt2_r", s, r_rows<true>, ceil_div(N, 256), 256, 0, X.P.off.as<i64>(), N,
                       X.P.hai.as<double>(), X.dpair.as<double>(), r);
        e2 += sum_to_host(ctx, X.term.as<double>(), X.G.nseg, s);
        nc += X.G.nseg;
    });
    if (nconn) *nconn = nc;
    return e2;
}

void pt2_stochastic(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, double e0, double eps2,
                    double eps2_d, const double* u, i64 nd, i64 nb, double* e2s, double* e2sd,
                    hipStream_t s) {
    const double hbm = heat_bath_max(ctx, s);
    IntView I = int_view(ctx->ints);
    VSet v;
    vset_build(ctx, dets, N, v, s);
    // integer draw weights and their exclusive prefix sums
    DevMem cmax = dev_alloc(ctx, sizeof(u64), s);
    HIP_CHECK(hipMemsetAsync(cmax.ptr, 0, sizeof(u64), s));
    HCI_LAUNCH(ctx, "pt2s_weights", s, abs_max_bits, ceil_div(N, 256), 256, 0, c, N,
               (unsigned long long*)cmax.as<u64>());
    HCI_REQUIRE(read_scalar(cmax.as<u64>(), s) != 0, HCI_E_ARG, "pt2: c is zero");
    DevMem q = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    HCI_LAUNCH(ctx, "pt2s_weights", s, draw_weights, ceil_div(N + 1, 256), 256, 0, c, N,
               (const unsigned long long*)cmax.as<u64>(), q.as<u32>());
    DevMem qex = dev_alloc(ctx, sizeof(i64) * (N + 1), s);
    scan_u32_to_i64(ctx, q.as<u32>(), qex.as<i64>(), N + 1, s);
    DevMem w = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    DevMem f = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    DevMem ex = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    DevMem bad = dev_alloc(ctx, sizeof(u64), s);
    for (i64 b = 0; b < nb; ++b) {
        HIP_CHECK(hipMemsetAsync(w.ptr, 0, sizeof(u32) * (N + 1), s));
        HIP_CHECK(hipMemsetAsync(bad.ptr, 0, sizeof(u64), s));
        HCI_LAUNCH(ctx, "pt2s_draw", s, draw_rows, ceil_div(nd, 256), 256, 0, u + b * nd, nd, qex.as<i64>(), N,
                   w.as<u32>(), (unsigned long long*)bad.as<u64>());
        HCI_REQUIRE(read_scalar(bad.as<u64>(), s) == 0, HCI_E_ARG, "pt2: a uniform lies outside [0, 1)");
        HCI_LAUNCH(ctx, "pt2s_draw", s, drawn_flags, ceil_div(N + 1, 256), 256, 0, w.as<u32>(), N, f.as<u32>());
        scan_u32_to_u32(ctx, f.as<u32>(), ex.as<u32>(), N + 1, s);
        const i64 ns = read_scalar(ex.as<u32>() + N, s);
        DevMem sdets = dev_alloc(ctx, sizeof(u64) * 2 * ns, s);
        DevMem sc = dev_alloc(ctx, sizeof(double) * ns, s);
        DevMem swp = dev_alloc(ctx, sizeof(double) * ns, s);
        HCI_LAUNCH(ctx, "pt2s_draw", s, drawn_gather, ceil_div(N, 256), 256, 0, w.as<u32>(), q.as<u32>(),
                   qex.as<i64>(), ex.as<u32>(), N, dets, c, sdets.as<u64>(), sc.as<double>(), swp.as<double>());
        Pairs P;
        walk_pairs(ctx, v, sdets.as<u64>(), sc.as<double>(), ns, eps2, hbm, 1, 0, P, s);
        if (P.M == 0) {
            e2s[b] = 0.0;
            e2sd[b] = 0.0;
            continue;
        }
        Segs G;
        sort_segments(ctx, P.a_hi.as<u64>(), P.a_lo.as<u64>(), P.M, G, s);
        DevMem term = dev_alloc(ctx, sizeof(double) * G.nseg, s);
        DevMem term_d = dev_alloc(ctx, sizeof(double) * G.nseg, s);
        HCI_LAUNCH(ctx, "pt2s_reduce", s, stoch_reduce, ceil_div(G.nseg, 256), 256, 0, I, G.start.as<i64>(),
                   G.nseg, P.M, G.perm.as<u32>(), P.hai.as<double>(), P.idx.as<u32>(), sc.as<double>(),
                   swp.as<double>(), G.ca.as<u64>(), G.cb.as<u64>(), e0, eps2_d, (double)nd, term.as<double>(),
                   term_d.as<double>());
        e2s[b] = sum_to_host(ctx, term.as<double>(), G.nseg, s);
        e2sd[b] = sum_to_host(ctx, term_d.as<double>(), G.nseg, s);
    }
}
