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

struct CountHits {
    const HashSet* H;
    u32 cnt = 0;
    __device__ __forceinline__ void operator()(bool ok, u64 aa, u64 ab) {
        const bool hit = ok && !det_contains(*H, aa, ab);
        cnt += (u32)__popcll(ballot(hit));
    }
};

struct FillHits {
    const HashSet* H;
    const IntView* I;
    u64 ai, bi;
    u32 row;
    i64 pos;
    u64* a_hi;
    u64* a_lo;
    u32* idx;
    double* hai;
    __device__ __forceinline__ void operator()(bool ok, u64 aa, u64 ab) {
        const bool hit = ok && !det_contains(*H, aa, ab);
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
                                                            double eps, double hb_max,
                                                            u32* __restrict__ counts) {
    const i64 i = (i64)blockIdx.x * PT_ROWS + threadIdx.x / HCI_WAVE;
    if (i >= N) return;
    const double ci = fabs(c[i]);
    CountHits v{&H};
    if (hb_max * ci > eps) heat_bath_walk(T, I, dets[2 * i], dets[2 * i + 1], ci, eps, v);
    if (lane_id() == 0) counts[i] = v.cnt;
}

__global__ void __launch_bounds__(PT_BLOCK) pt_fill_kernel(HBView T, IntView I, HashSet H,
                                                           const u64* __restrict__ dets,
                                                           const double* __restrict__ c, i64 N,
                                                           double eps, double hb_max,
                                                           const i64* __restrict__ off,
                                                           u64* __restrict__ a_hi,
                                                           u64* __restrict__ a_lo,
                                                           u32* __restrict__ idx,
                                                           double* __restrict__ hai,
                                                           unsigned long long* __restrict__ bad) {
    const i64 i = (i64)blockIdx.x * PT_ROWS + threadIdx.x / HCI_WAVE;
    if (i >= N) return;
    const double ci = fabs(c[i]);
    const u64 A = dets[2 * i], B = dets[2 * i + 1];
    FillHits v{&H, &I, A, B, (u32)i, off[i], a_hi, a_lo, idx, hai};
    if (hb_max * ci > eps) heat_bath_walk(T, I, A, B, ci, eps, v);
    if (lane_id() == 0 && v.pos != off[i + 1]) atomicAdd(bad, 1ull);
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
__global__ void r_rows(const i64* __restrict__ off, i64 N, const double* __restrict__ hai,
                       const double* __restrict__ dpair, double* __restrict__ r) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (i64 t = off[i]; t < off[i + 1]; ++t) acc += hai[t] * dpair[t];
    r[i] = 2.0 * acc;
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

Pt2State::~Pt2State() = default;

std::unique_ptr<Pt2State> pt2_run(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, double e0,
                                  double eps2, hipStream_t s) {
    const int n = ctx->n;
    auto st = std::make_unique<Pt2State>();
    const double hbm = heat_bath_max(ctx, s);
    HBView T = hb_view(ctx->ints);
    IntView I = int_view(ctx->ints);
    // hash set of V for the "outside V" test
    const bool packed = n <= 31;
    // flags: [1] overflow, [2..3] interned alpha / beta strings, [4] fill mismatch
    DevMem flags = dev_alloc(ctx, sizeof(u64) * 5, s);
    unsigned long long* fl = (unsigned long long*)flags.as<u64>();
    HIP_CHECK(hipMemsetAsync(flags.ptr, 0, sizeof(u64) * 5, s));
    const i64 slots = p2(std::max<i64>(4 * N, 1 << 16));
    DevMem table = dev_alloc(ctx, sizeof(u64) * slots, s);
    DevMem sa, sb;
    HCI_LAUNCH(ctx, "pt2_fill", s, pt_fill_u64, ceil_div(slots, 256), 256, 0, table.as<u64>(), slots,
               EMPTY);
    HashSet H{table.as<u64>(), (u64)(slots - 1), nullptr, 0, nullptr, 0, packed ? 1 : 0, fl + 1,
              fl + 2};
    if (!packed) {
        sa = dev_alloc(ctx, sizeof(u64) * slots, s);
        sb = dev_alloc(ctx, sizeof(u64) * slots, s);
        HCI_LAUNCH(ctx, "pt2_fill", s, pt_fill_u64, ceil_div(slots, 256), 256, 0, sa.as<u64>(), slots,
                   EMPTY);
        HCI_LAUNCH(ctx, "pt2_fill", s, pt_fill_u64, ceil_div(slots, 256), 256, 0, sb.as<u64>(), slots,
                   EMPTY);
        H.sa = sa.as<u64>();
        H.sb = sb.as<u64>();
        H.sa_mask = H.sb_mask = (u64)(slots - 1);
    }
    HCI_LAUNCH(ctx, "pt2_insert_v", s, pt_insert_v, ceil_div(N, 256), 256, 0, H, dets, N);
    // count, scan, fill (i order)
    DevMem counts = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    HCI_LAUNCH(ctx, "pt2_count", s, pt_count_kernel, ceil_div(N, PT_ROWS), PT_BLOCK, 0, T, I, H, dets,
               c, N, eps2, hbm, counts.as<u32>());
    HIP_CHECK(hipMemsetAsync(counts.as<u32>() + N, 0, sizeof(u32), s));
    st->off = dev_alloc(ctx, sizeof(i64) * (N + 1), s);
    scan_u32_to_i64(ctx, counts.as<u32>(), st->off.as<i64>(), N + 1, s);
    const i64 M = read_scalar(st->off.as<i64>() + N, s);
    HCI_REQUIRE(read_scalar(flags.as<u64>() + 1, s) == 0, HCI_E_NOMEM, "pt2: hash set of V overflowed");
    HCI_REQUIRE(M < ((i64)1 << 32) - 1, HCI_E_UNSUPPORTED, "pt2: more than 2^32 screened pairs");
    st->M = M;
    st->N = N;
    const i64 Ma = M > 0 ? M : 1;
    st->a_hi = dev_alloc(ctx, sizeof(u64) * Ma, s);
    st->a_lo = dev_alloc(ctx, sizeof(u64) * Ma, s);
    st->idx = dev_alloc(ctx, sizeof(u32) * Ma, s);
    st->hai = dev_alloc(ctx, sizeof(double) * Ma, s);
    st->dpair = dev_alloc(ctx, sizeof(double) * Ma, s);
    st->r = dev_alloc(ctx, sizeof(double) * N, s);
    if (M == 0) {
        HIP_CHECK(hipMemsetAsync(st->r.ptr, 0, sizeof(double) * N, s));
        st->e2 = 0.0;
        st->nC = 0;
        st->dd = 0.0;
        return st;
    }
    HCI_LAUNCH(ctx, "pt2_fill_pairs", s, pt_fill_kernel, ceil_div(N, PT_ROWS), PT_BLOCK, 0, T, I, H,
               dets, c, N, eps2, hbm, st->off.as<i64>(), st->a_hi.as<u64>(), st->a_lo.as<u64>(),
               st->idx.as<u32>(), st->hai.as<double>(), fl + 4);
    HCI_REQUIRE(read_scalar(flags.as<u64>() + 4, s) == 0, HCI_E_HIP,
                "internal: pt2 fill disagrees with the count pass");
    // stable sort of a copy of the keys, payload = pair position
    DevMem khi = dev_alloc(ctx, sizeof(u64) * M, s), klo = dev_alloc(ctx, sizeof(u64) * M, s);
    DevMem perm = dev_alloc(ctx, sizeof(u32) * M, s);
    HIP_CHECK(hipMemcpyAsync(khi.ptr, st->a_hi.ptr, sizeof(u64) * M, hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipMemcpyAsync(klo.ptr, st->a_lo.ptr, sizeof(u64) * M, hipMemcpyDeviceToDevice, s));
    HCI_LAUNCH(ctx, "pt2_iota", s, iota_u32, ceil_div(M, 256), 256, 0, perm.as<u32>(), M);
    {
        DevMem thi = dev_alloc(ctx, sizeof(u64) * M, s), tlo = dev_alloc(ctx, sizeof(u64) * M, s);
        DevMem tv = dev_alloc(ctx, sizeof(u32) * M, s);
        radix_sort128(ctx, khi.as<u64>(), klo.as<u64>(), perm.as<u32>(), thi.as<u64>(), tlo.as<u64>(),
                      tv.as<u32>(), M, n, n, s);
    }
    // segments = distinct a
    DevMem fl2 = dev_alloc(ctx, sizeof(u32) * (M + 1), s), ex = dev_alloc(ctx, sizeof(u32) * (M + 1), s);
    HCI_LAUNCH(ctx, "pt2_segflags", s, seg_flags, ceil_div(M, 256), 256, 0, khi.as<u64>(), klo.as<u64>(),
               M, fl2.as<u32>());
    HIP_CHECK(hipMemsetAsync(fl2.as<u32>() + M, 0, sizeof(u32), s));
    scan_u32_to_u32(ctx, fl2.as<u32>(), ex.as<u32>(), M + 1, s);
    const i64 nseg = read_scalar(ex.as<u32>() + M, s);
    st->nC = nseg;
    DevMem start = dev_alloc(ctx, sizeof(i64) * nseg, s);
    st->ca = dev_alloc(ctx, sizeof(u64) * nseg, s);
    st->cb = dev_alloc(ctx, sizeof(u64) * nseg, s);
    st->d = dev_alloc(ctx, sizeof(double) * nseg, s);
    DevMem term = dev_alloc(ctx, sizeof(double) * nseg, s);
    HCI_LAUNCH(ctx, "pt2_segstarts", s, seg_starts, ceil_div(M, 256), 256, 0, fl2.as<u32>(), ex.as<u32>(),
               M, start.as<i64>(), khi.as<u64>(), klo.as<u64>(), st->ca.as<u64>(), st->cb.as<u64>());
    HCI_LAUNCH(ctx, "pt2_reduce", s, seg_reduce, ceil_div(nseg, 256), 256, 0, I, start.as<i64>(), nseg,
               M, perm.as<u32>(), st->hai.as<double>(), st->idx.as<u32>(), c, st->ca.as<u64>(),
               st->cb.as<u64>(), e0, st->d.as<double>(), term.as<double>(), st->dpair.as<double>());
    HCI_LAUNCH(ctx, "pt2_r", s, r_rows, ceil_div(N, 256), 256, 0, st->off.as<i64>(), N,
               st->hai.as<double>(), st->dpair.as<double>(), st->r.as<double>());
    DevMem sums = dev_alloc(ctx, sizeof(double) * 2, s);
    HCI_LAUNCH(ctx, "pt2_sum", s, sum_fixed, 1, 256, 0, term.as<double>(), nseg, sums.as<double>());
    // d.d for the relaxed density matrix
    HCI_LAUNCH(ctx, "pt2_dd_sq", s, sq_kernel_pt, ceil_div(nseg, 256), 256, 0, st->d.as<double>(), nseg,
               term.as<double>());
    HCI_LAUNCH(ctx, "pt2_sum", s, sum_fixed, 1, 256, 0, term.as<double>(), nseg, sums.as<double>() + 1);
    double hv[2];
    HIP_CHECK(hipMemcpyAsync(hv, sums.ptr, sizeof(hv), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    st->e2 = hv[0];
    st->dd = hv[1];
    return st;
}
