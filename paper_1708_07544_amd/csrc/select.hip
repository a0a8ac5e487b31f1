// One HCI selection step: V' = V + C(eps1), where C(eps1) holds every
// determinant D_a outside V with |H_ai c_i| > eps1 for some D_i in V
// (Sec. "Variational Stage", eq. criteria and the HCI importance function).
// Candidates come from the heat-bath walk (no candidate lists are built
// for pairs that cannot pass); they are appended to V, radix-sorted and
// made unique, which also removes the members of V that were re-found.
#include "walk.h"

namespace {

constexpr int WALK_BLOCK = 256;
constexpr int WALK_ROWS = WALK_BLOCK / HCI_WAVE;

struct EmitVis {
    u64* out_hi;
    u64* out_lo;
    unsigned long long* counter;
    i64 cap;
    __device__ __forceinline__ void operator()(bool ok, u64 aa, u64 ab) {
        const u64 m = ballot(ok);
        if (!m) return;
        unsigned long long base = 0;
        if (lane_id() == 0) base = atomicAdd(counter, (unsigned long long)__popcll(m));
        base = __shfl(base, 0, 64);
        if (ok) {
            const i64 at = (i64)base + __popcll(m & lanemask_lt());
            if (at < cap) {
                out_hi[at] = aa;
                out_lo[at] = ab;
            }
        }
    }
};

__global__ void __launch_bounds__(WALK_BLOCK) select_walk_kernel(
    HBView T, IntView I, const u64* __restrict__ dets, const double* __restrict__ c, i64 N,
    double eps, double hb_max, u64* __restrict__ out_hi, u64* __restrict__ out_lo, i64 cap,
    unsigned long long* __restrict__ counter) {
    const i64 i = (i64)blockIdx.x * WALK_ROWS + threadIdx.x / HCI_WAVE;
    if (i >= N) return;
    const double ci = fabs(c[i]);
    if (!(hb_max * ci > eps)) return;  // nothing can pass from this determinant
    EmitVis v{out_hi, out_lo, counter, cap};
    heat_bath_walk(T, I, dets[2 * i], dets[2 * i + 1], ci, eps, v);
}

__global__ void split_kernel(const u64* __restrict__ dets, i64 N, u64* __restrict__ hi,
                             u64* __restrict__ lo) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        hi[i] = dets[2 * i];
        lo[i] = dets[2 * i + 1];
    }
}

__global__ void max_reduce_kernel(const double* __restrict__ a, i64 n, i64 stride,
                                  double* __restrict__ out) {
    // one block: max over a[k * stride], k < n
    __shared__ double red[256];
    double m = 0.0;
    for (i64 k = threadIdx.x; k < n; k += 256) m = fmax(m, a[k * stride]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = fmax(*out, red[0]);
}

// out[pos(V[k] in V')] = c[k]; missing members bump the error counter
__global__ void embed_kernel(const u64* __restrict__ dets, i64 n, const double* __restrict__ c,
                             const u64* __restrict__ dn, i64 nn, double* __restrict__ out,
                             unsigned long long* __restrict__ missing) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const u64 a = dets[2 * k], b = dets[2 * k + 1];
    i64 lo = 0, hi = nn;
    while (lo < hi) {
        const i64 mid = (lo + hi) >> 1;
        const u64 ma = dn[2 * mid], mb = dn[2 * mid + 1];
        if (ma < a || (ma == a && mb < b)) lo = mid + 1;
        else hi = mid;
    }
    if (lo < nn && dn[2 * lo] == a && dn[2 * lo + 1] == b) out[lo] = c[k];
    else atomicAdd(missing, 1ull);
}

}  // namespace

void embed_run(hci_ctx_s* ctx, const u64* dets, i64 n, const double* c, const u64* dn, i64 nn,
               double* out, hipStream_t s) {
    DevMem miss = dev_alloc(ctx, sizeof(u64), s);
    HIP_CHECK(hipMemsetAsync(miss.ptr, 0, sizeof(u64), s));
    HIP_CHECK(hipMemsetAsync(out, 0, sizeof(double) * nn, s));
    HCI_LAUNCH(ctx, "embed", s, embed_kernel, ceil_div(n, 256), 256, 0, dets, n, c, dn, nn, out,
               (unsigned long long*)miss.as<u64>());
    HCI_REQUIRE(read_scalar(miss.as<u64>(), s) == 0, HCI_E_ARG,
                "embed: a determinant of V is missing from V'");
}

// Largest magnitude any single or double element can have (list heads and
// single bounds): a determinant with hb_max * |c_i| <= eps emits nothing.
double heat_bath_max(hci_ctx_s* ctx, hipStream_t s) {
    Integrals& I = ctx->ints;
    const int n = ctx->n;
    DevMem m = dev_alloc(ctx, sizeof(double), s);
    HIP_CHECK(hipMemsetAsync(m.ptr, 0, sizeof(double), s));
    if (I.os_len > 0)
        HCI_LAUNCH(ctx, "hb_max", s, max_reduce_kernel, 1, 256, 0, I.os_abs.as<double>(),
                   (i64)n * n, (i64)I.os_len, m.as<double>());
    if (I.ss_len > 0)
        HCI_LAUNCH(ctx, "hb_max", s, max_reduce_kernel, 1, 256, 0, I.ss_abs.as<double>(),
                   (i64)n * (n - 1) / 2, (i64)I.ss_len, m.as<double>());
    HCI_LAUNCH(ctx, "hb_max", s, max_reduce_kernel, 1, 256, 0, I.single_bound.as<double>(),
               (i64)n * n, (i64)1, m.as<double>());
    return read_scalar(m.as<double>(), s);
}

i64 select_run(hci_ctx_s* ctx, const u64* dets, const double* c, i64 N, double eps, u64* out,
               i64 cap, hipStream_t s) {
    const int n = ctx->n;
    const double hbm = heat_bath_max(ctx, s);
    HBView T = hb_view(ctx->ints);
    IntView I = int_view(ctx->ints);
    DevMem counter = dev_alloc(ctx, sizeof(u64), s);
    i64 guess = std::max<i64>(4 * N, 1 << 20);
    i64 total = 0;
    DevMem hi, lo;
    for (int attempt = 0; attempt < 2; ++attempt) {
        hi = dev_alloc(ctx, sizeof(u64) * (N + guess), s);
        lo = dev_alloc(ctx, sizeof(u64) * (N + guess), s);
        HIP_CHECK(hipMemsetAsync(counter.ptr, 0, sizeof(u64), s));
        // candidates land after the copy of V
        HCI_LAUNCH(ctx, "select_walk", s, select_walk_kernel, ceil_div(N, WALK_ROWS), WALK_BLOCK, 0, T,
                   I, dets, c, N, eps, hbm, hi.as<u64>() + N, lo.as<u64>() + N, guess,
                   (unsigned long long*)counter.as<u64>());
        total = (i64)read_scalar(counter.as<u64>(), s);
        if (total <= guess) break;
        guess = total;
    }
    const i64 M = N + total;
    HCI_LAUNCH(ctx, "select_split", s, split_kernel, ceil_div(N, 256), 256, 0, dets, N, hi.as<u64>(),
               lo.as<u64>());
    {
        DevMem thi = dev_alloc(ctx, sizeof(u64) * M, s), tlo = dev_alloc(ctx, sizeof(u64) * M, s);
        radix_sort128(ctx, hi.as<u64>(), lo.as<u64>(), nullptr, thi.as<u64>(), tlo.as<u64>(), nullptr,
                      M, n, n, s);
    }
    return unique128_capped(ctx, hi.as<u64>(), lo.as<u64>(), out, M, cap, s);
}
