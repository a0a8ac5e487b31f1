// <S^2> of a state on a determinant list, to characterise the states the
// method targets (the paper's triplet and quintet states are the lowest of
// their spin projection).  S^2 = S_z (S_z + 1) + S_- S_+, so
//   <S^2> = S_z (S_z + 1) + |S_+ c|^2 / |c|^2,   S_+ = sum_p a+_{p,alpha} a_{p,beta}.
// a+_{p,alpha} a_{p,beta} maps D = (alpha, beta) with p in beta and not in
// alpha to D' = (alpha + p, beta - p), sign (-1)^(N_alpha + #beta below p +
// #alpha below p) (alpha creators left of beta creators, ascending orbitals).
// The images of every (D, p) are sorted by D' (stable, so the terms of one
// D' stay in list order), each D' sums its terms in that order, and the
// squares are summed in a fixed order.
#include "common.h"

namespace {

constexpr int SP_BLOCK = 256;

__global__ void raise_count_kernel(const u64* __restrict__ dets, i64 N, u32* __restrict__ cnt) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) cnt[i] = (u32)popc64(dets[2 * i + 1] & ~dets[2 * i]);
    if (i == N) cnt[i] = 0u;
}

__global__ void raise_fill_kernel(const u64* __restrict__ dets, const double* __restrict__ c, i64 N,
                                  int na, const i64* __restrict__ off, u64* __restrict__ khi,
                                  u64* __restrict__ klo, double* __restrict__ val, u32* __restrict__ perm) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const u64 A = dets[2 * i], B = dets[2 * i + 1];
    i64 k = off[i];
    for (u64 m = B & ~A; m; m &= m - 1) {
        const int p = ctz64(m);
        const u64 below = bit(p) - 1ull;
        const int par = (na + popc64(B & below) + popc64(A & below)) & 1;
        khi[k] = A | bit(p);
        klo[k] = B & ~bit(p);
        val[k] = par ? -c[i] : c[i];
        perm[k] = (u32)k;
        ++k;
    }
}

__global__ void key_change_kernel(const u64* __restrict__ hi, const u64* __restrict__ lo, i64 n,
                                  u32* __restrict__ flags) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = (i == 0 || hi[i] != hi[i - 1] || lo[i] != lo[i - 1]) ? 1u : 0u;
    if (i == n) flags[i] = 0u;
}

__global__ void segment_start_kernel(const u32* __restrict__ flags, const u32* __restrict__ excl, i64 n,
                                     i64* __restrict__ start) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flags[i]) start[excl[i]] = i;
    if (i == n) start[excl[n]] = n;
}

// one thread per image D': (sum of its terms in list order)^2
__global__ void segment_square_kernel(const i64* __restrict__ start, i64 nseg, const u32* __restrict__ perm,
                                      const double* __restrict__ val, double* __restrict__ sq) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    double a = 0.0;
    for (i64 k = start[s]; k < start[s + 1]; ++k) a += val[perm[k]];
    sq[s] = a * a;
}

__global__ void __launch_bounds__(SP_BLOCK) partial_sums_kernel(const double* __restrict__ x, i64 n,
                                                                const double* __restrict__ y, double* __restrict__ part) {
    __shared__ double lds[SP_BLOCK / 64];
    double a = 0.0;
    for (i64 i = (i64)blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += (i64)gridDim.x * SP_BLOCK)
        a += y ? x[i] * y[i] : x[i];
    const double v = block_sum_f64<SP_BLOCK>(a, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// fixed-order sum of x (or of x * y): block partials, then one block
double fixed_sum(hci_ctx_s* ctx, const double* x, const double* y, i64 n, hipStream_t s) {
    const i64 nb = std::max<i64>(1, std::min<i64>(1024, ceil_div(n, SP_BLOCK * 8)));
    DevMem part = dev_alloc(ctx, sizeof(double) * (nb + 1), s);
    HCI_LAUNCH(ctx, "spin_sum", s, partial_sums_kernel, nb, SP_BLOCK, 0, x, n, y, part.as<double>());
    HCI_LAUNCH(ctx, "spin_sum", s, partial_sums_kernel, 1, SP_BLOCK, 0, (const double*)part.as<double>(), nb,
               (const double*)nullptr, part.as<double>() + nb);
    return read_scalar(part.as<double>() + nb, s);
}

}  // namespace

double spin_square(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, hipStream_t s) {
    const double sz = 0.5 * (ctx->na - ctx->nb);
    const double norm2 = fixed_sum(ctx, c, c, N, s);
    HCI_REQUIRE(norm2 > 0.0, HCI_E_ARG, "spin_square: c is zero");
    DevMem cnt = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    HCI_LAUNCH(ctx, "spin_raise", s, raise_count_kernel, ceil_div(N + 1, SP_BLOCK), SP_BLOCK, 0, dets, N,
               cnt.as<u32>());
    DevMem off = dev_alloc(ctx, sizeof(i64) * (N + 1), s);
    scan_u32_to_i64(ctx, cnt.as<u32>(), off.as<i64>(), N + 1, s);
    const i64 M = read_scalar(off.as<i64>() + N, s);
    if (M == 0) return sz * (sz + 1.0);
    HCI_REQUIRE(M < ((i64)1 << 32) - 1, HCI_E_UNSUPPORTED, "spin_square: too many raised images");
    DevMem khi = dev_alloc(ctx, sizeof(u64) * M, s), klo = dev_alloc(ctx, sizeof(u64) * M, s);
    DevMem val = dev_alloc(ctx, sizeof(double) * M, s);
    DevMem perm = dev_alloc(ctx, sizeof(u32) * M, s);
    HCI_LAUNCH(ctx, "spin_raise", s, raise_fill_kernel, ceil_div(N, SP_BLOCK), SP_BLOCK, 0, dets, c, N,
               ctx->na, (const i64*)off.as<i64>(), khi.as<u64>(), klo.as<u64>(), val.as<double>(),
               perm.as<u32>());
    {
        DevMem thi = dev_alloc(ctx, sizeof(u64) * M, s), tlo = dev_alloc(ctx, sizeof(u64) * M, s);
        DevMem tv = dev_alloc(ctx, sizeof(u32) * M, s);
        radix_sort128(ctx, khi.as<u64>(), klo.as<u64>(), perm.as<u32>(), thi.as<u64>(), tlo.as<u64>(),
                      tv.as<u32>(), M, ctx->n, ctx->n, s);
    }
    DevMem flags = dev_alloc(ctx, sizeof(u32) * (M + 1), s), excl = dev_alloc(ctx, sizeof(u32) * (M + 1), s);
    HCI_LAUNCH(ctx, "spin_segments", s, key_change_kernel, ceil_div(M + 1, SP_BLOCK), SP_BLOCK, 0,
               khi.as<u64>(), klo.as<u64>(), M, flags.as<u32>());
    scan_u32_to_u32(ctx, flags.as<u32>(), excl.as<u32>(), M + 1, s);
    const i64 nseg = read_scalar(excl.as<u32>() + M, s);
    DevMem start = dev_alloc(ctx, sizeof(i64) * (nseg + 1), s);
    HCI_LAUNCH(ctx, "spin_segments", s, segment_start_kernel, ceil_div(M + 1, SP_BLOCK), SP_BLOCK, 0,
               flags.as<u32>(), excl.as<u32>(), M, start.as<i64>());
    DevMem sq = dev_alloc(ctx, sizeof(double) * nseg, s);
    HCI_LAUNCH(ctx, "spin_segments", s, segment_square_kernel, ceil_div(nseg, SP_BLOCK), SP_BLOCK, 0,
               (const i64*)start.as<i64>(), nseg, (const u32*)perm.as<u32>(), (const double*)val.as<double>(),
               sq.as<double>());
    const double raised = fixed_sum(ctx, sq.as<double>(), nullptr, nseg, s);
    return sz * (sz + 1.0) + raised / norm2;
}
