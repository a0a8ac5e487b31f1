// Structure of a sorted determinant list V, built once per list and cached:
//   * alpha-major buckets: V is sorted by (alpha, beta), so determinants that
//     share an alpha string are contiguous (ia, ua, aoff);
//   * beta-major order: a stable sort by beta gives (beta, alpha) order
//     (permb, ib, ub, boff);
//   * single-excitation adjacency among the unique alpha strings and among
//     the unique beta strings (as_ptr/as_idx, bs_ptr/bs_idx), each list
//     sorted by target index.
// Together they enumerate every pair of V at excitation degree <= 2 without
// candidate lists: same alpha (beta differs), same beta (alpha differs), and
// alpha-single x beta-single through the adjacency lists.
#include "common.h"

namespace {

__device__ __forceinline__ u64 mix64(u64 x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

// Validate (popcounts, bits above norb, strict ascending order), split into
// SoA words, and accumulate a position-dependent content hash (wrapping sum,
// order independent so the integer atomics give a deterministic value).
__global__ void validate_kernel(const u64* __restrict__ dets, i64 N, int n, int na, int nb,
                                u64* __restrict__ alpha, u64* __restrict__ beta,
                                unsigned long long* __restrict__ hash,
                                unsigned long long* __restrict__ bad) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    u64 hv = 0, err = 0;
    if (i < N) {
        const u64 a = dets[2 * i], b = dets[2 * i + 1];
        alpha[i] = a;
        beta[i] = b;
        const u64 mask = low_mask(n);
        if (__popcll(a) != na || __popcll(b) != nb || (a & ~mask) || (b & ~mask)) err = 1;
        if (i > 0) {
            const u64 pa = dets[2 * i - 2], pb = dets[2 * i - 1];
            if (!(pa < a || (pa == a && pb < b))) err = 1;
        }
        hv = mix64(a * 0x9e3779b97f4a7c15ull ^ mix64(b + 0x632be59bd9b4e019ull) ^ (u64)i);
    }
    hv = wave_sum_u64(hv);
    err = wave_sum_u64(err);
    if (lane_id() == 0) {
        if (hv) atomicAdd(hash, (unsigned long long)hv);
        if (err) atomicAdd(bad, (unsigned long long)err);
    }
}

__global__ void flag_change_kernel(const u64* __restrict__ x, i64 N, u32* __restrict__ flag) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) flag[i] = (i == 0 || x[i] != x[i - 1]) ? 1u : 0u;
}

// inclusive index of each element's group = exclusive scan + flag - 1
__global__ void group_fill_kernel(const u64* __restrict__ x, i64 N, const u32* __restrict__ flag,
                                  const u32* __restrict__ excl, u32* __restrict__ gidx,
                                  u64* __restrict__ uniq, u32* __restrict__ off) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const u32 gi = excl[i] + flag[i] - 1u;
    gidx[i] = gi;
    if (flag[i]) {
        uniq[gi] = x[i];
        off[gi] = (u32)i;
    }
}

__global__ void set_u32_kernel(u32* p, u32 v) { *p = v; }

__global__ void iota_kernel(u32* __restrict__ x, i64 N) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) x[i] = (u32)i;
}

__global__ void zero_u64_kernel(u64* __restrict__ x, i64 N) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) x[i] = 0;
}

__global__ void scatter_u32_kernel(const u32* __restrict__ src, const u32* __restrict__ perm, i64 N,
                                   u32* __restrict__ dst) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < N) dst[perm[k]] = src[k];
}

__device__ __forceinline__ i64 find_u64(const u64* __restrict__ arr, i64 len, u64 key) {
    i64 lo = 0, hi = len;
    while (lo < hi) {
        const i64 mid = (lo + hi) >> 1;
        if (arr[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < len && arr[lo] == key) ? lo : -1;
}

// One thread per unique string: count (or list) the unique strings one
// single excitation away.  Fill mode sorts the thread's list by index.
template <bool FILL>
__global__ void adjacency_kernel(const u64* __restrict__ uniq, i64 m, int n,
                                 const u32* __restrict__ ptr, u32* __restrict__ cnt_or_idx) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const u64 s = uniq[k];
    const u64 full = low_mask(n);
    u32 c = 0;
    u32* out = FILL ? cnt_or_idx + ptr[k] : nullptr;
    for (u64 occ = s; occ; occ &= occ - 1) {
        const int p = __builtin_ctzll(occ);
        for (u64 emp = ~s & full; emp; emp &= emp - 1) {
            const int r = __builtin_ctzll(emp);
            const i64 t = find_u64(uniq, m, s ^ bit(p) ^ bit(r));
            if (t >= 0) {
                if (FILL) out[c] = (u32)t;
                ++c;
            }
        }
    }
    if (!FILL) {
        cnt_or_idx[k] = c;
    } else {
        for (u32 x = 1; x < c; ++x) {  // insertion sort (lists are short)
            const u32 v = out[x];
            int y = (int)x - 1;
            while (y >= 0 && out[y] > v) {
                out[y + 1] = out[y];
                --y;
            }
            out[y + 1] = v;
        }
    }
}

void build_groups(hci_ctx_s* ctx, const u64* x, i64 N, DevMem& gidx, DevMem& uniq, DevMem& off,
                  i64& m, hipStream_t s) {
    DevMem flag = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    DevMem excl = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    HCI_LAUNCH(ctx, "space_flags", s, flag_change_kernel, ceil_div(N, 256), 256, 0, x, N,
               flag.as<u32>());
    HIP_CHECK(hipMemsetAsync(flag.as<u32>() + N, 0, sizeof(u32), s));
    scan_u32_to_u32(ctx, flag.as<u32>(), excl.as<u32>(), N + 1, s);
    m = read_scalar(excl.as<u32>() + N, s);
    gidx = dev_alloc(ctx, sizeof(u32) * N, s);
    uniq = dev_alloc(ctx, sizeof(u64) * m, s);
    off = dev_alloc(ctx, sizeof(u32) * (m + 1), s);
    HCI_LAUNCH(ctx, "space_groups", s, group_fill_kernel, ceil_div(N, 256), 256, 0, x, N,
               flag.as<u32>(), excl.as<u32>(), gidx.as<u32>(), uniq.as<u64>(), off.as<u32>());
    HCI_LAUNCH(ctx, "set_u32", s, set_u32_kernel, 1, 1, 0, off.as<u32>() + m, (u32)N);
}

void build_adjacency(hci_ctx_s* ctx, const DevMem& uniq, i64 m, int n, DevMem& ptr, DevMem& idx,
                     i64& total, hipStream_t s) {
    DevMem cnt = dev_alloc(ctx, sizeof(u32) * (m + 1), s);
    ptr = dev_alloc(ctx, sizeof(u32) * (m + 1), s);
    HCI_LAUNCH(ctx, "adjacency_count", s, adjacency_kernel<false>, ceil_div(m, 128), 128, 0,
               uniq.as<u64>(), m, n, (const u32*)nullptr, cnt.as<u32>());
    HIP_CHECK(hipMemsetAsync(cnt.as<u32>() + m, 0, sizeof(u32), s));
    {
        // the offsets below and the per-bucket position tables of the stored
        // layout (one entry per link and per string) are 32-bit: refuse a
        // space whose links would wrap them, before anything is written
        DevMem wide = dev_alloc(ctx, sizeof(i64) * (m + 1), s);
        scan_u32_to_i64(ctx, cnt.as<u32>(), wide.as<i64>(), m + 1, s);
        const i64 links = read_scalar(wide.as<i64>() + m, s);
        HCI_REQUIRE(links + m < ((i64)1 << 32) - 1, HCI_E_UNSUPPORTED,
                    "the unique strings of this list have " + std::to_string(links) +
                        " single-excitation links; at most 2^32 - 2 minus the string count are supported");
    }
    scan_u32_to_u32(ctx, cnt.as<u32>(), ptr.as<u32>(), m + 1, s);
    total = read_scalar(ptr.as<u32>() + m, s);
    idx = dev_alloc(ctx, sizeof(u32) * (total > 0 ? total : 1), s);
    HCI_LAUNCH(ctx, "adjacency_fill", s, adjacency_kernel<true>, ceil_div(m, 128), 128, 0,
               uniq.as<u64>(), m, n, ptr.as<u32>(), idx.as<u32>());
}

}  // namespace

// Strings, groups, the beta-major permutation and the single-excitation
// adjacency of a validated list.
namespace {
__global__ void permute_u64_kernel(const u64* __restrict__ in, const u32* __restrict__ permb, i64 N,
                                   u64* __restrict__ out) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < N) out[k] = in[permb[k]];
}
}  // namespace

void ensure_alpha_b(hci_ctx_s* ctx, Space* sp, hipStream_t s) {
    if (sp->alpha_b.ptr) return;
    sp->alpha_b = dev_alloc(ctx, sizeof(u64) * sp->N, s);
    HCI_LAUNCH(ctx, "alpha_beta_major", s, permute_u64_kernel, ceil_div(sp->N, 256), 256, 0, sp->alpha.as<u64>(),
               sp->permb.as<u32>(), sp->N, sp->alpha_b.as<u64>());
}

static void build_structure(hci_ctx_s* ctx, Space* sp, int n, hipStream_t s) {
    const i64 N = sp->N;
    // alpha-major groups
    build_groups(ctx, sp->alpha.as<u64>(), N, sp->ia, sp->ua, sp->aoff, sp->nua, s);
    // beta-major order: stable sort of beta with det index as payload
    {
        DevMem khi = dev_alloc(ctx, sizeof(u64) * N, s), klo = dev_alloc(ctx, sizeof(u64) * N, s);
        DevMem thi = dev_alloc(ctx, sizeof(u64) * N, s), tlo = dev_alloc(ctx, sizeof(u64) * N, s);
        DevMem tv = dev_alloc(ctx, sizeof(u32) * N, s);
        sp->permb = dev_alloc(ctx, sizeof(u32) * N, s);
        HCI_LAUNCH(ctx, "zero_u64", s, zero_u64_kernel, ceil_div(N, 256), 256, 0, khi.as<u64>(), N);
        HIP_CHECK(hipMemcpyAsync(klo.ptr, sp->beta.ptr, sizeof(u64) * N, hipMemcpyDeviceToDevice, s));
        HCI_LAUNCH(ctx, "iota", s, iota_kernel, ceil_div(N, 256), 256, 0, sp->permb.as<u32>(), N);
        radix_sort128(ctx, khi.as<u64>(), klo.as<u64>(), sp->permb.as<u32>(), thi.as<u64>(),
                      tlo.as<u64>(), tv.as<u32>(), N, 0, n, s);
        DevMem ib_sorted;
        build_groups(ctx, klo.as<u64>(), N, ib_sorted, sp->ub, sp->boff, sp->nub, s);
        sp->ib = dev_alloc(ctx, sizeof(u32) * N, s);
        HCI_LAUNCH(ctx, "scatter_u32", s, scatter_u32_kernel, ceil_div(N, 256), 256, 0,
                   ib_sorted.as<u32>(), sp->permb.as<u32>(), N, sp->ib.as<u32>());
    }
    build_adjacency(ctx, sp->ua, sp->nua, n, sp->as_ptr, sp->as_idx, sp->n_as, s);
    build_adjacency(ctx, sp->ub, sp->nub, n, sp->bs_ptr, sp->bs_idx, sp->n_bs, s);
}

Space* get_space(hci_ctx_s* ctx, const u64* dets, i64 N, hipStream_t s) {
    HCI_REQUIRE(dets != nullptr && N > 0, HCI_E_ARG, "empty or null determinant list");
    HCI_REQUIRE(N < ((i64)1 << 32) - 1, HCI_E_UNSUPPORTED, "more than 2^32-2 determinants");
    const int n = ctx->n;
    // validate + hash into fresh SoA buffers
    DevMem alpha = dev_alloc(ctx, sizeof(u64) * N, s);
    DevMem beta = dev_alloc(ctx, sizeof(u64) * N, s);
    DevMem hb = dev_alloc(ctx, sizeof(u64) * 2, s);
    HIP_CHECK(hipMemsetAsync(hb.ptr, 0, sizeof(u64) * 2, s));
    HCI_LAUNCH(ctx, "space_validate", s, validate_kernel, ceil_div(N, 256), 256, 0, dets, N, n,
               ctx->na, ctx->nb, alpha.as<u64>(), beta.as<u64>(),
               (unsigned long long*)hb.as<u64>(), (unsigned long long*)(hb.as<u64>() + 1));
    u64 hv[2];
    HIP_CHECK(hipMemcpyAsync(hv, hb.ptr, sizeof(hv), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    HCI_REQUIRE(hv[1] == 0, HCI_E_ARG,
                "determinant list not strictly ascending or wrong electron counts");
    Space* sp = ctx->space;
    // the cache is keyed by content (length and hash), not by address, so an
    // equal list in another buffer reuses the built structure
    if (sp && sp->N == N && sp->hash == hv[0]) return sp;
    drop_space(ctx);
    sp = new Space();
    ctx->space = sp;
    sp->key_ptr = dets;
    sp->N = N;
    sp->hash = hv[0];
    sp->alpha = std::move(alpha);
    sp->beta = std::move(beta);
    try {
        build_structure(ctx, sp, n, s);
    } catch (...) {
        drop_space(ctx);  // never leave a half-built entry under this list's key
        throw;
    }
    return sp;
}
