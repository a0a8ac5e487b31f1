// Device-wide primitives: exclusive scans, a stable LSD radix sort of
// 128-bit keys (optionally with a 32-bit payload) and adjacent-unique
// compaction.  All reductions are in a fixed order (no floating point here).
#include "common.h"

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T t = __shfl_up(v, off, 64);
        if (lane_id() >= off) v += t;
    }
    return v;
}

// Exclusive scan of one tile per block; block totals to sums.
template <class In, class Out>
__global__ void __launch_bounds__(SCAN_BLOCK) scan_tile_kernel(const In* __restrict__ in,
                                                               Out* __restrict__ out,
                                                               Out* __restrict__ sums, i64 n) {
    __shared__ Out wsum[SCAN_BLOCK / 64];
    const i64 base = (i64)blockIdx.x * SCAN_TILE + (i64)threadIdx.x * SCAN_ITEMS;
    Out v[SCAN_ITEMS];
    Out tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        i64 idx = base + k;
        v[k] = idx < n ? (Out)in[idx] : (Out)0;
        tot += v[k];
    }
    Out incl = wave_incl_scan<Out>(tot);
    const int w = threadIdx.x / 64;
    if (lane_id() == 63) wsum[w] = incl;
    __syncthreads();
    Out wave_off = 0;
    for (int k = 0; k < w; ++k) wave_off += wsum[k];
    Out run = wave_off + incl - tot;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        i64 idx = base + k;
        if (idx < n) out[idx] = run;
        run += v[k];
    }
    if (threadIdx.x == SCAN_BLOCK - 1) sums[blockIdx.x] = run;
}

template <class T>
__global__ void add_offsets_kernel(T* __restrict__ out, const T* __restrict__ offs, i64 n) {
    const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] += offs[idx / SCAN_TILE];
}

template <class In, class Out>
void scan_impl(hci_ctx_s* ctx, const In* in, Out* out, i64 n, hipStream_t s) {
    if (n <= 0) return;
    const i64 nb = ceil_div(n, SCAN_TILE);
    DevMem sums = dev_alloc(ctx, sizeof(Out) * nb, s);
    HCI_LAUNCH(ctx, "scan_tile", s, (scan_tile_kernel<In, Out>), nb, SCAN_BLOCK, 0, in, out,
               sums.as<Out>(), n);
    if (nb > 1) {
        DevMem sums2 = dev_alloc(ctx, sizeof(Out) * nb, s);
        scan_impl<Out, Out>(ctx, sums.as<Out>(), sums2.as<Out>(), nb, s);
        HCI_LAUNCH(ctx, "scan_add", s, add_offsets_kernel<Out>, ceil_div(n, 256), 256, 0, out,
                   sums2.as<Out>(), n);
    }
}

// ------------------------------------------------------------ radix sort
constexpr int RS_BLOCK = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;

__device__ __forceinline__ u32 digit_of(u64 hi, u64 lo, int pass, int passes_lo) {
    return pass < passes_lo ? byte_of(lo, pass) : byte_of(hi, pass - passes_lo);
}

__global__ void __launch_bounds__(RS_BLOCK) rs_hist_kernel(const u64* __restrict__ hi,
                                                           const u64* __restrict__ lo, i64 n,
                                                           int pass, int passes_lo,
                                                           u32* __restrict__ counts, i64 nblocks) {
    __shared__ u32 hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const i64 base = (i64)blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_ITEMS; ++k) {
        i64 idx = base + (i64)k * RS_BLOCK + threadIdx.x;
        if (idx < n) atomicAdd(&hist[digit_of(hi ? hi[idx] : 0ull, lo[idx], pass, passes_lo)], 1u);
    }
    __syncthreads();
    counts[(i64)threadIdx.x * nblocks + blockIdx.x] = hist[threadIdx.x];
}

// Stable scatter: keys of a tile are ranked in memory order.  Each round a
// wavefront ranks 64 consecutive keys with a ballot-built peer mask; waves of
// the block are combined in wave order through LDS.
template <bool HAS_VAL>
__global__ void __launch_bounds__(RS_BLOCK) rs_scatter_kernel(
    const u64* __restrict__ hi, const u64* __restrict__ lo, const u32* __restrict__ vals, i64 n,
    int pass, int passes_lo, const u32* __restrict__ offsets, i64 nblocks, u64* __restrict__ ohi,
    u64* __restrict__ olo, u32* __restrict__ ovals) {
    __shared__ u32 run[256];
    __shared__ u32 wcnt[RS_BLOCK / 64][256];
    run[threadIdx.x] = offsets[(i64)threadIdx.x * nblocks + blockIdx.x];
    const int w = threadIdx.x / 64;
    const int lane = lane_id();
    const i64 base = (i64)blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_ITEMS; ++k) {
        for (int t = threadIdx.x; t < (RS_BLOCK / 64) * 256; t += RS_BLOCK) (&wcnt[0][0])[t] = 0;
        __syncthreads();
        const i64 idx = base + (i64)k * RS_BLOCK + threadIdx.x;
        const bool valid = idx < n;
        u64 khi = 0, klo = 0;
        u32 kv = 0;
        u32 d = 0;
        if (valid) {
            khi = hi ? hi[idx] : 0ull;
            klo = lo[idx];
            if (HAS_VAL) kv = vals[idx];
            d = digit_of(khi, klo, pass, passes_lo);
        }
        u64 peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            u64 m = ballot(((d >> b) & 1u) != 0);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        u32 rank = rank_in(peers);
        if (valid && rank == 0) wcnt[w][d] = (u32)__popcll(peers);
        __syncthreads();
        if (valid) {
            u32 pos = run[d] + rank;
            for (int q = 0; q < w; ++q) pos += wcnt[q][d];
            if (ohi) ohi[pos] = khi;
            olo[pos] = klo;
            if (HAS_VAL) ovals[pos] = kv;
        }
        __syncthreads();
        {
            u32 add = 0;
            for (int q = 0; q < RS_BLOCK / 64; ++q) add += wcnt[q][threadIdx.x];
            run[threadIdx.x] += add;
        }
        __syncthreads();
    }
}

__global__ void unique_flags_kernel(const u64* __restrict__ hi, const u64* __restrict__ lo, i64 n,
                                    u32* __restrict__ flags) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flags[i] = (i == 0 || hi[i] != hi[i - 1] || lo[i] != lo[i - 1]) ? 1u : 0u;
}

__global__ void unique_write_kernel(const u64* __restrict__ hi, const u64* __restrict__ lo, i64 n,
                                    const u32* __restrict__ flags, const u32* __restrict__ pos,
                                    u64* __restrict__ out) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flags[i]) return;
    const u32 p = pos[i];
    out[2 * (i64)p] = hi[i];
    out[2 * (i64)p + 1] = lo[i];
}

}  // namespace

void scan_u32_to_u32(hci_ctx_s* ctx, const u32* in, u32* out, i64 n, hipStream_t s) {
    scan_impl<u32, u32>(ctx, in, out, n, s);
}
void scan_u32_to_i64(hci_ctx_s* ctx, const u32* in, i64* out, i64 n, hipStream_t s) {
    scan_impl<u32, i64>(ctx, in, out, n, s);
}
void scan_i64(hci_ctx_s* ctx, const i64* in, i64* out, i64 n, hipStream_t s) {
    scan_impl<i64, i64>(ctx, in, out, n, s);
}

void radix_sort128(hci_ctx_s* ctx, u64* hi, u64* lo, u32* vals, u64* thi, u64* tlo, u32* tvals,
                   i64 n, int bits_hi, int bits_lo, hipStream_t s) {
    if (n <= 1) return;
    HCI_REQUIRE(n < ((i64)1 << 32), HCI_E_UNSUPPORTED, "radix sort: more than 2^32 keys");
    const int passes_lo = (bits_lo + 7) / 8;
    const int passes_hi = (bits_hi + 7) / 8;
    const int passes = passes_lo + passes_hi;
    const i64 nb = ceil_div(n, RS_TILE);
    DevMem counts = dev_alloc(ctx, sizeof(u32) * 256 * nb, s);
    DevMem offs = dev_alloc(ctx, sizeof(u32) * 256 * nb, s);
    u64 *shi = hi, *slo = lo, *dhi = thi, *dlo = tlo;
    u32 *sv = vals, *dv = tvals;
    for (int p = 0; p < passes; ++p) {
        HCI_LAUNCH(ctx, "radix_hist", s, rs_hist_kernel, nb, RS_BLOCK, 0, shi, slo, n, p, passes_lo,
                   counts.as<u32>(), nb);
        scan_u32_to_u32(ctx, counts.as<u32>(), offs.as<u32>(), 256 * nb, s);
        if (vals) {
            HCI_LAUNCH(ctx, "radix_scatter", s, rs_scatter_kernel<true>, nb, RS_BLOCK, 0, shi, slo,
                       sv, n, p, passes_lo, offs.as<u32>(), nb, dhi, dlo, dv);
        } else {
            HCI_LAUNCH(ctx, "radix_scatter", s, rs_scatter_kernel<false>, nb, RS_BLOCK, 0, shi, slo,
                       (const u32*)nullptr, n, p, passes_lo, offs.as<u32>(), nb, dhi, dlo,
                       (u32*)nullptr);
        }
        std::swap(shi, dhi);
        std::swap(slo, dlo);
        std::swap(sv, dv);
    }
    if (passes & 1) {
        HIP_CHECK(hipMemcpyAsync(hi, shi, sizeof(u64) * n, hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(lo, slo, sizeof(u64) * n, hipMemcpyDeviceToDevice, s));
        if (vals) HIP_CHECK(hipMemcpyAsync(vals, sv, sizeof(u32) * n, hipMemcpyDeviceToDevice, s));
    }
}

void radix_sort64_bytes(hci_ctx_s* ctx, u64* keys, u64* tmp, i64 n, int byte_lo, int byte_hi, hipStream_t s) {
    if (n <= 1 || byte_hi <= byte_lo) return;
    HCI_REQUIRE(n < ((i64)1 << 32), HCI_E_UNSUPPORTED, "radix sort: more than 2^32 keys");
    HCI_REQUIRE(byte_lo >= 0 && byte_hi <= 8, HCI_E_ARG, "radix sort: byte range outside a 64-bit key");
    const i64 nb = ceil_div(n, RS_TILE);
    DevMem counts = dev_alloc(ctx, sizeof(u32) * 256 * nb, s);
    DevMem offs = dev_alloc(ctx, sizeof(u32) * 256 * nb, s);
    u64 *src = keys, *dst = tmp;
    for (int p = byte_lo; p < byte_hi; ++p) {  // passes_lo = 8: every digit is a byte of the one word
        HCI_LAUNCH(ctx, "radix_hist", s, rs_hist_kernel, nb, RS_BLOCK, 0, (const u64*)nullptr, src, n, p, 8,
                   counts.as<u32>(), nb);
        scan_u32_to_u32(ctx, counts.as<u32>(), offs.as<u32>(), 256 * nb, s);
        HCI_LAUNCH(ctx, "radix_scatter", s, rs_scatter_kernel<false>, nb, RS_BLOCK, 0, (const u64*)nullptr, src,
                   (const u32*)nullptr, n, p, 8, offs.as<u32>(), nb, (u64*)nullptr, dst, (u32*)nullptr);
        std::swap(src, dst);
    }
    if ((byte_hi - byte_lo) & 1) HIP_CHECK(hipMemcpyAsync(keys, src, sizeof(u64) * n, hipMemcpyDeviceToDevice, s));
}

i64 unique128_capped(hci_ctx_s* ctx, const u64* hi, const u64* lo, u64* out_pairs, i64 n, i64 cap,
                     hipStream_t s) {
    if (n <= 0) return 0;
    DevMem flags = dev_alloc(ctx, sizeof(u32) * (n + 1), s);
    DevMem pos = dev_alloc(ctx, sizeof(u32) * (n + 1), s);
    HCI_LAUNCH(ctx, "unique_flags", s, unique_flags_kernel, ceil_div(n, 256), 256, 0, hi, lo, n,
               flags.as<u32>());
    HIP_CHECK(hipMemsetAsync(flags.as<u32>() + n, 0, sizeof(u32), s));
    scan_u32_to_u32(ctx, flags.as<u32>(), pos.as<u32>(), n + 1, s);
    const u32 m = read_scalar(pos.as<u32>() + n, s);
    if ((i64)m > cap) return (i64)m;
    HCI_LAUNCH(ctx, "unique_write", s, unique_write_kernel, ceil_div(n, 256), 256, 0, hi, lo, n,
               flags.as<u32>(), pos.as<u32>(), out_pairs);
    return (i64)m;
}
