// sigma = H c on the variational space: the product inside the Davidson
// solver (Sec. "Variational Stage") over every single and double connection
// between members of V (Sec. "Computational Details").
//
// Stored mode: the off-diagonal connections of each row are enumerated once
// (count pass, scan, fill pass) into CSR with u32 columns and float64 or
// float32 values; each product then streams the CSR once (HBM-bound).
// Recompute mode (recompute.hip): every product regenerates the connections
// and elements on the fly (no storage).  The stored product uses one
// wavefront per row and fixed-order reductions (no atomics).
#include "slater.h"

namespace {

constexpr int ROW_BLOCK = 256;               // 4 wavefronts, one row each
constexpr int ROWS_PER_BLOCK = ROW_BLOCK / HCI_WAVE;

__global__ void diag_kernel(SpaceView S, IntView I, double* __restrict__ hd) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S.N) hd[i] = diag_f64(I, S.alpha[i], S.beta[i]);
}

struct CountVis {
    u32 cnt = 0;
    __device__ __forceinline__ void operator()(bool ok, u32, u64, u64) {
        cnt += (u32)__popcll(ballot(ok));
    }
};

// one wavefront per row, striding over the rows beyond one launch's grid
__global__ void __launch_bounds__(ROW_BLOCK) count_kernel(SpaceView S, u32* __restrict__ counts) {
    for (i64 i = (i64)blockIdx.x * ROWS_PER_BLOCK + threadIdx.x / HCI_WAVE; i < S.N;
         i += (i64)gridDim.x * ROWS_PER_BLOCK) {
        CountVis v;
        enumerate_row(S, (u32)i, v);
        if (lane_id() == 0) counts[i] = v.cnt;
    }
}

// Connectivity pass of the stored matrix: column indices only (integer work).
struct ColsVis {
    u32* cols;
    i64 pos;
    __device__ __forceinline__ void operator()(bool ok, u32 j, u64, u64) {
        const u64 m = ballot(ok);
        if (ok) cols[pos + rank_in(m)] = j;
        pos += __popcll(m);
    }
};

__global__ void __launch_bounds__(ROW_BLOCK) fill_cols_kernel(SpaceView S,
                                                              const i64* __restrict__ rowptr,
                                                              u32* __restrict__ cols,
                                                              unsigned long long* __restrict__ bad) {
    const i64 i = (i64)blockIdx.x * ROWS_PER_BLOCK + threadIdx.x / HCI_WAVE;
    if (i >= S.N) return;
    ColsVis v{cols, rowptr[i]};
    enumerate_row(S, (u32)i, v);
    // the fill must reproduce the count pass exactly
    if (lane_id() == 0 && (v.pos > rowptr[i + 1] || v.pos + 4 <= rowptr[i + 1])) atomicAdd(bad, 1ull);
    // pad the row to a multiple of 4 entries with the row's own index (element 0)
    for (i64 k = v.pos + lane_id(); k < rowptr[i + 1]; k += HCI_WAVE) cols[k] = (u32)i;
}

// Element pass: one wavefront per row evaluates H_ij for its stored columns
// (padding entries, whose column is the row itself, get 0).
template <class VT>
__global__ void __launch_bounds__(ROW_BLOCK) fill_vals_kernel(SpaceView S, IntView I,
                                                              const i64* __restrict__ rowptr,
                                                              const u32* __restrict__ cols,
                                                              VT* __restrict__ vals) {
    const i64 i = (i64)blockIdx.x * ROWS_PER_BLOCK + threadIdx.x / HCI_WAVE;
    if (i >= S.N) return;
    const u64 ai = S.alpha[i], bi = S.beta[i];
    const i64 k1 = rowptr[i + 1];
    for (i64 k = rowptr[i] + lane_id(); k < k1; k += HCI_WAVE) {
        const u32 j = cols[k];
        double v = 0.0;
        if (j != (u32)i) v = hij_f64(I, ai, bi, S.alpha[j], S.beta[j]);
        vals[k] = (VT)v;
    }
}

// Stored product: one wavefront per row, lane partial sums in float64,
// butterfly reduction, float64 diagonal term.  The gathers of c_j dominate
// (the column/element stream alone runs at ~77% of HBM peak): blocks of 8
// consecutive rows, which mostly share their alpha-neighbour buckets, keep
// those gathers in the CU's L1 (measured: 512-thread blocks beat 256 and
// 1024, and 16-byte vector loads lose to 4-byte lane-contiguous loads
// because they spread each gather instruction over 4x more cache lines).
constexpr int SPMV_BLOCK = 512;
constexpr int SPMV_ROWS = SPMV_BLOCK / HCI_WAVE;

template <class VT, class CT>
__global__ void __launch_bounds__(SPMV_BLOCK) spmv_kernel(i64 N, const i64* __restrict__ rowptr,
                                                          const u32* __restrict__ cols,
                                                          const VT* __restrict__ vals,
                                                          const CT* __restrict__ cx,
                                                          const double* __restrict__ c,
                                                          const double* __restrict__ hd,
                                                          double* __restrict__ sigma) {
    const i64 i = (i64)blockIdx.x * SPMV_ROWS + threadIdx.x / HCI_WAVE;
    if (i >= N) return;
    const i64 k0 = rowptr[i], k1 = rowptr[i + 1];
    double acc = 0.0;
    for (i64 k = k0 + lane_id(); k < k1; k += HCI_WAVE) acc += (double)vals[k] * (double)cx[cols[k]];
    acc = wave_sum_f64(acc);
    if (lane_id() == 0) sigma[i] = hd[i] * c[i] + acc;
}

__global__ void pad4_kernel(const u32* __restrict__ counts, i64 n, u32* __restrict__ padded) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) padded[i] = (counts[i] + 3u) & ~3u;
}

__global__ void f64_to_f32_kernel(const double* __restrict__ x, float* __restrict__ y, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

__global__ void u32_to_i64_sum_kernel(const u32* __restrict__ x, i64 n, unsigned long long* out) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    u64 v = i < n ? (u64)x[i] : 0ull;
    v = wave_sum_u64(v);
    if (lane_id() == 0 && v) atomicAdd(out, (unsigned long long)v);
}

void ensure_rowptr(hci_ctx_s* ctx, Space* sp, hipStream_t s) {
    if (sp->layout == 1) return;
    const i64 N = sp->N;
    SpaceView S = space_view(*sp, ctx->n);
    DevMem counts = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    HCI_LAUNCH(ctx, "conn_count", s, count_kernel, row_grid(N, ROWS_PER_BLOCK, ROW_BLOCK), ROW_BLOCK, 0, S,
               counts.as<u32>());
    HIP_CHECK(hipMemsetAsync(counts.as<u32>() + N, 0, sizeof(u32), s));
    DevMem total = dev_alloc(ctx, sizeof(u64), s);
    HIP_CHECK(hipMemsetAsync(total.ptr, 0, sizeof(u64), s));
    HCI_LAUNCH(ctx, "conn_total", s, u32_to_i64_sum_kernel, ceil_div(N, 256), 256, 0, counts.as<u32>(),
               N, (unsigned long long*)total.as<u64>());
    // padded row starts (multiples of 4 entries) for the stored matrix
    DevMem padded = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    HCI_LAUNCH(ctx, "conn_pad", s, pad4_kernel, ceil_div(N + 1, 256), 256, 0, counts.as<u32>(), N + 1,
               padded.as<u32>());
    sp->rowptr = dev_alloc(ctx, sizeof(i64) * (N + 1), s);
    scan_u32_to_i64(ctx, padded.as<u32>(), sp->rowptr.as<i64>(), N + 1, s);
    sp->nnz_off = (i64)read_scalar(total.as<u64>(), s);
    sp->nnz_pad = read_scalar(sp->rowptr.as<i64>() + N, s);
    sp->layout = 1;
}

// Count pass of the stored layout: the alpha-bucket-staged layout when the
// space fits its limits, else the plain CSR.  Sets nnz_off either way.
void ensure_layout(hci_ctx_s* ctx, Space* sp, hipStream_t s) {
    if (sp->layout != 0) return;
    if (!staged_prepare(ctx, sp, s)) ensure_rowptr(ctx, sp, s);
}

}  // namespace

void ensure_diag(hci_ctx_s* ctx, Space* sp, hipStream_t s) {
    if (sp->have_diag) return;
    sp->hdiag = dev_alloc(ctx, sizeof(double) * sp->N, s);
    HCI_LAUNCH(ctx, "hdiag", s, diag_kernel, ceil_div(sp->N, 256), 256, 0, space_view(*sp, ctx->n),
               int_view(ctx->ints), sp->hdiag.as<double>());
    sp->have_diag = true;
}

i64 count_connections(hci_ctx_s* ctx, Space* sp, hipStream_t s) {
    ensure_layout(ctx, sp, s);
    return sp->nnz_off + sp->N;
}

void ensure_csr(hci_ctx_s* ctx, Space* sp, int precision, hipStream_t s) {
    ensure_layout(ctx, sp, s);
    if (sp->layout == 2) {
        staged_ensure_vals(ctx, sp, precision, s);
        return;
    }
    const bool f32 = precision == HCI_FP32_MIXED;
    if (f32 ? sp->have_csr32 : sp->have_csr64) return;
    const i64 nnz = sp->nnz_pad;
    SpaceView S = space_view(*sp, ctx->n);
    IntView I = int_view(ctx->ints);
    const i64 grid = ceil_div(sp->N, ROWS_PER_BLOCK);
    if (!sp->cols.ptr) {
        sp->cols = dev_alloc(ctx, sizeof(u32) * (nnz > 0 ? nnz : 1), s);
        DevMem bad = dev_alloc(ctx, sizeof(u64), s);
        HIP_CHECK(hipMemsetAsync(bad.ptr, 0, sizeof(u64), s));
        HCI_LAUNCH(ctx, "csr_cols", s, fill_cols_kernel, grid, ROW_BLOCK, 0, S, sp->rowptr.as<i64>(),
                   sp->cols.as<u32>(), (unsigned long long*)bad.as<u64>());
        const u64 nbad = read_scalar(bad.as<u64>(), s);
        HCI_REQUIRE(nbad == 0, HCI_E_HIP,
                    "internal: " + std::to_string(nbad) + " rows disagree with the count pass");
    }
    if (f32) {
        sp->vals32 = dev_alloc(ctx, sizeof(float) * (nnz > 0 ? nnz : 1), s);
        HCI_LAUNCH(ctx, "csr_vals_f32", s, fill_vals_kernel<float>, grid, ROW_BLOCK, 0, S, I,
                   sp->rowptr.as<i64>(), sp->cols.as<u32>(), sp->vals32.as<float>());
    } else {
        sp->vals64 = dev_alloc(ctx, sizeof(double) * (nnz > 0 ? nnz : 1), s);
        HCI_LAUNCH(ctx, "csr_vals_f64", s, fill_vals_kernel<double>, grid, ROW_BLOCK, 0, S, I,
                   sp->rowptr.as<i64>(), sp->cols.as<u32>(), sp->vals64.as<double>());
    }
    (f32 ? sp->have_csr32 : sp->have_csr64) = true;
}

int choose_mode(hci_ctx_s* ctx, Space* sp, int precision, int mode, hipStream_t s) {
    if (mode == HCI_SIGMA_STORED || mode == HCI_SIGMA_RECOMPUTE) return mode;
    // the stored builds and the plain product take one wavefront per row in
    // one launch; more rows than that are recomputed (striding kernels)
    if (ceil_div(sp->N, ROWS_PER_BLOCK) * ROW_BLOCK >= ((i64)1 << 32)) return HCI_SIGMA_RECOMPUTE;
    ensure_layout(ctx, sp, s);
    const bool f32 = precision == HCI_FP32_MIXED;
    // bytes per stored entry: value + column (u16 staged, u32 plain)
    const i64 bytes = sp->layout == 2 ? sp->st_nnz * (f32 ? 6 : 10) : sp->nnz_pad * (f32 ? 8 : 12);
    return bytes <= ctx->stored_budget ? HCI_SIGMA_STORED : HCI_SIGMA_RECOMPUTE;
}

void sigma_apply(hci_ctx_s* ctx, Space* sp, const double* c, double* sigma, int precision, int mode,
                 hipStream_t s) {
    ensure_diag(ctx, sp, s);
    const i64 N = sp->N;
    const bool f32 = precision == HCI_FP32_MIXED;
    const i64 gridp = ceil_div(N, SPMV_ROWS);
    DevMem& c32 = sp->c32;
    if (mode == HCI_SIGMA_STORED) {
        ensure_layout(ctx, sp, s);
        if (sp->layout == 2) {
            staged_apply(ctx, sp, c, sigma, precision, s);
            return;
        }
    }
    if (mode != HCI_SIGMA_STORED) {
        recompute_apply(ctx, sp, c, sigma, precision, s);
        return;
    }
    if (f32) {
        if (!c32.ptr) c32 = dev_alloc(ctx, sizeof(float) * N, s);
        HCI_LAUNCH(ctx, "c_to_f32", s, f64_to_f32_kernel, ceil_div(N, 256), 256, 0, c,
                   c32.as<float>(), N);
    }
    {
        ensure_csr(ctx, sp, precision, s);
        if (f32) {
            HCI_LAUNCH(ctx, "sigma_stored_f32", s, (spmv_kernel<float, float>), gridp, SPMV_BLOCK, 0,
                       N, sp->rowptr.as<i64>(), sp->cols.as<u32>(), sp->vals32.as<float>(),
                       c32.as<float>(), c, sp->hdiag.as<double>(), sigma);
        } else {
            HCI_LAUNCH(ctx, "sigma_stored_f64", s, (spmv_kernel<double, double>), gridp, SPMV_BLOCK,
                       0, N, sp->rowptr.as<i64>(), sp->cols.as<u32>(), sp->vals64.as<double>(), c,
                       c, sp->hdiag.as<double>(), sigma);
        }
    }
}
