// Integral staging and heat-bath tables.
//
// The magnitude of a double-excitation element depends on the four orbitals
// only, so for every occupied pair the candidate (r,s) are listed once per
// integral set, sorted by descending magnitude (Sec. "Variational Stage",
// Fig. 1b).  Opposite-spin pair (p alpha, q beta): all r != p, s != q with
// |(rp|sq)|.  Same-spin pair p < q: all r < s outside {p,q} with
// |(rp|sq) - (rq|sp)|.  Each list is sorted by one workgroup in LDS.
#include "common.h"

namespace {

constexpr int TB_BLOCK = 256;

__global__ void derived_kernel(const double* __restrict__ g, const double* __restrict__ h, int n,
                               double* __restrict__ jk, double* __restrict__ jj,
                               double* __restrict__ jdiag, double* __restrict__ kdiag,
                               float* __restrict__ jk32, float* __restrict__ jj32,
                               float* __restrict__ h32) {
    const i64 n3 = (i64)n * n * n;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n3) {
        const int q = (int)(t / ((i64)n * n)), p = (int)((t / n) % n), r = (int)(t % n);
        const double a = g[(((i64)q * n + p) * n + r) * n + r];
        const double b = g[(((i64)q * n + r) * n + r) * n + p];
        jk[t] = a - b;
        jj[t] = a;
        jk32[t] = (float)(a - b);
        jj32[t] = (float)a;
    }
    if (t < (i64)n * n) {
        const int p = (int)(t / n), q = (int)(t % n);
        jdiag[t] = g[(((i64)p * n + p) * n + q) * n + q];
        kdiag[t] = g[(((i64)p * n + q) * n + q) * n + p];
        h32[t] = (float)h[t];
    }
}

__global__ void to_f32_kernel(const double* __restrict__ x, float* __restrict__ y, i64 m) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) y[t] = (float)x[t];
}

// true when (ka, va) must come before (kb, vb): larger magnitude first,
// ties by packed (r,s) ascending
__device__ __forceinline__ bool before(double ka, u32 va, double kb, u32 vb) {
    return ka > kb || (ka == kb && va < vb);
}

__device__ void bitonic_desc(double* keys, u32* vals, int len_pad) {
    for (int k = 2; k <= len_pad; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < len_pad; t += blockDim.x) {
                const int x = t ^ j;
                if (x > t) {
                    const bool up = (t & k) == 0;
                    const double a = keys[t], b = keys[x];
                    const u32 va = vals[t], vb = vals[x];
                    const bool ok = up ? before(a, va, b, vb) : before(b, vb, a, va);
                    if (!ok) {
                        keys[t] = b;
                        keys[x] = a;
                        vals[t] = vb;
                        vals[x] = va;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(TB_BLOCK) os_table_kernel(const double* __restrict__ g, int n,
                                                            int len, int len_pad,
                                                            double* __restrict__ out_abs,
                                                            u32* __restrict__ out_rs) {
    extern __shared__ unsigned char smem[];
    double* keys = reinterpret_cast<double*>(smem);
    u32* vals = reinterpret_cast<u32*>(keys + len_pad);
    const int P = blockIdx.x;
    const int p = P / n, q = P % n;
    for (int t = threadIdx.x; t < len_pad; t += blockDim.x) {
        if (t < len) {
            int r = t / (n - 1), s = t % (n - 1);
            r += (r >= p);
            s += (s >= q);
            keys[t] = fabs(g[(((i64)r * n + p) * n + s) * n + q]);
            vals[t] = (u32)r | ((u32)s << 8);
        } else {
            keys[t] = -1.0;
            vals[t] = 0xffffffffu;
        }
    }
    __syncthreads();
    bitonic_desc(keys, vals, len_pad);
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
        out_abs[(i64)P * len + t] = keys[t];
        out_rs[(i64)P * len + t] = vals[t];
    }
}

__global__ void __launch_bounds__(TB_BLOCK) ss_table_kernel(const double* __restrict__ g, int n,
                                                            int len, int len_pad,
                                                            double* __restrict__ out_abs,
                                                            u32* __restrict__ out_rs) {
    extern __shared__ unsigned char smem[];
    double* keys = reinterpret_cast<double*>(smem);
    u32* vals = reinterpret_cast<u32*>(keys + len_pad);
    const int P = blockIdx.x;  // pair index q(q-1)/2 + p, p < q
    int q = 1;
    while ((q + 1) * q / 2 <= P) ++q;
    const int p = P - q * (q - 1) / 2;
    for (int t = threadIdx.x; t < len_pad; t += blockDim.x) {
        if (t < len) {
            int s = 1;
            while ((s + 1) * s / 2 <= t) ++s;
            int r = t - s * (s - 1) / 2;
            // map indices over the n-2 orbitals outside {p,q} to orbitals
            if (r >= p) ++r;
            if (r >= q) ++r;
            if (s >= p) ++s;
            if (s >= q) ++s;
            const double v = g[(((i64)r * n + p) * n + s) * n + q] - g[(((i64)r * n + q) * n + s) * n + p];
            keys[t] = fabs(v);
            vals[t] = (u32)r | ((u32)s << 8);
        } else {
            keys[t] = -1.0;
            vals[t] = 0xffffffffu;
        }
    }
    __syncthreads();
    bitonic_desc(keys, vals, len_pad);
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
        out_abs[(i64)P * len + t] = keys[t];
        out_rs[(i64)P * len + t] = vals[t];
    }
}

// Upper bound of |single element| for p -> r over every determinant:
// |h_rp| + sum_k |(rp|kk) - (rk|kp)| + sum_k |(rp|kk)|, padded against rounding.
__global__ void single_bound_kernel(const double* __restrict__ h, const double* __restrict__ jk,
                                    const double* __restrict__ jj, int n,
                                    double* __restrict__ bound) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const int p = t / n, r = t % n;
    double b = fabs(h[r * n + p]);
    for (int k = 0; k < n; ++k) {
        b += fabs(jk[((i64)r * n + p) * n + k]);
        b += fabs(jj[((i64)r * n + p) * n + k]);
    }
    bound[t] = b * (1.0 + 1e-10);
}

int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

void integrals_stage(hci_ctx_s* ctx, const double* h, const double* g, hipStream_t s) {
    Integrals& I = ctx->ints;
    const int n = ctx->n;
    I.n = n;
    const i64 n2 = (i64)n * n, n3 = n2 * n, n4 = n2 * n2;
    I.h = dev_alloc(ctx, sizeof(double) * n2, s);
    I.g = dev_alloc(ctx, sizeof(double) * n4, s);
    I.g32 = dev_alloc(ctx, sizeof(float) * n4, s);
    I.jk = dev_alloc(ctx, sizeof(double) * n3, s);
    I.jj = dev_alloc(ctx, sizeof(double) * n3, s);
    I.jk32 = dev_alloc(ctx, sizeof(float) * n3, s);
    I.jj32 = dev_alloc(ctx, sizeof(float) * n3, s);
    I.h32 = dev_alloc(ctx, sizeof(float) * n2, s);
    I.jdiag = dev_alloc(ctx, sizeof(double) * n2, s);
    I.kdiag = dev_alloc(ctx, sizeof(double) * n2, s);
    I.single_bound = dev_alloc(ctx, sizeof(double) * n2, s);
    HIP_CHECK(hipMemcpyAsync(I.h.ptr, h, sizeof(double) * n2, hipMemcpyDefault, s));
    HIP_CHECK(hipMemcpyAsync(I.g.ptr, g, sizeof(double) * n4, hipMemcpyDefault, s));
    HCI_LAUNCH(ctx, "to_f32", s, to_f32_kernel, ceil_div(n4, 256), 256, 0, I.g.as<double>(),
               I.g32.as<float>(), n4);
    HCI_LAUNCH(ctx, "integral_derived", s, derived_kernel, ceil_div(n3 > n2 ? n3 : n2, 256), 256, 0,
               I.g.as<double>(), I.h.as<double>(), n, I.jk.as<double>(), I.jj.as<double>(),
               I.jdiag.as<double>(), I.kdiag.as<double>(), I.jk32.as<float>(), I.jj32.as<float>(),
               I.h32.as<float>());
    HCI_LAUNCH(ctx, "single_bound", s, single_bound_kernel, ceil_div(n2, 256), 256, 0,
               I.h.as<double>(), I.jk.as<double>(), I.jj.as<double>(), n,
               I.single_bound.as<double>());
    // heat-bath lists
    I.os_len = (n - 1) * (n - 1);
    I.ss_len = n >= 4 ? (n - 2) * (n - 3) / 2 : 0;
    const int npair_os = n * n, npair_ss = n * (n - 1) / 2;
    if (I.os_len > 0) {
        const int lp = next_pow2(I.os_len);
        I.os_abs = dev_alloc(ctx, sizeof(double) * npair_os * (i64)I.os_len, s);
        I.os_rs = dev_alloc(ctx, sizeof(u32) * npair_os * (i64)I.os_len, s);
        HCI_LAUNCH(ctx, "hb_table_os", s, os_table_kernel, npair_os, TB_BLOCK,
                   lp * (sizeof(double) + sizeof(u32)), I.g.as<double>(), n, I.os_len, lp,
                   I.os_abs.as<double>(), I.os_rs.as<u32>());
    }
    if (I.ss_len > 0 && npair_ss > 0) {
        const int lp = next_pow2(I.ss_len);
        I.ss_abs = dev_alloc(ctx, sizeof(double) * npair_ss * (i64)I.ss_len, s);
        I.ss_rs = dev_alloc(ctx, sizeof(u32) * npair_ss * (i64)I.ss_len, s);
        HCI_LAUNCH(ctx, "hb_table_ss", s, ss_table_kernel, npair_ss, TB_BLOCK,
                   lp * (sizeof(double) + sizeof(u32)), I.g.as<double>(), n, I.ss_len, lp,
                   I.ss_abs.as<double>(), I.ss_rs.as<u32>());
    }
}
