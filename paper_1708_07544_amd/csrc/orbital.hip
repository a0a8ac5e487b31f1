// Orbital step for active-active rotations (Sec. "HCI self-consistent
// field": eq. lambda and eq. vdedk2 contract integral derivatives in the
// rotation parameters kappa with the density matrices).  With U = exp(kappa)
// (kappa antisymmetric), h' = U^T h U and (pq|rs)' = sum U_ap U_bq U_cr U_ds
// (ab|cd); for E = sum h gamma + 1/2 sum (pq|rs) Gamma the derivative is
//   dE/dkappa_xy = 2 (F_xy - F_yx),  F = h gamma + G,
//   G_xy = sum_qrs (xq|rs) Gamma_yqrs.
// Both are dense contractions and run on the float64 matrix cores
// (v_mfma_f64_16x16x4): G as an n x n^3 by n^3 x n product split over
// workgroups, the rotation as four quarter transforms, each an n^3 x n by
// n x n product that moves the transformed index to the back.
#include <map>
#include <mutex>

#include "common.h"

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// 16x16x4 float64 tile: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and receives D[l / 16 + 4 v][l % 16], v = 0..3 (checked on gfx950).
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int OB_BLOCK = 256;               // 4 wavefronts
constexpr int OB_WAVES = OB_BLOCK / HCI_WAVE;
constexpr int OB_MAXT = 4;                  // n <= 64: up to 4 tiles of 16

// out[j][i] = sum_k A[k][j] U[k][i] for j < J, i < n (A: [n][J], out: [J][n]).
// One wavefront per 16 consecutive j, every column tile of U.
__global__ void __launch_bounds__(OB_BLOCK) quarter_kernel(const double* __restrict__ A, i64 J, int n,
                                                           const double* __restrict__ U,
                                                           double* __restrict__ out) {
    const int lane = lane_id();
    const i64 j0 = ((i64)blockIdx.x * OB_WAVES + threadIdx.x / HCI_WAVE) * 16;
    if (j0 >= J) return;
    const int nt = (n + 15) / 16;
    const int lr = lane % 16, lk = lane / 16;
    const i64 ja = j0 + lr;
    v4d acc[OB_MAXT];
#pragma unroll
    for (int t = 0; t < OB_MAXT; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += 4) {
        const int k = k0 + lk;
        const double a = (k < n && ja < J) ? A[(i64)k * J + ja] : 0.0;
#pragma unroll
        for (int t = 0; t < OB_MAXT; ++t) {
            if (t < nt) {
                const int i = t * 16 + lr;
                const double b = (k < n && i < n) ? U[(i64)k * n + i] : 0.0;
                acc[t] = mfma16(a, b, acc[t]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < OB_MAXT; ++t) {
        if (t < nt) {
            const int i = t * 16 + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const i64 j = j0 + lk + 4 * v;
                if (j < J && i < n) out[j * n + i] = acc[t][v];
            }
        }
    }
}

// Partial sums of G_xy = sum_K g[x][K] Gamma[y][K] (K < n^3) over the chunks
// of 32 K of this workgroup: both 32-wide slices staged in LDS (rows padded
// to 33 doubles against bank conflicts), then every (x, y) tile on the matrix
// cores.  part[b][x][y], x, y < 64.
constexpr int GK = 32;
constexpr int GLD = GK + 1;

__global__ void __launch_bounds__(OB_BLOCK) gfock_partial_kernel(const double* __restrict__ g,
                                                                 const double* __restrict__ gam, int n,
                                                                 i64 K, i64 chunks_per_block,
                                                                 double* __restrict__ part) {
    __shared__ double sg[64 * GLD];
    __shared__ double sh[64 * GLD];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid / HCI_WAVE;
    const int nt = (n + 15) / 16;
    const int npair = nt * nt;
    const int lr = lane % 16, lk = lane / 16;
    v4d acc[4];  // pairs wave, wave + 4, ... (at most 16 pairs)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
    const i64 nchunk = (K + GK - 1) / GK;
    const i64 c0 = (i64)blockIdx.x * chunks_per_block;
    const i64 c1 = c0 + chunks_per_block < nchunk ? c0 + chunks_per_block : nchunk;
    for (i64 c = c0; c < c1; ++c) {
        const i64 kb = c * GK;
        __syncthreads();  // the previous slices are consumed
        for (int e = tid; e < 64 * GK; e += OB_BLOCK) {
            const int row = e / GK, col = e % GK;
            const i64 k = kb + col;
            const bool ok = row < n && k < K;
            sg[row * GLD + col] = ok ? g[(i64)row * K + k] : 0.0;
            sh[row * GLD + col] = ok ? gam[(i64)row * K + k] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int pr = wave + OB_WAVES * q;
            if (pr < npair) {
                const int tx = pr / nt, ty = pr % nt;
                for (int k0 = 0; k0 < GK; k0 += 4) {
                    const double a = sg[(tx * 16 + lr) * GLD + k0 + lk];
                    const double b = sh[(ty * 16 + lr) * GLD + k0 + lk];
                    acc[q] = mfma16(a, b, acc[q]);
                }
            }
        }
    }
    double* P = part + (i64)blockIdx.x * 64 * 64;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int pr = wave + OB_WAVES * q;
        if (pr < npair) {
            const int tx = pr / nt, ty = pr % nt;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int x = tx * 16 + lk + 4 * v, y = ty * 16 + lr;
                P[x * 64 + y] = acc[q][v];
            }
        }
    }
}

// F = h gamma + sum_b part[b] (fixed order), grad = 2 (F - F^T); one thread
// per (x, y), F of both orders computed by the same thread.
__global__ void gfock_finish_kernel(const double* __restrict__ part, int nblk, const double* __restrict__ h,
                                    const double* __restrict__ gamma1, int n, double* __restrict__ grad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int x = e / n, y = e % n;
    double fxy = 0.0, fyx = 0.0;
    for (int b = 0; b < nblk; ++b) {
        fxy += part[(i64)b * 4096 + x * 64 + y];
        fyx += part[(i64)b * 4096 + y * 64 + x];
    }
    for (int r = 0; r < n; ++r) {
        fxy += h[x * n + r] * gamma1[r * n + y];
        fyx += h[y * n + r] * gamma1[r * n + x];
    }
    grad[x * n + y] = 2.0 * (fxy - fyx);
}

// Partial-sum scratch of the allocation-free gradient entry point: one
// 64 x 64 float64 tile per workgroup of gfock_partial_kernel, at most
// ORB_SCRATCH_BLOCKS workgroups (the most that orbital_gradient's split uses
// for any n <= 64), 16 MiB per GPU, held until the process ends.  Host code
// never passes this name to a kernel: it is only the stand-in of the device
// symbol; the device address comes from hipGetSymbolAddress, per device.
constexpr i64 ORB_SCRATCH_BLOCKS = 512;
static __device__ __align__(256) double scratch[ORB_SCRATCH_BLOCKS * 4096];

// Workgroups of the gradient's K split: about 2 chunks of 32 K per
// workgroup, at most 512 workgroups (so the scratch above always suffices).
i64 gradient_split(int n, i64* per_out) {
    const i64 K = (i64)n * n * n;
    const i64 nchunk = ceil_div(K, GK);
    const i64 per = std::max<i64>(2, ceil_div(nchunk, 512));
    *per_out = per;
    return ceil_div(nchunk, per);
}

void quarter(hci_ctx_s* ctx, const double* A, i64 J, int n, const double* U, double* out, hipStream_t s) {
    const i64 waves = ceil_div(J, 16);
    HCI_LAUNCH(ctx, "orb_rotate", s, quarter_kernel, ceil_div(waves, OB_WAVES), OB_BLOCK, 0, A, J, n, U, out);
}

}  // namespace

namespace {

// The two launches of the gradient with the partial sums in `part`
// (nblk x 4096 float64, every entry the finish kernel reads is written by
// the partial kernel first, so nothing needs clearing).
void gradient_launch(hci_ctx_s* ctx, const double* rdm1, const double* rdm2, double* grad, double* part,
                     i64 nblk, i64 per, hipStream_t s) {
    const int n = ctx->n;
    const i64 K = (i64)n * n * n;
    HCI_LAUNCH(ctx, "orb_gradient", s, gfock_partial_kernel, nblk, OB_BLOCK, 0, ctx->ints.g.as<double>(), rdm2,
               n, K, per, part);
    HCI_LAUNCH(ctx, "orb_gradient", s, gfock_finish_kernel, ceil_div((i64)n * n, 256), 256, 0,
               (const double*)part, (int)nblk, ctx->ints.h.as<double>(), rdm1, n, grad);
}

// Device address of `scratch` on each device (resolved once per device).
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;

}  // namespace

void orbital_gradient(hci_ctx_s* ctx, const double* rdm1, const double* rdm2, double* grad, hipStream_t s) {
    i64 per = 0;
    const i64 nblk = gradient_split(ctx->n, &per);
    DevMem part = dev_alloc(ctx, sizeof(double) * 4096 * nblk, s);
    gradient_launch(ctx, rdm1, rdm2, grad, part.as<double>(), nblk, per, s);
}

void orbital_scratch_setup(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return;
    int cur = 0;
    HIP_CHECK(hipGetDevice(&cur));
    HCI_REQUIRE(cur == device, HCI_E_HIP, "scratch set-up: the context's device is not current");
    void* ptr = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    HCI_REQUIRE(ptr != nullptr, HCI_E_HIP, "scratch set-up: no device address for the gradient scratch");
    g_scratch_ptr[device] = static_cast<double*>(ptr);
}

void orbital_gradient_noalloc(hci_ctx_s* ctx, const double* rdm1, const double* rdm2, double* grad,
                              hipStream_t s) {
    i64 per = 0;
    const i64 nblk = gradient_split(ctx->n, &per);
    HCI_REQUIRE(nblk <= ORB_SCRATCH_BLOCKS, HCI_E_UNSUPPORTED,
                "the gradient needs " + std::to_string(nblk) + " partial tiles; the fixed scratch holds " +
                    std::to_string(ORB_SCRATCH_BLOCKS));
    double* part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        auto it = g_scratch_ptr.find(ctx->device);
        HCI_REQUIRE(it != g_scratch_ptr.end(), HCI_E_HIP, "scratch of this device was not set up");
        part = it->second;
    }
    gradient_launch(ctx, rdm1, rdm2, grad, part, nblk, per, s);
}

void rotate_integrals(hci_ctx_s* ctx, const double* U, double* h_out, double* g_out, hipStream_t s) {
    const int n = ctx->n;
    const i64 n2 = (i64)n * n, n3 = n2 * n, n4 = n3 * n;
    // h: two quarter steps (J = n); g: four (J = n^3), each moving the
    // transformed index to the back: (a,b,c,d) -> (b,c,d,p) -> ... -> (p,q,r,s)
    DevMem th = dev_alloc(ctx, sizeof(double) * n2, s);
    quarter(ctx, ctx->ints.h.as<double>(), n, n, U, th.as<double>(), s);
    quarter(ctx, th.as<double>(), n, n, U, h_out, s);
    DevMem t1 = dev_alloc(ctx, sizeof(double) * n4, s), t2 = dev_alloc(ctx, sizeof(double) * n4, s);
    quarter(ctx, ctx->ints.g.as<double>(), n3, n, U, t1.as<double>(), s);
    quarter(ctx, t1.as<double>(), n3, n, U, t2.as<double>(), s);
    quarter(ctx, t2.as<double>(), n3, n, U, t1.as<double>(), s);
    quarter(ctx, t1.as<double>(), n3, n, U, g_out, s);
}
