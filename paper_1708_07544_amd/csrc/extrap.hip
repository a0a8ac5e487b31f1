// Extrapolation to the full-CI limit (Sec. "Results and discussion", the
// procedure of the butadiene calculations): after the largest HCI
// calculation, single-step calculations each drop a fraction of the least
// important determinants; E_var + E2 is fitted by a straight line in E2 and
// evaluated at E2 = 0.
//
// Importance is |c_i| of the given (largest) calculation: one ranking by
// decreasing |c_i|, ties by increasing index, so the levels are nested.  Level
// k keeps m_k = max(1, ceil(m_{k-1} (1 - fraction))) determinants (in their
// sorted order), solves for its lowest eigenpair (Davidson, warm start from
// the given c) and its screened E2 (deterministic, eps2).  The line is the
// least-squares fit over the levels; the error estimate is 25% of the
// distance from the extrapolated energy to the largest calculation's total.
#include <cmath>

#include "common.h"

namespace {

// sort key: decreasing |c| (the bit pattern of a non-negative double is
// monotone in its value), then increasing index
__global__ void rank_keys(const double* __restrict__ c, i64 N, u64* __restrict__ hi, u64* __restrict__ lo,
                          u32* __restrict__ idx) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    hi[i] = 0x7FFFFFFFFFFFFFFFull - (u64)__double_as_longlong(fabs(c[i]));
    lo[i] = (u64)i;
    idx[i] = (u32)i;
}

__global__ void rank_of(const u32* __restrict__ order, i64 N, u32* __restrict__ rank) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < N) rank[order[k]] = (u32)k;
}

__global__ void keep_flags(const u32* __restrict__ rank, i64 N, i64 m, u32* __restrict__ f) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) f[i] = (i64)rank[i] < m ? 1u : 0u;
    if (i == N) f[N] = 0u;
}

__global__ void compact_level(const u32* __restrict__ f, const u32* __restrict__ ex, i64 N,
                              const u64* __restrict__ dets, const double* __restrict__ c,
                              u64* __restrict__ odets, double* __restrict__ oc) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || f[i] == 0u) return;
    const i64 k = ex[i];
    odets[2 * k] = dets[2 * i];
    odets[2 * k + 1] = dets[2 * i + 1];
    oc[k] = c[i];
}

}  // namespace

void extrapolate(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, double fraction, int levels,
                 double eps2, double tol, int precision, i64* nvar, double* evar, double* e2, double* fit,
                 hipStream_t s) {
    // ranking by the given coefficients
    DevMem khi = dev_alloc(ctx, sizeof(u64) * N, s), klo = dev_alloc(ctx, sizeof(u64) * N, s);
    DevMem order = dev_alloc(ctx, sizeof(u32) * N, s);
    HCI_LAUNCH(ctx, "extrap_rank", s, rank_keys, ceil_div(N, 256), 256, 0, c, N, khi.as<u64>(), klo.as<u64>(),
               order.as<u32>());
    {
        DevMem thi = dev_alloc(ctx, sizeof(u64) * N, s), tlo = dev_alloc(ctx, sizeof(u64) * N, s);
        DevMem tv = dev_alloc(ctx, sizeof(u32) * N, s);
        radix_sort128(ctx, khi.as<u64>(), klo.as<u64>(), order.as<u32>(), thi.as<u64>(), tlo.as<u64>(),
                      tv.as<u32>(), N, 63, 32, s);
    }
    DevMem rank = dev_alloc(ctx, sizeof(u32) * N, s);
    HCI_LAUNCH(ctx, "extrap_rank", s, rank_of, ceil_div(N, 256), 256, 0, order.as<u32>(), N, rank.as<u32>());
    DevMem f = dev_alloc(ctx, sizeof(u32) * (N + 1), s), ex = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    i64 m = N;
    for (int k = 0; k < levels; ++k) {
        if (k > 0) m = std::max<i64>(1, (i64)std::ceil((double)m * (1.0 - fraction)));
        // this level's determinants (sorted order kept) and its warm start
        DevMem vd = dev_alloc(ctx, sizeof(u64) * 2 * m, s);
        DevMem vc = dev_alloc(ctx, sizeof(double) * m, s);
        HCI_LAUNCH(ctx, "extrap_level", s, keep_flags, ceil_div(N + 1, 256), 256, 0, rank.as<u32>(), N, m,
                   f.as<u32>());
        scan_u32_to_u32(ctx, f.as<u32>(), ex.as<u32>(), N + 1, s);
        HCI_LAUNCH(ctx, "extrap_level", s, compact_level, ceil_div(N, 256), 256, 0, f.as<u32>(), ex.as<u32>(), N,
                   dets, c, vd.as<u64>(), vc.as<double>());
        Space* sp = get_space(ctx, vd.as<u64>(), m, s);
        double e = 0.0;
        int iters = 0;
        const int rc = davidson_run(ctx, sp, vc.as<double>(), &e, tol, 100000, precision, HCI_SIGMA_AUTO, &iters, s);
        HCI_REQUIRE(rc == HCI_OK, rc, "extrapolation: Davidson did not converge at level " + std::to_string(k));
        nvar[k] = m;
        evar[k] = e;
        e2[k] = pt2_energy(ctx, vd.as<u64>(), m, vc.as<double>(), e - ctx->ecore, eps2, nullptr, nullptr, nullptr, s);
        drop_space(ctx);  // the level's list is freed next
    }
    // least-squares line E_var + E2 = a + b E2
    double xm = 0.0, ym = 0.0;
    for (int k = 0; k < levels; ++k) {
        xm += e2[k];
        ym += evar[k] + e2[k];
    }
    xm /= levels;
    ym /= levels;
    double sxy = 0.0, sxx = 0.0;
    for (int k = 0; k < levels; ++k) {
        sxy += (e2[k] - xm) * (evar[k] + e2[k] - ym);
        sxx += (e2[k] - xm) * (e2[k] - xm);
    }
    const double b = sxx > 0.0 ? sxy / sxx : 0.0;
    const double a = ym - b * xm;
    fit[0] = a;
    fit[1] = b;
    fit[2] = 0.25 * std::fabs(a - (evar[0] + e2[0]));
}
