// Lagrange multipliers of the HCISCF Lagrangian (eq. lagd / eq. lagc): with
// lambda_d = 0 the remaining condition is the z-vector equation
//   Q (H - E) Q z = -Q r,   Q = 1 - c c^T,   z orthogonal to c,
// where r = dF/dc (for the eps2-PT2 energy, r = dE2/dc at fixed E).  The
// projected operator is positive semidefinite on c-perp for the ground
// state, so it is solved by conjugate gradients with the projected Jacobi
// preconditioner
//   y = D^-1 x - D^-1 c (c^T D^-1 x) / (c^T D^-1 c),   D = diag(H) - E,
// which maps c-perp into c-perp.
//
// Precision HCI_FP32_MIXED runs the CG iterations on float32-mixed products
// and refines: each outer step recomputes the residual b - A z with float64
// products and solves for the correction to relative accuracy 1e-3, until
// the float64 residual meets tol * |b|.
#include "common.h"

namespace {

constexpr int ZB = 256;
constexpr int ZNBLK = 1024;

__global__ void __launch_bounds__(ZB) zdot_partial(const double* __restrict__ x,
                                                   const double* __restrict__ y, i64 n,
                                                   double* __restrict__ part) {
    __shared__ double lds[ZB / 64];
    double acc = 0.0;
    for (i64 i = (i64)blockIdx.x * ZB + threadIdx.x; i < n; i += (i64)gridDim.x * ZB) acc += x[i] * y[i];
    const double v = block_sum_f64<ZB>(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ void __launch_bounds__(ZB) zdot_final(const double* __restrict__ part, int m,
                                                 double* __restrict__ out) {
    __shared__ double lds[ZB / 64];
    double acc = 0.0;
    for (int k = threadIdx.x; k < m; k += ZB) acc += part[k];
    const double v = block_sum_f64<ZB>(acc, lds);
    if (threadIdx.x == 0) *out = v;
}

// y = a*x + b*y  (scalars on the host)
__global__ void zaxpby(double a, const double* __restrict__ x, double b, double* __restrict__ y, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}

// CG scalars on the device, so an iteration reads back only what its stop
// test needs: s[0] = rz, s[1] = p.q, s[2] = r.r, s[3] = rz', s[4] = alpha,
// s[5] = beta, s[6] = 1 when p.q <= 0 (alpha is then 0: x and r stay as they were)
__global__ void zcg_alpha(double* __restrict__ sc) {
    const bool ok = sc[1] > 0.0;
    sc[4] = ok ? sc[0] / sc[1] : 0.0;
    sc[6] = ok ? 0.0 : 1.0;
}
__global__ void zcg_beta(double* __restrict__ sc) {
    sc[5] = sc[3] / sc[0];
    sc[0] = sc[3];
}
// y = sgn * (*a) * x + y
__global__ void zaxpy_dev(const double* __restrict__ a, double sgn, const double* __restrict__ x,
                          double* __restrict__ y, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += sgn * (*a) * x[i];
}
// p = y + (*b) p
__global__ void zxpby_dev(const double* __restrict__ y, const double* __restrict__ b, double* __restrict__ p,
                          i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = y[i] + (*b) * p[i];
}

// out = x - (*cx) c   (projection with a device scalar)
__global__ void zproject(const double* __restrict__ x, const double* __restrict__ c,
                         const double* __restrict__ cx, double* __restrict__ out, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = x[i] - (*cx) * c[i];
}

// out = hx - e x
__global__ void zshift(const double* __restrict__ hx, const double* __restrict__ x, double e,
                       double* __restrict__ out, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = hx[i] - e * x[i];
}

__global__ void zdinv(const double* __restrict__ hd, double e, double* __restrict__ dinv, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        double den = hd[i] - e;
        if (fabs(den) < 1e-4) den = den < 0 ? -1e-4 : 1e-4;
        dinv[i] = 1.0 / den;
    }
}

__global__ void zmul(const double* __restrict__ a, const double* __restrict__ b,
                     double* __restrict__ out, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] * b[i];
}

// y = dinv*x - (*num / *den) dc   with dc = dinv*c
__global__ void zprecond_final(const double* __restrict__ dinv, const double* __restrict__ x,
                               const double* __restrict__ dc, const double* __restrict__ num,
                               const double* __restrict__ den, double* __restrict__ y, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = dinv[i] * x[i] - (*num / *den) * dc[i];
}

struct Vec {
    hci_ctx_s* ctx;
    hipStream_t s;
    i64 n;
    i64 g;
    DevMem part, scal;
    Vec(hci_ctx_s* c, i64 nn, hipStream_t st) : ctx(c), s(st), n(nn), g(ceil_div(nn, 256)) {
        part = dev_alloc(c, sizeof(double) * ZNBLK, st);
        scal = dev_alloc(c, sizeof(double) * 16, st);
    }
    double* sc(int k) { return scal.as<double>() + k; }
    void dot_dev(const double* x, const double* y, double* out) {
        const int nb = (int)std::min<i64>(ZNBLK, ceil_div(n, ZB));
        HCI_LAUNCH(ctx, "z_dot", s, zdot_partial, nb, ZB, 0, x, y, n, part.as<double>());
        HCI_LAUNCH(ctx, "z_dot", s, zdot_final, 1, ZB, 0, part.as<double>(), nb, out);
    }
    double dot(const double* x, const double* y) {
        dot_dev(x, y, sc(7));
        return read_scalar(sc(7), s);
    }
    void axpby(double a, const double* x, double b, double* y) {
        HCI_LAUNCH(ctx, "z_axpby", s, zaxpby, g, 256, 0, a, x, b, y, n);
    }
    // out = Q x
    void project(const double* x, const double* c, double* out) {
        dot_dev(c, x, sc(0));
        HCI_LAUNCH(ctx, "z_project", s, zproject, g, 256, 0, x, c, sc(0), out, n);
    }
};

}  // namespace

int zvector_solve(hci_ctx_s* ctx, Space* sp, const double* c, double e, const double* r, double* z,
                  double tol, int precision, int max_products, hipStream_t s) {
    const i64 N = sp->N;
    ensure_diag(ctx, sp, s);
    const double E = e - ctx->ecore;
    Vec v(ctx, N, s);
    DevMem buf = dev_alloc(ctx, sizeof(double) * 9 * N, s);
    double* b = buf.as<double>();
    double* res = b + N;
    double* x = b + 2 * N;   // inner solution (correction)
    double* rr = b + 3 * N;  // inner residual
    double* y = b + 4 * N;
    double* p = b + 5 * N;
    double* q = b + 6 * N;
    double* dinv = b + 7 * N;
    double* dc = b + 8 * N;
    const i64 g = ceil_div(N, 256);
    HCI_LAUNCH(ctx, "z_dinv", s, zdinv, g, 256, 0, sp->hdiag.as<double>(), E, dinv, N);
    HCI_LAUNCH(ctx, "z_mul", s, zmul, g, 256, 0, dinv, c, dc, N);
    v.dot_dev(c, dc, v.sc(2));  // c^T D^-1 c
    int products = 0;
    const int mode64 = choose_mode(ctx, sp, HCI_FP64, HCI_SIGMA_AUTO, s);
    const int mode32 = choose_mode(ctx, sp, HCI_FP32_MIXED, HCI_SIGMA_AUTO, s);
    // A x = Q (H x - E x)  for x in c-perp
    auto apply = [&](const double* xin, double* out, int prec) {
        sigma_apply(ctx, sp, xin, q, prec, prec == HCI_FP64 ? mode64 : mode32, s);
        ++products;
        HCI_LAUNCH(ctx, "z_shift", s, zshift, g, 256, 0, q, xin, E, q, N);
        v.project(q, c, out);
    };
    auto precond = [&](const double* xin, double* out) {
        v.dot_dev(dc, xin, v.sc(1));  // c^T D^-1 x
        HCI_LAUNCH(ctx, "z_precond", s, zprecond_final, g, 256, 0, dinv, xin, dc, v.sc(1), v.sc(2), out, N);
    };
    // b = -Q r
    v.project(r, c, b);
    HCI_LAUNCH(ctx, "z_axpby", s, zaxpby, g, 256, 0, 0.0, b, -1.0, b, N);
    const double bnorm = sqrt(std::max(v.dot(b, b), 0.0));
    HIP_CHECK(hipMemsetAsync(z, 0, sizeof(double) * N, s));
    if (bnorm == 0.0) return 0;
    const bool mixed = precision == HCI_FP32_MIXED;
    bool first = true;
    for (int outer = 0; outer < 50; ++outer) {
        // float64 residual of the current z
        if (first) {
            HIP_CHECK(hipMemcpyAsync(res, b, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        } else {
            apply(z, res, HCI_FP64);
            HCI_LAUNCH(ctx, "z_axpby", s, zaxpby, g, 256, 0, 1.0, b, -1.0, res, N);
        }
        first = false;
        const double rn = sqrt(std::max(v.dot(res, res), 0.0));
        if (rn <= tol * bnorm) return products;
        if (products >= max_products) break;
        // inner CG on A d = res
        const int inner_prec = mixed ? HCI_FP32_MIXED : HCI_FP64;
        const double target = mixed ? std::max(1e-3 * rn, 0.5 * tol * bnorm) : 0.5 * tol * bnorm;
        HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * N, s));
        HIP_CHECK(hipMemcpyAsync(rr, res, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        precond(rr, y);
        HIP_CHECK(hipMemcpyAsync(p, y, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        double* cg = v.sc(8);  // the CG scalars (zcg_alpha)
        v.dot_dev(rr, y, cg);
        for (int it = 0; it < 1000 && products < max_products; ++it) {
            apply(p, q, inner_prec);
            v.dot_dev(p, q, cg + 1);
            HCI_LAUNCH(ctx, "z_cg", s, zcg_alpha, 1, 1, 0, cg);
            HCI_LAUNCH(ctx, "z_axpby", s, zaxpy_dev, g, 256, 0, (const double*)(cg + 4), 1.0, (const double*)p, x, N);
            HCI_LAUNCH(ctx, "z_axpby", s, zaxpy_dev, g, 256, 0, (const double*)(cg + 4), -1.0, (const double*)q, rr, N);
            v.dot_dev(rr, rr, cg + 2);
            // the next direction is enqueued before the stop test is read back
            // (one read per iteration; the last direction is not used)
            precond(rr, y);
            v.dot_dev(rr, y, cg + 3);
            HCI_LAUNCH(ctx, "z_cg", s, zcg_beta, 1, 1, 0, cg);
            HCI_LAUNCH(ctx, "z_axpby", s, zxpby_dev, g, 256, 0, (const double*)y, (const double*)(cg + 5), p, N);
            double h[7];
            HIP_CHECK(hipMemcpyAsync(h, cg, sizeof(double) * 7, hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
            if (h[6] != 0.0) break;  // p.q <= 0: alpha was 0, x and r unchanged
            if (sqrt(std::max(h[2], 0.0)) <= target) break;
        }
        // z += Q x
        v.project(x, c, x);
        v.axpby(1.0, x, 1.0, z);
    }
    return -products;  // not converged
}
