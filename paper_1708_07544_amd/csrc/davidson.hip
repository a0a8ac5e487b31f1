// Davidson eigensolver for the lowest eigenpair of H on V: it minimises
// <Psi|H|Psi> - E(<Psi|Psi> - 1) over the coefficients (eq. variational).
//
// All vector algebra is float64 on the device with fixed-order reductions:
// subspace basis V_k and products W_k = H V_k, Gram matrix G = V^T W grown
// one column per iteration, lowest Ritz pair of G by cyclic Jacobi in one
// wavefront, residual r = W y - theta V y, diagonal preconditioner
// r_i / (H_ii - theta) (guarded), two rounds of classical Gram-Schmidt.
// The host only reads (theta, |r|^2) once per iteration.
//
// Precision HCI_FP32_MIXED: iterate with the mixed product (float32 elements
// times a float32 copy of the vector, float64 row sums) until the residual is
// below max(tol, 1e-7 |theta|) (the float32 operator is not more accurate than
// that), then restart from the Ritz vector with float64 products until the
// float64 residual meets tol.  Restarts keep the current and the previous
// Ritz vectors.
//
// Several states (deflation): with nlock converged orthonormal vectors L
// given, the solver works on Q H Q restricted to the complement of L
// (Q = 1 - L L^T): every new basis vector is orthogonalised against L before
// the basis, and every product H v is projected by Q.  Its lowest eigenpair
// there is the next state, and its residual is orthogonal to L.  For several
// states every start vector gets a small fixed pseudo-random component, so
// that the lowest state of the complement is reached whatever its symmetry.
#include <atomic>
#include <cfloat>
#include <chrono>
#include <cstdlib>

#include "common.h"

namespace {

constexpr int DV_BLOCK = 256;
constexpr int DV_MAXK = 32;   // capacity of the small dense arrays
constexpr int DV_KMAX = 32;   // subspace size before a thick restart

// partial[j * nblk + b] = sum over the block's rows of X_j[i] * t[i], j < k
__global__ void __launch_bounds__(DV_BLOCK) dots_kernel(const double* __restrict__ X, i64 ld, int k,
                                                        const double* __restrict__ t, i64 N,
                                                        double* __restrict__ partial, int nblk) {
    double acc[DV_MAXK];
#pragma unroll
    for (int j = 0; j < DV_MAXK; ++j) acc[j] = 0.0;
    for (i64 i = (i64)blockIdx.x * DV_BLOCK + threadIdx.x; i < N; i += (i64)nblk * DV_BLOCK) {
        const double ti = t[i];
#pragma unroll
        for (int j = 0; j < DV_MAXK; ++j)
            if (j < k) acc[j] += X[(i64)j * ld + i] * ti;
    }
    // wavefront sums of every column, one exchange through LDS, then a
    // fixed-order sum over the block's wavefronts
    __shared__ double wsum[DV_BLOCK / 64][DV_MAXK];
    const int w = threadIdx.x / 64;
#pragma unroll
    for (int j = 0; j < DV_MAXK; ++j) {
        if (j < k) {
            const double v = wave_sum_f64(acc[j]);
            if (lane_id() == 0) wsum[w][j] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < k) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < DV_BLOCK / 64; ++q) v += wsum[q][threadIdx.x];
        partial[(i64)threadIdx.x * nblk + blockIdx.x] = v;
    }
}

// out[j * ostride] = sum_b partial[j * nblk + b] (fixed order), or, when out0
// is given, column 0 to *out0 and column j > 0 to out[(j - 1) * ostride];
// block 0 also copies *copy_src to *copy_dst when given (scalars the host
// reads together).  (A last-block reduction inside the producing kernels was
// tried: the device-scope fence each block then needs before its ticket costs
// ~0.1 ms per kernel on this GPU, more than the separate launch.)
// With host given, block 0 then copies the four scalars out0[0..4) into
// host[0..4) (pinned, coherent host memory) and, after a system-scope fence,
// writes seq into host[4] for the host to poll.
__global__ void reduce_partials_kernel(const double* __restrict__ partial, int k, int nblk,
                                       double* __restrict__ out, i64 ostride,
                                       const double* __restrict__ copy_src, double* copy_dst,
                                       double* out0, double* host, unsigned long long seq) {
    __shared__ double lds[DV_BLOCK / 64];
    const int j = blockIdx.x;
    if (j >= k) return;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += DV_BLOCK) acc += partial[(i64)j * nblk + b];
    const double v = block_sum_f64<DV_BLOCK>(acc, lds);
    if (threadIdx.x == 0) {
        if (out0 == nullptr) out[(i64)j * ostride] = v;
        else if (j == 0) *out0 = v;
        else out[(i64)(j - 1) * ostride] = v;
        if (j == 0 && copy_dst) *copy_dst = *copy_src;
        if (j == 0 && host != nullptr) {
            const volatile double* src = out0;  // (this thread wrote out0[0] and out0[3])
            for (int q = 0; q < 4; ++q) host[q] = src[q];
            __threadfence_system();
            *reinterpret_cast<volatile unsigned long long*>(host + 4) = seq;
        }
    }
}

// One classical Gram-Schmidt sweep fused with what follows it:
// t -= sum_j coef[j] X_j, then (NORM) the partial sums of |t|^2, else those of
// X_j . t (the next sweep's coefficients), with the partition and order of
// dots_kernel.
template <bool NORM>
__global__ void __launch_bounds__(DV_BLOCK) sub_dots_kernel(const double* __restrict__ X, i64 ld, int k,
                                                            const double* __restrict__ coef,
                                                            double* __restrict__ t, i64 N,
                                                            double* __restrict__ partial, int nblk) {
    __shared__ double cf[DV_MAXK];
    __shared__ double wsum[DV_BLOCK / 64][DV_MAXK];
    if ((int)threadIdx.x < k) cf[threadIdx.x] = coef[threadIdx.x];
    __syncthreads();
    constexpr int NACC = NORM ? 1 : DV_MAXK;
    double acc[NACC];
#pragma unroll
    for (int j = 0; j < NACC; ++j) acc[j] = 0.0;
    for (i64 i = (i64)blockIdx.x * DV_BLOCK + threadIdx.x; i < N; i += (i64)nblk * DV_BLOCK) {
        double si = t[i];
        for (int j = 0; j < k; ++j) si -= cf[j] * X[(i64)j * ld + i];
        t[i] = si;
        if constexpr (NORM) {
            acc[0] += si * si;
        } else {
#pragma unroll
            for (int j = 0; j < DV_MAXK; ++j)
                if (j < k) acc[j] += X[(i64)j * ld + i] * si;
        }
    }
    const int kk = NORM ? 1 : k;
    const int w = threadIdx.x / 64;
#pragma unroll
    for (int j = 0; j < NACC; ++j) {
        if (j < kk) {
            const double v = wave_sum_f64(acc[j]);
            if (lane_id() == 0) wsum[w][j] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < kk) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < DV_BLOCK / 64; ++q) v += wsum[q][threadIdx.x];
        partial[(i64)threadIdx.x * nblk + blockIdx.x] = v;
    }
}

// dst = src / sqrt(*nrm2)
__global__ void normalize_kernel(const double* __restrict__ src, const double* __restrict__ nrm2,
                                 double* __restrict__ dst, i64 N) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) dst[i] = src[i] / sqrt(*nrm2);
}

// Normalise a new search direction without a host round trip: a direction
// with no norm left after orthogonalisation becomes the zero vector and
// raises *dead (the projected eigensolver then ignores it and the host
// restarts at its next synchronisation).
__global__ void normalize_guard_kernel(const double* __restrict__ src, const double* __restrict__ nrm2,
                                       double* __restrict__ dst, i64 N, double* __restrict__ dead) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const double nn = *nrm2;
    const bool ok = nn > 1e-28;
    if (i < N) dst[i] = ok ? src[i] / sqrt(nn) : 0.0;
    if (i == 0 && !ok) *dead = 1.0;
}

// x = V y, w = W y, r = w - theta x, t = r / guard(H_ii - theta); partial
// sums of |r|^2 (column 0) and, for kd > 0, of the first Gram-Schmidt
// sweep's coefficients V_j . t, j < kd (columns 1..kd, with the partition and
// order of dots_kernel).  ritz[0] = theta, ritz[1..k] = y.
__global__ void __launch_bounds__(DV_BLOCK) combine_kernel(
    const double* __restrict__ V, const double* __restrict__ W, i64 ld, int k, int kd,
    const double* __restrict__ ritz, const double* __restrict__ hd, double* __restrict__ x,
    double* __restrict__ w, double* __restrict__ t, i64 N, double* __restrict__ partial, int nblk) {
    __shared__ double wsum[DV_BLOCK / 64][DV_MAXK];
    __shared__ double y[DV_MAXK + 1];
    if (threadIdx.x <= k) y[threadIdx.x] = ritz[threadIdx.x];
    __syncthreads();
    const double theta = y[0];
    double acc[DV_MAXK];  // acc[0] = |r|^2, acc[1 + j] = V_j . t
#pragma unroll
    for (int j = 0; j < DV_MAXK; ++j) acc[j] = 0.0;
    for (i64 i = (i64)blockIdx.x * DV_BLOCK + threadIdx.x; i < N; i += (i64)nblk * DV_BLOCK) {
        double xi = 0.0, wi = 0.0;
        for (int j = 0; j < k; ++j) {
            xi += y[j + 1] * V[(i64)j * ld + i];
            wi += y[j + 1] * W[(i64)j * ld + i];
        }
        const double ri = wi - theta * xi;
        double den = hd[i] - theta;
        if (fabs(den) < 1e-4) den = den < 0 ? -1e-4 : 1e-4;
        const double ti = ri / den;
        x[i] = xi;
        w[i] = wi;
        t[i] = ti;
        acc[0] += ri * ri;
        // V_j[i] again: the line was just read by this thread (a cache hit)
#pragma unroll
        for (int j = 0; j + 1 < DV_MAXK; ++j)
            if (j < kd) acc[j + 1] += V[(i64)j * ld + i] * ti;
    }
    const int wv = threadIdx.x / 64;
#pragma unroll
    for (int j = 0; j < DV_MAXK; ++j) {
        if (j <= kd) {
            const double v = wave_sum_f64(acc[j]);
            if (lane_id() == 0) wsum[wv][j] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x <= kd) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < DV_BLOCK / 64; ++q) v += wsum[q][threadIdx.x];
        partial[(i64)threadIdx.x * nblk + blockIdx.x] = v;
    }
}

// Lowest eigenpair of the k x k projected matrix (upper triangle of G),
// one wavefront: Householder reduction to tridiagonal form, the lowest
// eigenvalue of the tridiagonal matrix by Sturm-count multisection (64 shifts
// per round), its eigenvector by two steps of inverse iteration (LDL^T
// factorisation shifted just below the eigenvalue), back-transformation, and
// the Rayleigh quotient with the original matrix.  out = {theta, y[0..k)}.
__device__ __forceinline__ double wave_min_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__global__ void __launch_bounds__(64) lowest_eig_kernel(const double* __restrict__ G, int ldg,
                                                        int kall, const double* __restrict__ dead,
                                                        double* __restrict__ out) {
    // a dead newest direction (zero vector) is left out of the eigenproblem
    const int k = (dead != nullptr && *dead != 0.0) ? kall - 1 : kall;
    __shared__ double A[DV_MAXK][DV_MAXK + 1];
    __shared__ double A0[DV_MAXK][DV_MAXK + 1];  // the matrix itself, for the Rayleigh quotient
    __shared__ double H[DV_MAXK][DV_MAXK];  // Householder vector of step j in row j
    __shared__ double vv[DV_MAXK], pw[DV_MAXK], d[DV_MAXK], e[DV_MAXK], y[DV_MAXK];
    const int l = threadIdx.x;
    static_assert(DV_MAXK == 32, "entries of the projected matrix are addressed as r * 32 + c");
    {  // every load in flight before the first store
        constexpr int PER = DV_MAXK * DV_MAXK / 64;
        double g[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int x = l + 64 * u;
            const int r = x >> 5, c = x & 31;
            g[u] = r < k && c < k ? G[(r < c ? r : c) * ldg + (r < c ? c : r)] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int x = l + 64 * u;
            const int r = x >> 5, c = x & 31;
            if (r < k && c < k) {
                A[r][c] = g[u];
                A0[r][c] = g[u];
            }
        }
    }
    __syncthreads();
    // Householder: column j's entries below the subdiagonal are annihilated
    for (int j = 0; j + 2 < k; ++j) {
        const int m = k - j - 1;  // trailing rows j+1 .. k-1
        const double xi = l < m ? A[j + 1 + l][j] : 0.0;
        const double nrm2 = wave_sum_f64(xi * xi);
        if (nrm2 == 0.0) {  // already reduced: identity reflector
            if (l < m) H[j][l] = 0.0;
            __syncthreads();
            continue;
        }
        const double x0 = __shfl(xi, 0, 64);
        const double alpha = x0 >= 0.0 ? -sqrt(nrm2) : sqrt(nrm2);
        double vi = l < m ? xi - (l == 0 ? alpha : 0.0) : 0.0;
        const double vn = sqrt(wave_sum_f64(vi * vi));
        vi /= vn;
        if (l < m) {
            H[j][l] = vi;
            vv[l] = vi;
        }
        __syncthreads();
        // p = A v: row l & 31 by lanes l and l + 32, each over half the columns
        const int pr = l & 31, half = l >> 5;
        double pi = 0.0;
        if (pr < m)
            for (int c = half; c < m; c += 2) pi += A[j + 1 + pr][j + 1 + c] * vv[c];
        pi += __shfl_xor(pi, 32, 64);
        if (l >= 32) pi = 0.0;
        const double K = wave_sum_f64(vi * pi);
        if (l < m) pw[l] = pi - K * vi;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < DV_MAXK * DV_MAXK / 64; ++u) {
            const int x = l + 64 * u;
            const int r = x >> 5, c = x & 31;
            if (r < m && c < m) A[j + 1 + r][j + 1 + c] -= 2.0 * (vv[r] * pw[c] + pw[r] * vv[c]);
        }
        if (l == 0) {
            A[j + 1][j] = alpha;
            A[j][j + 1] = alpha;
        }
        __syncthreads();
    }
    if (l < k) {
        d[l] = A[l][l];
        e[l] = l + 1 < k ? A[l + 1][l] : 0.0;
    }
    __syncthreads();
    // Gershgorin interval of the tridiagonal matrix
    double glo = 1e300, ghi = -1e300, scale = 0.0;
    if (l < k) {
        const double r = fabs(e[l]) + (l > 0 ? fabs(e[l - 1]) : 0.0);
        glo = d[l] - r;
        ghi = d[l] + r;
        scale = fabs(d[l]) + r;
    }
    double lo = wave_min_f64(glo), hi = wave_max_f64(ghi);
    scale = wave_max_f64(scale);
    const double pivmin = 1e-300 + 1e-30 * scale * scale;
    // multisection: lane l tests the shift lo + (hi - lo)(l + 1)/65
    for (int round = 0; round < 16; ++round) {
        if (!(hi - lo > 4.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)))) break;
        const double xl = lo + (hi - lo) * (double)(l + 1) / 65.0;
        int cnt = 0;
        double q = 1.0;
        for (int i = 0; i < k; ++i) {
            q = d[i] - xl - (i > 0 ? e[i - 1] * e[i - 1] / q : 0.0);
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += q < 0.0;
        }
        const u64 mask = ballot(cnt >= 1);
        if (mask == 0) {
            lo = __shfl(xl, 63, 64);
        } else {
            const int f = ctz64(mask);
            const double xf = __shfl(xl, f, 64);
            const double xp = __shfl(xl, f > 0 ? f - 1 : 0, 64);
            hi = xf;
            if (f > 0) lo = xp;
        }
    }
    // inverse iteration with T - mu I positive definite (mu just below lambda)
    if (l == 0) {  // LDL^T pivots in vv, multipliers in pw, iterate in y
        const double mu = lo - 4.0 * DBL_EPSILON * fmax(fabs(lo), scale);
        vv[0] = fmax(d[0] - mu, pivmin);
        for (int i = 1; i < k; ++i) {
            pw[i] = e[i - 1] / vv[i - 1];
            vv[i] = fmax(d[i] - mu - pw[i] * e[i - 1], pivmin);
        }
        for (int i = 0; i < k; ++i) y[i] = 1.0;
        for (int it = 0; it < 2; ++it) {
            for (int i = 1; i < k; ++i) y[i] -= pw[i] * y[i - 1];
            for (int i = 0; i < k; ++i) y[i] /= vv[i];
            for (int i = k - 2; i >= 0; --i) y[i] -= pw[i + 1] * y[i + 1];
            double nn = 0.0;
            for (int i = 0; i < k; ++i) nn += y[i] * y[i];
            nn = 1.0 / sqrt(nn);
            for (int i = 0; i < k; ++i) y[i] *= nn;
        }
    }
    __syncthreads();
    // back-transformation y <- H_0 ... H_{k-3} y
    for (int j = k - 3; j >= 0; --j) {
        const int m = k - j - 1;
        const double hv = l < m ? H[j][l] : 0.0;
        const double yv = l < m ? y[j + 1 + l] : 0.0;
        const double dot = wave_sum_f64(hv * yv);
        if (l < m) y[j + 1 + l] = yv - 2.0 * dot * hv;
        __syncthreads();
    }
    // Rayleigh quotient with the original matrix
    const double yl = l < k ? y[l] : 0.0;
    double ay = 0.0;
    if (l < k)
        for (int c = 0; c < k; ++c) ay += A0[l][c] * y[c];
    const double nrm = wave_sum_f64(yl * yl);
    const double th = wave_sum_f64(yl * ay) / nrm;
    if (l == 0) out[0] = th;
    if (l < k) out[1 + l] = yl / sqrt(nrm);
    if (l >= k && l < kall) out[1 + l] = 0.0;
}

__global__ void argmin_seed_kernel(const double* __restrict__ hd, i64 N, double* __restrict__ x) {
    // one block: index of the smallest diagonal (first on ties), then x = e_idx
    __shared__ double bv[256];
    __shared__ i64 bi[256];
    double v = 1e300;
    i64 idx = 0;
    for (i64 i = threadIdx.x; i < N; i += 256)
        if (hd[i] < v) {
            v = hd[i];
            idx = i;
        }
    bv[threadIdx.x] = v;
    bi[threadIdx.x] = idx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double ov = bv[threadIdx.x + s];
            const i64 oi = bi[threadIdx.x + s];
            if (ov < bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = ov;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    for (i64 i = threadIdx.x; i < N; i += 256) x[i] = (i == bi[0]) ? 1.0 : 0.0;
}

// Start vector for a deflated solve: e_j for the determinant of lowest
// diagonal among those that the locked vectors hold less than half of
// (w_j = sum_l L_lj^2 <= 1/2), else the one they hold least (first index on
// ties).  At most 2 nlock determinants have w_j > 1/2, so with N >= 2 nlock
// the first rule always applies; e_j is never inside the span of L.
__device__ __forceinline__ bool seed_less(int fa, double va, i64 ia, int fb, double vb, i64 ib) {
    if (fa != fb) return fa < fb;
    if (va != vb) return va < vb;
    return ia < ib;
}

__global__ void __launch_bounds__(256) deflated_seed_kernel(const double* __restrict__ hd, i64 N,
                                                            const double* __restrict__ L, int nlock,
                                                            double* __restrict__ x) {
    __shared__ int bf[256];
    __shared__ double bv[256];
    __shared__ i64 bi[256];
    int f = 2;
    double v = 0.0;
    i64 idx = 0;
    for (i64 i = threadIdx.x; i < N; i += 256) {
        double w = 0.0;
        for (int l = 0; l < nlock; ++l) w += L[(i64)l * N + i] * L[(i64)l * N + i];
        const int fi = w > 0.5 ? 1 : 0;
        const double vi = fi ? w : hd[i];
        if (seed_less(fi, vi, i, f, v, idx)) {
            f = fi;
            v = vi;
            idx = i;
        }
    }
    bf[threadIdx.x] = f;
    bv[threadIdx.x] = v;
    bi[threadIdx.x] = idx;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            const int o = threadIdx.x + st;
            if (seed_less(bf[o], bv[o], bi[o], bf[threadIdx.x], bv[threadIdx.x], bi[threadIdx.x])) {
                bf[threadIdx.x] = bf[o];
                bv[threadIdx.x] = bv[o];
                bi[threadIdx.x] = bi[o];
            }
        }
        __syncthreads();
    }
    for (i64 i = threadIdx.x; i < N; i += 256) x[i] = (i == bi[0]) ? 1.0 : 0.0;
}

// x += delta z with z_i uniform in [-1, 1) from the splitmix64 generator
// (Steele, Lea and Flood, OOPSLA 2014) at counter i, and |delta z| about
// 1e-3 |x| (E z_i^2 = 1/3).  A start vector confined to one symmetry sector
// of H (even or odd under the exchange of alpha and beta strings when
// N_alpha = N_beta, for instance) otherwise only reaches other sectors
// through rounding errors.
__device__ __forceinline__ u64 splitmix64_at(u64 i) {
    u64 z = (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void generic_start_kernel(double* __restrict__ x, i64 N, const double* __restrict__ nrm2) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double delta = 1e-3 * sqrt(3.0 * *nrm2 / (double)N);
    const double z = (double)(splitmix64_at((u64)i) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    x[i] += delta * z;
}

// Sign convention: the first entry whose magnitude is within SIGN_TIE
// (relative) of the largest is made positive.  Entries equal in exact
// arithmetic (symmetry-related determinants) come out of a converged solve
// equal only to about the solve's accuracy, so the band is wide enough that
// they tie and the sign does not depend on rounding.  Block partials of
// max |x_i|, a one-block maximum, block partials of the first index inside
// the band, a one-block decision, then a grid-wide multiply by +-1.
constexpr double SIGN_TIE = 1e-6;

__global__ void __launch_bounds__(256) absmax_partial_kernel(const double* __restrict__ x, i64 N,
                                                             double* __restrict__ pv) {
    __shared__ double bv[256];
    double v = 0.0;
    for (i64 i = (i64)blockIdx.x * 256 + threadIdx.x; i < N; i += (i64)gridDim.x * 256) v = fmax(v, fabs(x[i]));
    bv[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) bv[threadIdx.x] = fmax(bv[threadIdx.x], bv[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) pv[blockIdx.x] = bv[0];
}

// first index i with |x_i| >= (1 - SIGN_TIE) max|x| (max from the partials)
__global__ void __launch_bounds__(256) tie_index_partial_kernel(const double* __restrict__ x, i64 N,
                                                                const double* __restrict__ pv, int nblk,
                                                                i64* __restrict__ pi) {
    __shared__ double bm[256];
    __shared__ i64 bi[256];
    double m = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) m = fmax(m, pv[b]);
    bm[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) bm[threadIdx.x] = fmax(bm[threadIdx.x], bm[threadIdx.x + st]);
        __syncthreads();
    }
    const double band = bm[0] * (1.0 - SIGN_TIE);
    i64 idx = N;
    for (i64 i = (i64)blockIdx.x * 256 + threadIdx.x; i < N && idx == N; i += (i64)gridDim.x * 256)
        if (fabs(x[i]) >= band) idx = i;
    bi[threadIdx.x] = idx;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) bi[threadIdx.x] = min(bi[threadIdx.x], bi[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) pi[blockIdx.x] = bi[0];
}

__global__ void __launch_bounds__(256) sign_decide_kernel(const double* __restrict__ x, i64 N,
                                                          const i64* __restrict__ pi, int nblk,
                                                          double* __restrict__ factor) {
    __shared__ i64 bi[256];
    i64 idx = N;
    for (int b = threadIdx.x; b < nblk; b += 256) idx = min(idx, pi[b]);
    bi[threadIdx.x] = idx;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) bi[threadIdx.x] = min(bi[threadIdx.x], bi[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *factor = (bi[0] < N && x[bi[0]] < 0.0) ? -1.0 : 1.0;
}

__global__ void scale_kernel(double* __restrict__ x, i64 N, const double* __restrict__ factor) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) x[i] *= *factor;
}

struct Workspace {
    hci_ctx_s* ctx;
    hipStream_t s;
    i64 N;
    int nblk;
    DevMem partial, scal;
    Workspace(hci_ctx_s* c, i64 n, hipStream_t st) : ctx(c), s(st), N(n) {
        nblk = (int)std::min<i64>(ceil_div(n, DV_BLOCK), 1024);
        partial = dev_alloc(c, sizeof(double) * DV_MAXK * nblk, st);
        scal = dev_alloc(c, sizeof(double) * (DV_MAXK + 8), st);
    }
    // out[j * ostride] = X_j . t, j < k
    void dots(const double* X, i64 ld, int k, const double* t, double* out, i64 ostride = 1) {
        HCI_LAUNCH(ctx, "dv_dots", s, dots_kernel, nblk, DV_BLOCK, 0, X, ld, k, t, N,
                   partial.as<double>(), nblk);
        reduce(k, out, ostride);
    }
    void reduce(int k, double* out, i64 ostride = 1, const double* copy_src = nullptr,
                double* copy_dst = nullptr, double* out0 = nullptr, double* host = nullptr,
                unsigned long long seq = 0) {
        HCI_LAUNCH(ctx, "dv_reduce", s, reduce_partials_kernel, k, DV_BLOCK, 0, partial.as<double>(),
                   k, nblk, out, ostride, copy_src, copy_dst, out0, host, seq);
    }
    // two-sweep classical Gram-Schmidt of t against X_0..X_{k-1}; nrm2 = |t|^2
    void cgs2(const double* X, i64 ld, int k, double* t, double* coef, double* nrm2) {
        dots(X, ld, k, t, coef);
        cgs2_after_dots(X, ld, k, t, coef, nrm2);
    }
    // the same with coef = X^T t already computed
    void cgs2_after_dots(const double* X, i64 ld, int k, double* t, double* coef, double* nrm2) {
        HCI_LAUNCH(ctx, "dv_subcombo", s, sub_dots_kernel<false>, nblk, DV_BLOCK, 0, X, ld, k,
                   (const double*)coef, t, N, partial.as<double>(), nblk);
        reduce(k, coef);
        HCI_LAUNCH(ctx, "dv_subcombo", s, sub_dots_kernel<true>, nblk, DV_BLOCK, 0, X, ld, k,
                   (const double*)coef, t, N, partial.as<double>(), nblk);
        reduce(1, nrm2);
    }
    // w -= L L^T w (one sweep: w is H v with v orthogonal to L, so its
    // component along L is of the order of the locked residuals)
    void project(const double* L, int nl, double* w, double* coef) {
        if (nl == 0) return;
        dots(L, N, nl, w, coef);
        HCI_LAUNCH(ctx, "dv_deflate", s, sub_dots_kernel<true>, nblk, DV_BLOCK, 0, L, N, nl,
                   (const double*)coef, w, N, partial.as<double>(), nblk);
    }
};

// The four scalars {|r|^2, |t|^2, dead, theta} of the iteration whose
// reduction was given sequence number seq: poll the pinned words for up to
// poll_ms (a long product ahead of them), then wait on the stream instead.
void wait_host_scalars(hci_ctx_s* ctx, unsigned long long seq, hipStream_t s, double* hv, int poll_ms) {
    const volatile unsigned long long* flag =
        reinterpret_cast<const volatile unsigned long long*>(ctx->host_scal + 4);
    if (*flag != seq && poll_ms > 0) {
        const auto t0 = std::chrono::steady_clock::now();
        for (unsigned spins = 1; *flag != seq; ++spins)
            if ((spins & 1023u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(poll_ms))
                break;
    }
    if (*flag != seq) {
        HIP_CHECK(hipStreamSynchronize(s));
        HCI_REQUIRE(*flag == seq, HCI_E_HIP, "internal: Davidson scalars were not written");
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    const volatile double* h = ctx->host_scal;
    for (int q = 0; q < 4; ++q) hv[q] = h[q];
}

}  // namespace

int davidson_run(hci_ctx_s* ctx, Space* sp, double* c, double* e_out, double tol, int max_iter,
                 int precision, int mode, int* iters_out, hipStream_t s, const double* lock, int nlock,
                 bool generic_start) {
    const i64 N = sp->N;
    HCI_REQUIRE(nlock >= 0 && nlock < DV_MAXK && nlock < N && (nlock == 0 || lock != nullptr), HCI_E_ARG,
                "bad number of locked vectors");
    ensure_diag(ctx, sp, s);
    const double* hd = sp->hdiag.as<double>();
    const int kmax = (int)std::min<i64>(DV_KMAX, N - nlock);
    Workspace ws(ctx, N, s);
    DevMem Vb = dev_alloc(ctx, sizeof(double) * kmax * N, s);
    DevMem Wb = dev_alloc(ctx, sizeof(double) * kmax * N, s);
    DevMem G = dev_alloc(ctx, sizeof(double) * DV_MAXK * DV_MAXK, s);
    DevMem ritz = dev_alloc(ctx, sizeof(double) * (DV_MAXK + 1), s);
    DevMem vec = dev_alloc(ctx, sizeof(double) * 5 * N, s);
    double* V = Vb.as<double>();
    double* W = Wb.as<double>();
    // current Ritz pair (xc, wc = H xc), previous one, and the correction
    double* xc = vec.as<double>();
    double* wc = xc + N;
    double* xp = xc + 2 * N;
    double* wp = xc + 3 * N;
    double* t = xc + 4 * N;
    double* sc = ws.scal.as<double>();  // sc[0..DV_MAXK) coefficients, then scalars below
    double* nrm_x = sc + DV_MAXK;
    double* rr = sc + DV_MAXK + 1;
    double* nrm_t = sc + DV_MAXK + 2;
    double* dead = sc + DV_MAXK + 3;
    double* theta_h = sc + DV_MAXK + 4;  // rr, nrm_t, dead, theta: read back together
    HIP_CHECK(hipMemsetAsync(dead, 0, sizeof(double), s));
    const i64 g1 = ceil_div(N, 256);
    // how long the host polls for an iteration's scalars before it waits on
    // the stream (HCI_DAVIDSON_POLL_MS, default 200; 0 always waits)
    const char* poll_env = std::getenv("HCI_DAVIDSON_POLL_MS");
    const int poll_ms = poll_env ? std::max(0, std::atoi(poll_env)) : 200;
    if (!ctx->host_scal) {
        void* hp = nullptr;
        HIP_CHECK(hipHostMalloc(&hp, 8 * sizeof(double), hipHostMallocCoherent));
        ctx->host_scal = static_cast<double*>(hp);
        *reinterpret_cast<volatile unsigned long long*>(ctx->host_scal + 4) = 0ull;
    }

    // start vector (a zero vector selects the lowest diagonal determinant);
    // deflated: its part outside the locked vectors, or a seed when nothing
    // of it is left
    HIP_CHECK(hipMemcpyAsync(xc, c, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    ws.dots(xc, N, 1, xc, nrm_x);
    if (nlock == 0) {
        if (read_scalar(nrm_x, s) <= 0.0)
            HCI_LAUNCH(ctx, "dv_seed", s, argmin_seed_kernel, 1, 256, 0, hd, N, xc);
    } else {
        const double n0 = read_scalar(nrm_x, s);
        ws.cgs2(lock, N, nlock, xc, sc, nrm_x);
        if (!(read_scalar(nrm_x, s) > 1e-12 * n0) || n0 <= 0.0) {
            HCI_LAUNCH(ctx, "dv_seed", s, deflated_seed_kernel, 1, 256, 0, hd, N, lock, nlock, xc);
            ws.cgs2(lock, N, nlock, xc, sc, nrm_x);
        }
    }
    if (generic_start) {
        ws.dots(xc, N, 1, xc, nrm_x);
        HCI_LAUNCH(ctx, "dv_seed", s, generic_start_kernel, g1, 256, 0, xc, N, (const double*)nrm_x);
        if (nlock > 0) ws.cgs2(lock, N, nlock, xc, sc, nrm_x);
    }

    const bool mixed = precision == HCI_FP32_MIXED;
    int phase_prec = mixed ? HCI_FP32_MIXED : HCI_FP64;
    int phase_mode = choose_mode(ctx, sp, phase_prec, mode, s);
    int products = 0;
    double theta = 0.0, rnorm = 1e300;
    bool converged = false, need_sigma = true, have_prev = false;

    while (true) {
        // (re)start: V0 = x/|x| with W0 = H V0 (a new product only when the
        // operator changed), plus the previous Ritz vector orthogonalised
        // against it (thick restart keeps the last search direction)
        ws.dots(xc, N, 1, xc, nrm_x);
        HCI_LAUNCH(ctx, "dv_normalize", s, normalize_kernel, g1, 256, 0, xc, nrm_x, V, N);
        if (need_sigma) {
            sigma_apply(ctx, sp, V, W, phase_prec, phase_mode, s);
            ws.project(lock, nlock, W, sc);
            ++products;
            have_prev = false;
        } else {
            HCI_LAUNCH(ctx, "dv_normalize", s, normalize_kernel, g1, 256, 0, wc, nrm_x, W, N);
        }
        need_sigma = false;
        int k = 1;
        if (have_prev && kmax > 1 && products < max_iter) {
            // x_prev minus its component along x is a small difference of two
            // nearly parallel vectors: orthogonalise it twice and take its
            // image from a fresh product (combining the old images would
            // amplify their rounding errors)
            HIP_CHECK(hipMemcpyAsync(t, xp, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
            ws.cgs2(V, N, 1, t, sc, nrm_t);
            if (read_scalar(nrm_t, s) > 1e-24) {
                HCI_LAUNCH(ctx, "dv_normalize", s, normalize_kernel, g1, 256, 0, t, nrm_t, V + N, N);
                sigma_apply(ctx, sp, V + N, W + N, phase_prec, phase_mode, s);
                ws.project(lock, nlock, W + N, sc);
                ++products;
                k = 2;
            }
        }
        for (int j = 0; j < k; ++j) ws.dots(V, N, j + 1, W + (i64)j * N, G.as<double>() + j, DV_MAXK);
        bool phase_done = false;
        while (true) {
            HCI_LAUNCH(ctx, "dv_eig", s, lowest_eig_kernel, 1, 64, 0, G.as<double>(), DV_MAXK,
                       k, (const double*)dead, ritz.as<double>());
            std::swap(xc, xp);
            std::swap(wc, wp);
            // without locked vectors the first sweep of the next direction's
            // orthogonalisation comes with the combination (unused when the
            // basis is full or the iteration ends here)
            const int kd = (nlock == 0 && k < kmax) ? k : 0;
            HCI_LAUNCH(ctx, "dv_combine", s, combine_kernel, ws.nblk, DV_BLOCK, 0, V, W, N, k, kd,
                       ritz.as<double>(), hd, xc, wc, t, N, ws.partial.as<double>(), ws.nblk);
            const unsigned long long seq = ++ctx->host_seq;
            ws.reduce(kd + 1, sc, 1, ritz.as<double>(), theta_h, rr, ctx->host_scal, seq);
            have_prev = true;
            double hv[4];
            wait_host_scalars(ctx, seq, s, hv, poll_ms);
            rnorm = sqrt(std::max(hv[0], 0.0));
            const bool was_dead = hv[2] != 0.0;  // the newest direction had no norm
            theta = hv[3];
            // the float32 operator is only meaningful down to ~1e-7 |theta|
            const double target =
                phase_prec == HCI_FP32_MIXED ? std::max(tol, 1e-7 * std::max(1.0, fabs(theta))) : tol;
            if (rnorm <= target) {
                phase_done = true;
                break;
            }
            if (was_dead) {  // no new direction: restart from the Ritz pair
                HIP_CHECK(hipMemsetAsync(dead, 0, sizeof(double), s));
                break;
            }
            if (products >= max_iter) break;
            if (k == kmax) break;  // thick restart
            // orthogonalise the preconditioned residual against the locked
            // vectors and the basis (CGS2)
            if (nlock > 0) {
                ws.cgs2(lock, N, nlock, t, sc, nrm_t);
                ws.cgs2(V, N, k, t, sc, nrm_t);
            } else {
                ws.cgs2_after_dots(V, N, k, t, sc, nrm_t);
            }
            HCI_LAUNCH(ctx, "dv_normalize", s, normalize_guard_kernel, g1, 256, 0, t, nrm_t,
                       V + (i64)k * N, N, dead);
            sigma_apply(ctx, sp, V + (i64)k * N, W + (i64)k * N, phase_prec, phase_mode, s);
            ws.project(lock, nlock, W + (i64)k * N, sc);
            ++products;
            // new Gram column: G[j][k] = V_j . W_k, j <= k
            ws.dots(V, N, k + 1, W + (i64)k * N, G.as<double>() + k, DV_MAXK);
            ++k;
        }
        if (phase_done) {
            if (phase_prec == HCI_FP32_MIXED) {
                // refine with float64 products from the current Ritz vector
                phase_prec = HCI_FP64;
                phase_mode = choose_mode(ctx, sp, HCI_FP64, mode, s);
                need_sigma = true;
                continue;
            }
            converged = true;
            break;
        }
        if (products >= max_iter) break;
    }
    // normalise and fix the sign of the final vector
    ws.dots(xc, N, 1, xc, nrm_x);
    HCI_LAUNCH(ctx, "dv_normalize", s, normalize_kernel, g1, 256, 0, xc, nrm_x, c, N);
    {
        DevMem pv = dev_alloc(ctx, sizeof(double) * ws.nblk, s);
        DevMem pi = dev_alloc(ctx, sizeof(i64) * ws.nblk, s);
        HCI_LAUNCH(ctx, "dv_signfix", s, absmax_partial_kernel, ws.nblk, 256, 0, c, N, pv.as<double>());
        HCI_LAUNCH(ctx, "dv_signfix", s, tie_index_partial_kernel, ws.nblk, 256, 0, c, N, (const double*)pv.as<double>(),
                   ws.nblk, pi.as<i64>());
        HCI_LAUNCH(ctx, "dv_signfix", s, sign_decide_kernel, 1, 256, 0, c, N, (const i64*)pi.as<i64>(), ws.nblk,
                   nrm_x);
        HCI_LAUNCH(ctx, "dv_signfix", s, scale_kernel, g1, 256, 0, c, N, (const double*)nrm_x);
    }
    *e_out = theta + ctx->ecore;
    if (iters_out) *iters_out = products;
    HIP_CHECK(hipStreamSynchronize(s));
    return converged ? HCI_OK : HCI_E_NOCONV;
}
