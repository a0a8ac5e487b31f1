// Spin-traced one- and two-particle (transition) density matrices on V,
//   rdm1[p][q]       = sum_s  <bra| a+_ps a_qs |ket>,
//   rdm2[p][q][r][s] = sum_st <bra| a+_ps a+_rt a_st a_qs |ket>,
// accumulated by looping over the same single and double connections as
// the Hamiltonian product (Sec. "Computational Details").
//
// Diagonal pairs (i = j) only involve occupation numbers, so they are
// reduced without atomics: D[x][y] = sum_i bra_i ket_i n_x(i) n_y(i) over
// spin orbitals x, y, block partials then a fixed-order sum.  Each
// off-diagonal pair (row i, connection j) adds bra_i ket_j times the
// operator matrix element of the excitation D_j -> D_i to the few
// rdm entries it touches, with float64 atomics.
#include "slater.h"

namespace {

constexpr int ROW_BLOCK = 256;
constexpr int ROWS_PER_BLOCK = ROW_BLOCK / HCI_WAVE;
constexpr int OCC_CHUNK = 256;

__device__ __forceinline__ void add64(double* p, double v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ i64 r2idx(int n, int p, int q, int r, int s) {
    return (((i64)p * n + q) * n + r) * n + s;
}

// contributions of <D_i| ... |D_j> for a single excitation v -> u in the
// string sj (spin s) of D_j, with `other` the opposite-spin string of D_j
__device__ __forceinline__ void single_contrib(int n, double x, u64 sj, u64 other, int v, int u,
                                               double* r1, double* r2) {
    add64(&r1[(i64)u * n + v], x);
    if (!r2) return;
    for (u64 m = sj & ~bit(v); m; m &= m - 1) {  // same-spin spectators
        const int k = ctz64(m);
        add64(&r2[r2idx(n, u, v, k, k)], x);
        add64(&r2[r2idx(n, k, k, u, v)], x);
        add64(&r2[r2idx(n, u, k, k, v)], -x);
        add64(&r2[r2idx(n, k, v, u, k)], -x);
    }
    for (u64 m = other; m; m &= m - 1) {  // opposite-spin spectators
        const int k = ctz64(m);
        add64(&r2[r2idx(n, u, v, k, k)], x);
        add64(&r2[r2idx(n, k, k, u, v)], x);
    }
}

__device__ __forceinline__ void pair_contrib(int n, double w, u64 ai, u64 bi, u64 aj, u64 bj,
                                             double* r1, double* r2) {
    const u64 xa = ai ^ aj, xb = bi ^ bj;
    const int da = popc64(xa) >> 1, db = popc64(xb) >> 1;
    if (da == 1 && db == 0) {
        const int v = ctz64(aj & xa), u = ctz64(ai & xa);
        single_contrib(n, w * sign_between(aj, v, u), aj, bj, v, u, r1, r2);
        return;
    }
    if (da == 0 && db == 1) {
        const int v = ctz64(bj & xb), u = ctz64(bi & xb);
        single_contrib(n, w * sign_between(bj, v, u), bj, aj, v, u, r1, r2);
        return;
    }
    if (!r2) return;
    if (da == 1 && db == 1) {
        const int v1 = ctz64(aj & xa), u1 = ctz64(ai & xa);
        const int v2 = ctz64(bj & xb), u2 = ctz64(bi & xb);
        const double x = w * (sign_between(aj, v1, u1) * sign_between(bj, v2, u2));
        add64(&r2[r2idx(n, u1, v1, u2, v2)], x);
        add64(&r2[r2idx(n, u2, v2, u1, v1)], x);
        return;
    }
    const u64 sj = da == 2 ? aj : bj;
    const u64 x2 = da == 2 ? xa : xb;
    u64 holes = sj & x2, parts = x2 & ~sj;
    const int v1 = ctz64(holes);
    holes &= holes - 1;
    const int v2 = ctz64(holes);
    const int u1 = ctz64(parts);
    parts &= parts - 1;
    const int u2 = ctz64(parts);
    const double sg = sign_double(sj, v1, u1, v2, u2);
    const double x = w * sg;
    add64(&r2[r2idx(n, u1, v1, u2, v2)], x);
    add64(&r2[r2idx(n, u2, v2, u1, v1)], x);
    add64(&r2[r2idx(n, u1, v2, u2, v1)], -x);
    add64(&r2[r2idx(n, u2, v1, u1, v2)], -x);
}

struct RdmVis {
    const double* ket;
    double bra_i;
    u64 ai, bi;
    int n;
    double* r1;
    double* r2;
    __device__ __forceinline__ void operator()(bool ok, u32 j, u64 aj, u64 bj) {
        if (!ok) return;
        const double w = bra_i * ket[j];
        if (w == 0.0) return;
        pair_contrib(n, w, ai, bi, aj, bj, r1, r2);
    }
};

__global__ void __launch_bounds__(ROW_BLOCK) rdm_offdiag_kernel(SpaceView S,
                                                                const double* __restrict__ bra,
                                                                const double* __restrict__ ket,
                                                                double* __restrict__ r1,
                                                                double* __restrict__ r2) {
    const i64 i = (i64)blockIdx.x * ROWS_PER_BLOCK + threadIdx.x / HCI_WAVE;
    if (i >= S.N) return;
    const double bi_ = bra[i];
    if (bi_ == 0.0) return;  // wave-uniform
    RdmVis v{ket, bi_, S.alpha[i], S.beta[i], S.n, r1, r2};
    enumerate_row(S, (u32)i, v);
}

// Occupation correlation D[x][y] = sum_i w_i n_x(i) n_y(i) over spin
// orbitals x, y in [0, 2n) (alpha first), w_i = bra_i ket_i; one partial
// matrix per block, threads own entries, determinants staged through LDS.
constexpr int OCC_PER_THREAD = 8;
constexpr int OCC_TILE = 256 * OCC_PER_THREAD;

__global__ void __launch_bounds__(256) occ_corr_kernel(const u64* __restrict__ alpha,
                                                       const u64* __restrict__ beta,
                                                       const double* __restrict__ bra,
                                                       const double* __restrict__ ket, i64 N,
                                                       int n, i64 chunk, double* __restrict__ part) {
    __shared__ u64 sa[OCC_CHUNK], sb[OCC_CHUNK];
    __shared__ double sw[OCC_CHUNK];
    const int m = 2 * n;
    const int entries = m * m;
    const int tile0 = blockIdx.y * OCC_TILE;
    const i64 begin = (i64)blockIdx.x * chunk, end = min(begin + chunk, N);
    double acc[OCC_PER_THREAD];
#pragma unroll
    for (int e = 0; e < OCC_PER_THREAD; ++e) acc[e] = 0.0;
    for (i64 base = begin; base < end; base += OCC_CHUNK) {
        const i64 t = base + threadIdx.x;
        if (threadIdx.x < OCC_CHUNK) {
            if (t < end) {
                sa[threadIdx.x] = alpha[t];
                sb[threadIdx.x] = beta[t];
                sw[threadIdx.x] = bra[t] * ket[t];
            } else {
                sa[threadIdx.x] = 0;
                sb[threadIdx.x] = 0;
                sw[threadIdx.x] = 0.0;
            }
        }
        __syncthreads();
        const int cnt = (int)min((i64)OCC_CHUNK, end - base);
#pragma unroll
        for (int e = 0; e < OCC_PER_THREAD; ++e) {
            const int idx = tile0 + threadIdx.x + e * 256;
            if (idx < entries) {
                const int x = idx / m, y = idx % m;
                const bool xa = x < n, ya = y < n;
                const int bx = xa ? x : x - n, by = ya ? y : y - n;
                double s = 0.0;
                for (int k = 0; k < cnt; ++k) {
                    const u64 wx = xa ? sa[k] : sb[k];
                    const u64 wy = ya ? sa[k] : sb[k];
                    if (test_bit(wx, bx) && test_bit(wy, by)) s += sw[k];
                }
                acc[e] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < OCC_PER_THREAD; ++e) {
        const int idx = tile0 + threadIdx.x + e * 256;
        if (idx < entries) part[(i64)blockIdx.x * entries + idx] = acc[e];
    }
}

__global__ void occ_reduce_kernel(const double* __restrict__ part, int nblk, int entries,
                                  double* __restrict__ D) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= entries) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(i64)b * entries + idx];
    D[idx] = s;
}

// Add the diagonal-pair terms from D: rdm1[p][p] += D[pa][pa] + D[pb][pb];
// rdm2[p][p][r][r] += sum over spin pairs of D[x][y] (x != y);
// rdm2[p][r][r][p] -= same-spin D[x][y] (p != r).
__global__ void diag_terms_kernel(const double* __restrict__ D, int n, double* __restrict__ r1,
                                  double* __restrict__ r2) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    const int p = idx / n, r = idx % n;
    const int m = 2 * n;
    const double daa = D[p * m + r], dbb = D[(p + n) * m + (r + n)];
    const double dab = D[p * m + (r + n)], dba = D[(p + n) * m + r];
    if (p == r) r1[(i64)p * n + p] += daa + dbb;
    if (!r2) return;
    if (p == r) {
        r2[r2idx(n, p, p, p, p)] += dab + dba;
    } else {
        r2[r2idx(n, p, p, r, r)] += daa + dbb + dab + dba;
        r2[r2idx(n, p, r, r, p)] -= daa + dbb;
    }
}

// Gamma^{dc}: one thread per screened pair (i, a), weight d_a c_i, bra D_a,
// ket D_i (Sec. "Computational Details": the connection list of the PT2).
__global__ void pt2_pairs_kernel(const u64* __restrict__ a_hi, const u64* __restrict__ a_lo,
                                 const u32* __restrict__ idx, const double* __restrict__ dpair,
                                 const u64* __restrict__ dets, const double* __restrict__ c, i64 M,
                                 int n, double* __restrict__ r1, double* __restrict__ r2) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    const u32 i = idx[t];
    const double w = dpair[t] * c[i];
    if (w == 0.0) return;
    pair_contrib(n, w, a_hi[t], a_lo[t], dets[2 * (i64)i], dets[2 * (i64)i + 1], r1, r2);
}

}  // namespace

// Diagonal-pair terms of sum_k wa_k wb_k <D_k| ops |D_k> added to rdm1/rdm2.
void rdm_add_diag(hci_ctx_s* ctx, const u64* alpha, const u64* beta, const double* wa,
                  const double* wb, i64 M, double* rdm1, double* rdm2, hipStream_t s) {
    if (M <= 0) return;
    const int n = ctx->n;
    const i64 n2 = (i64)n * n;
    const int entries = 4 * n * n;
    const i64 chunk = std::max<i64>(OCC_CHUNK, ceil_div(M, 512));
    const int nblk = (int)ceil_div(M, chunk);
    DevMem part = dev_alloc(ctx, sizeof(double) * (i64)nblk * entries, s);
    DevMem D = dev_alloc(ctx, sizeof(double) * entries, s);
    HCI_LAUNCH(ctx, "rdm_occ", s, occ_corr_kernel, dim3(nblk, (unsigned)ceil_div(entries, OCC_TILE)),
               256, 0, alpha, beta, wa, wb, M, n, chunk, part.as<double>());
    HCI_LAUNCH(ctx, "rdm_occ_reduce", s, occ_reduce_kernel, ceil_div(entries, 256), 256, 0,
               part.as<double>(), nblk, entries, D.as<double>());
    HCI_LAUNCH(ctx, "rdm_diag_terms", s, diag_terms_kernel, ceil_div(n2, 256), 256, 0,
               D.as<double>(), n, rdm1, rdm2);
}

void rdm_compute(hci_ctx_s* ctx, Space* sp, const double* bra, const double* ket, double* rdm1,
                 double* rdm2, hipStream_t s) {
    const int n = ctx->n;
    const i64 N = sp->N;
    const i64 n2 = (i64)n * n;
    HIP_CHECK(hipMemsetAsync(rdm1, 0, sizeof(double) * n2, s));
    if (rdm2) HIP_CHECK(hipMemsetAsync(rdm2, 0, sizeof(double) * n2 * n2, s));
    SpaceView S = space_view(*sp, n);
    HCI_LAUNCH(ctx, "rdm_offdiag", s, rdm_offdiag_kernel, ceil_div(N, ROWS_PER_BLOCK), ROW_BLOCK, 0,
               S, bra, ket, rdm1, rdm2);
    rdm_add_diag(ctx, sp->alpha.as<u64>(), sp->beta.as<u64>(), bra, ket, N, rdm1, rdm2, s);
}

void rdm_add_pt2_pairs(hci_ctx_s* ctx, const Pt2State& st, const u64* dets, const double* c,
                       double* rdm1, double* rdm2, hipStream_t s) {
    if (st.M <= 0) return;
    HCI_LAUNCH(ctx, "rdm_pt2_pairs", s, pt2_pairs_kernel, ceil_div(st.M, 256), 256, 0,
               st.a_hi.as<u64>(), st.a_lo.as<u64>(), st.idx.as<u32>(), st.dpair.as<double>(), dets, c,
               st.M, ctx->n, rdm1, rdm2);
}
