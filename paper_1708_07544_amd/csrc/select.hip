// One HCI selection step: V' = V + C(eps1), where C(eps1) holds every
// determinant D_a outside V with |H_ai c_i| > eps1 for some D_i in V
// (Sec. "Variational Stage", eq. criteria and the HCI importance function).
//
// Candidates come from the heat-bath walk, so no candidate list is built for
// an occupied pair that cannot pass.  A determinant is usually reached from
// many D_i; instead of storing every hit and sorting the duplicates away, the
// walk inserts each hit into a device hash set pre-filled with V (open
// addressing, 64-bit CAS).  Only first insertions are appended to the list of
// new determinants, which is then sorted together with V.  The set content,
// hence V', does not depend on the insertion order.
//
// Keys: for norb <= 31 a determinant packs into one word (alpha << 32 |
// beta).  Otherwise alpha and beta strings are first interned in their own
// hash sets and the determinant key is the pair of slot indices.
#include "hashset.h"
#include "walk.h"

namespace {

constexpr int WALK_BLOCK = 256;
constexpr int WALK_ROWS = WALK_BLOCK / HCI_WAVE;
using namespace hset;

// Inserts the visited candidates.  Once the set holds `limit` new
// determinants (its load factor would pass 1/2) or an insert fails, the
// overflow flag is raised and the wave stops inserting: the host grows the
// set and walks again, so the rest of this walk would be wasted probing of
// an ever fuller table.  Every lane of a wave calls the visitor together,
// so `stop` stays uniform.
struct InsertVis {
    HashSet H;
    u64* out;
    unsigned long long* counter;
    i64 cap;
    i64 limit;
    bool stop;
    __device__ __forceinline__ void operator()(bool ok, u64 aa, u64 ab) {
        if (stop) return;
        bool fresh = false, failed = false, sfailed = false;
        u64 key = 0;
        if (ok) {
            if (!det_key(H, aa, ab, key)) {
                sfailed = true;
            } else if (hash_insert(H.det, H.det_mask, key, fresh) < 0) {
                failed = true;
                fresh = false;
            }
        }
        const u64 m = ballot(fresh);
        unsigned long long base = 0;
        if (m && lane_id() == 0) base = atomicAdd(counter, (unsigned long long)__popcll(m));
        base = __shfl(base, 0, 64);
        if (fresh) {
            const i64 at = (i64)base + rank_in(m);
            if (at < cap) out[at] = key;
        }
        const bool sfail = ballot(sfailed) != 0;
        const bool dfail = ballot(failed) != 0 || (m && (i64)base + __popcll(m) > limit);
        if (sfail || dfail) {
            if (lane_id() == 0) atomicOr(H.overflow, (sfail ? OVER_STR : 0ull) | (dfail ? OVER_DET : 0ull));
            stop = true;
        }
    }
};

__global__ void __launch_bounds__(WALK_BLOCK) select_walk_kernel(
    HBView T, IntView I, const u64* __restrict__ dets, const double* __restrict__ c, i64 N,
    double eps, double hb_max, HashSet H, u64* __restrict__ out, i64 cap, i64 limit,
    unsigned long long* __restrict__ counter) {
    // one wavefront per row, striding over the rows beyond one launch's grid
    for (i64 i = (i64)blockIdx.x * WALK_ROWS + threadIdx.x / HCI_WAVE; i < N;
         i += (i64)gridDim.x * WALK_ROWS) {
        const double ci = fabs(c[i]);
        if (!(hb_max * ci > eps)) continue;  // nothing can pass from this determinant
        if (*(volatile unsigned long long*)H.overflow != 0ull) return;  // the set is being regrown
        InsertVis v{H, out, counter, cap, limit, false};
        heat_bath_walk(T, I, dets[2 * i], dets[2 * i + 1], ci, eps, v);
    }
}

// V followed by the decoded new determinants, split into (alpha, beta) words
__global__ void gather_kernel(const u64* __restrict__ dets, i64 N, const u64* __restrict__ keys,
                              i64 m, HashSet H, u64* __restrict__ hi, u64* __restrict__ lo) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N) {
        hi[t] = dets[2 * t];
        lo[t] = dets[2 * t + 1];
    } else if (t < N + m) {
        const u64 k = keys[t - N];
        if (H.packed) {
            hi[t] = k >> 32;
            lo[t] = k & 0xffffffffull;
        } else {
            hi[t] = H.sa[k >> 32];
            lo[t] = H.sb[k & 0xffffffffull];
        }
    }
}

__global__ void interleave_kernel(const u64* __restrict__ hi, const u64* __restrict__ lo, i64 n,
                                  u64* __restrict__ out) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        out[2 * t] = hi[t];
        out[2 * t + 1] = lo[t];
    }
}

__global__ void max_reduce_kernel(const double* __restrict__ a, i64 n, i64 stride,
                                  double* __restrict__ out) {
    // one block: max over a[k * stride], k < n
    __shared__ double red[256];
    double m = 0.0;
    for (i64 k = threadIdx.x; k < n; k += 256) m = fmax(m, a[k * stride]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = fmax(*out, red[0]);
}

// out[pos(V[k] in V')] = c[k]; missing members bump the error counter
__global__ void embed_kernel(const u64* __restrict__ dets, i64 n, const double* __restrict__ c,
                             const u64* __restrict__ dn, i64 nn, double* __restrict__ out,
                             unsigned long long* __restrict__ missing) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const u64 a = dets[2 * k], b = dets[2 * k + 1];
    i64 lo = 0, hi = nn;
    while (lo < hi) {
        const i64 mid = (lo + hi) >> 1;
        const u64 ma = dn[2 * mid], mb = dn[2 * mid + 1];
        if (ma < a || (ma == a && mb < b)) lo = mid + 1;
        else hi = mid;
    }
    if (lo < nn && dn[2 * lo] == a && dn[2 * lo + 1] == b) out[lo] = c[k];
    else atomicAdd(missing, 1ull);
}

i64 pow2_at_least(i64 x) {
    i64 p = 1;
    while (p < x) p <<= 1;
    return p;
}

// w_i = max_r |C_r,i| over the states r (rows of C): fl(|H_ai| x) is
// non-decreasing in x, so fl(|H_ai| w_i) > eps exactly when some state
// passes, and one walk with w selects the union of the states' sets.
__global__ void roots_weight_kernel(const double* __restrict__ C, int nroots, i64 N, double* __restrict__ w) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double m = 0.0;
    for (int r = 0; r < nroots; ++r) m = fmax(m, fabs(C[(i64)r * N + i]));
    w[i] = m;
}

// Content hash of a float64 vector (wrapping sum of position-mixed words:
// order independent, so the integer atomics give one value).
__global__ void hash_f64_kernel(const double* __restrict__ x, i64 n, unsigned long long* __restrict__ h) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    u64 v = 0;
    if (i < n) {
        u64 z = (u64)__double_as_longlong(x[i]) * 0x9e3779b97f4a7c15ull ^ ((u64)i + 0x632be59bd9b4e019ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        v = z ^ (z >> 31);
    }
    v = wave_sum_u64(v);
    if (lane_id() == 0 && v) atomicAdd(h, (unsigned long long)v);
}

u64 hash_f64(hci_ctx_s* ctx, const double* x, i64 n, hipStream_t s) {
    DevMem h = dev_alloc(ctx, sizeof(u64), s);
    HIP_CHECK(hipMemsetAsync(h.ptr, 0, sizeof(u64), s));
    HCI_LAUNCH(ctx, "select_hash", s, hash_f64_kernel, ceil_div(n, 256), 256, 0, x, n,
               (unsigned long long*)h.as<u64>());
    return read_scalar(h.as<u64>(), s);
}

// Largest result kept for a capacity retry (larger ones walk again).
constexpr i64 SELECT_KEEP_MAX = (i64)1 << 28;  // determinants (4 GiB)

}  // namespace

i64 select_roots_run(hci_ctx_s* ctx, const u64* dets, const double* C, int nroots, i64 N, double eps,
                     u64* out, i64 cap, hipStream_t s) {
    DevMem w = dev_alloc(ctx, sizeof(double) * N, s);
    HCI_LAUNCH(ctx, "select_roots", s, roots_weight_kernel, ceil_div(N, 256), 256, 0, C, nroots, N,
               w.as<double>());
    return select_run(ctx, dets, w.as<double>(), N, eps, out, cap, s);
}

void embed_run(hci_ctx_s* ctx, const u64* dets, i64 n, const double* c, const u64* dn, i64 nn,
               double* out, hipStream_t s) {
    DevMem miss = dev_alloc(ctx, sizeof(u64), s);
    HIP_CHECK(hipMemsetAsync(miss.ptr, 0, sizeof(u64), s));
    HIP_CHECK(hipMemsetAsync(out, 0, sizeof(double) * nn, s));
    HCI_LAUNCH(ctx, "embed", s, embed_kernel, ceil_div(n, 256), 256, 0, dets, n, c, dn, nn, out,
               (unsigned long long*)miss.as<u64>());
    HCI_REQUIRE(read_scalar(miss.as<u64>(), s) == 0, HCI_E_ARG,
                "embed: a determinant of V is missing from V'");
}

// Largest magnitude any single or double element can have (list heads and
// single bounds): a determinant with hb_max * |c_i| <= eps emits nothing.
double heat_bath_max(hci_ctx_s* ctx, hipStream_t s) {
    Integrals& I = ctx->ints;
    const int n = ctx->n;
    DevMem m = dev_alloc(ctx, sizeof(double), s);
    HIP_CHECK(hipMemsetAsync(m.ptr, 0, sizeof(double), s));
    if (I.os_len > 0)
        HCI_LAUNCH(ctx, "hb_max", s, max_reduce_kernel, 1, 256, 0, I.os_abs.as<double>(),
                   (i64)n * n, (i64)I.os_len, m.as<double>());
    if (I.ss_len > 0)
        HCI_LAUNCH(ctx, "hb_max", s, max_reduce_kernel, 1, 256, 0, I.ss_abs.as<double>(),
                   (i64)n * (n - 1) / 2, (i64)I.ss_len, m.as<double>());
    HCI_LAUNCH(ctx, "hb_max", s, max_reduce_kernel, 1, 256, 0, I.single_bound.as<double>(),
               (i64)n * n, (i64)1, m.as<double>());
    return read_scalar(m.as<double>(), s);
}

i64 select_run(hci_ctx_s* ctx, const u64* dets, const double* c, i64 N, double eps, u64* out,
               i64 cap, hipStream_t s) {
    const int n = ctx->n;
    // the caller validated dets as the context's space: its content hash
    // and that of c key a result kept by an earlier call that did not fit
    HCI_REQUIRE(ctx->space != nullptr && ctx->space->N == N, HCI_E_HIP, "internal: selection without its space");
    const u64 d_hash = ctx->space->hash;
    const u64 c_hash = hash_f64(ctx, c, N, s);
    if (SelectKept* k = ctx->sel_kept) {
        const bool same = k->N == N && k->dets_hash == d_hash && k->c_hash == c_hash && k->eps == eps;
        if (same && k->M <= cap) {
            const i64 M = k->M;
            HIP_CHECK(hipMemcpyAsync(out, k->out.ptr, sizeof(u64) * 2 * M, hipMemcpyDeviceToDevice, s));
            HIP_CHECK(hipStreamSynchronize(s));
            delete k;
            ctx->sel_kept = nullptr;
            return M;
        }
        delete k;
        ctx->sel_kept = nullptr;
    }
    const double hbm = heat_bath_max(ctx, s);
    HBView T = hb_view(ctx->ints);
    IntView I = int_view(ctx->ints);
    const bool packed = n <= 31;
    // [0] new determinants, [1] overflow, [2..3] interned alpha / beta strings
    DevMem flags = dev_alloc(ctx, sizeof(u64) * 4, s);
    unsigned long long* counter = (unsigned long long*)flags.as<u64>();
    unsigned long long* overflow = counter + 1;
    unsigned long long* strings = counter + 2;
    // V' is often 10-200x larger than V: start generous (a retry repeats the walk)
    i64 det_slots = pow2_at_least(std::max<i64>(64 * N, 1 << 22));
    i64 str_slots = pow2_at_least(std::max<i64>(2 * N, 1 << 16));
    DevMem table, sa, sb, keys;
    i64 m = 0;
    for (int attempt = 0;; ++attempt) {
        HCI_REQUIRE(attempt < 10 && det_slots <= ((i64)1 << 32) && str_slots <= ((i64)1 << 32), HCI_E_NOMEM,
                    "selection hash set cannot grow further (more than 2^31 determinants or strings)");
        table = dev_alloc(ctx, sizeof(u64) * det_slots, s);
        HCI_LAUNCH(ctx, "select_fill", s, fill_kernel, std::min<i64>(ceil_div(det_slots, 256), 1 << 20), 256, 0,
                   table.as<u64>(), det_slots, EMPTY);
        HashSet H{table.as<u64>(), (u64)(det_slots - 1), nullptr, 0, nullptr, 0, packed ? 1 : 0,
                  overflow, strings};
        if (!packed) {
            sa = dev_alloc(ctx, sizeof(u64) * str_slots, s);
            sb = dev_alloc(ctx, sizeof(u64) * str_slots, s);
            HCI_LAUNCH(ctx, "select_fill", s, fill_kernel, std::min<i64>(ceil_div(str_slots, 256), 1 << 20), 256, 0,
                       sa.as<u64>(), str_slots, EMPTY);
            HCI_LAUNCH(ctx, "select_fill", s, fill_kernel, std::min<i64>(ceil_div(str_slots, 256), 1 << 20), 256, 0,
                       sb.as<u64>(), str_slots, EMPTY);
            H.sa = sa.as<u64>();
            H.sb = sb.as<u64>();
            H.sa_mask = H.sb_mask = (u64)(str_slots - 1);
        }
        HIP_CHECK(hipMemsetAsync(flags.ptr, 0, sizeof(u64) * 4, s));
        HCI_LAUNCH(ctx, "select_insert_v", s, insert_v_kernel, ceil_div(N, 256), 256, 0, H, dets, N);
        // new determinants can never exceed the free slots
        const i64 kcap = det_slots / 2;
        keys = dev_alloc(ctx, sizeof(u64) * kcap, s);
        // stop the walk once the new determinants would take the load factor past 1/2
        const i64 limit = std::max<i64>(0, std::min<i64>(kcap, det_slots / 2 - N));
        HCI_LAUNCH(ctx, "select_walk", s, select_walk_kernel, row_grid(N, WALK_ROWS, WALK_BLOCK), WALK_BLOCK, 0, T,
                   I, dets, c, N, eps, hbm, H, keys.as<u64>(), kcap, limit, counter);
        u64 hv[4];
        HIP_CHECK(hipMemcpyAsync(hv, flags.ptr, sizeof(hv), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        m = (i64)hv[0];
        // keep every load factor at most 1/2: otherwise grow the table that
        // filled (only that one) and walk again
        const i64 nstr = (i64)std::max(hv[2], hv[3]);
        const bool det_full = (hv[1] & OVER_DET) != 0 || N + m > det_slots / 2 || m > kcap;
        const bool str_full = !packed && ((hv[1] & OVER_STR) != 0 || nstr > str_slots / 2);
        if (!det_full && !str_full) break;
        // (a table already at 2^32 slots cannot grow: the next attempt fails)
        const i64 top = (i64)1 << 32;
        if (det_full)
            det_slots = det_slots >= top ? 2 * top : std::min(top, pow2_at_least(std::max<i64>(4 * (N + m), 8 * det_slots)));
        if (str_full)
            str_slots = str_slots >= top ? 2 * top : std::min(top, pow2_at_least(std::max<i64>(4 * nstr, 2 * str_slots)));
    }
    const i64 M = N + m;
    // V + C sorted into dst
    auto write_to = [&](u64* dst) {
        HashSet H{table.as<u64>(), (u64)(det_slots - 1), sa.as<u64>(), (u64)(str_slots - 1),
                  sb.as<u64>(), (u64)(str_slots - 1), packed ? 1 : 0, overflow, strings};
        DevMem hi = dev_alloc(ctx, sizeof(u64) * M, s), lo = dev_alloc(ctx, sizeof(u64) * M, s);
        HCI_LAUNCH(ctx, "select_gather", s, gather_kernel, ceil_div(M, 256), 256, 0, dets, N,
                   keys.as<u64>(), m, H, hi.as<u64>(), lo.as<u64>());
        {
            DevMem thi = dev_alloc(ctx, sizeof(u64) * M, s), tlo = dev_alloc(ctx, sizeof(u64) * M, s);
            radix_sort128(ctx, hi.as<u64>(), lo.as<u64>(), nullptr, thi.as<u64>(), tlo.as<u64>(), nullptr,
                          M, n, n, s);
        }
        HCI_LAUNCH(ctx, "select_write", s, interleave_kernel, ceil_div(M, 256), 256, 0, hi.as<u64>(),
                   lo.as<u64>(), M, dst);
    };
    if (M > cap) {
        // the caller retries with capacity M: keep the result for it (when
        // it is of a size worth holding and the memory is there)
        if (M <= SELECT_KEEP_MAX) {
            try {
                std::unique_ptr<SelectKept> keep(new SelectKept());
                keep->out = dev_alloc(ctx, sizeof(u64) * 2 * M, s);
                keep->M = M;
                keep->N = N;
                keep->dets_hash = d_hash;
                keep->c_hash = c_hash;
                keep->eps = eps;
                write_to(keep->out.as<u64>());
                ctx->sel_kept = keep.release();
            } catch (const HciError& e) {
                if (e.code != HCI_E_NOMEM) throw;
            }
        }
        return M;
    }
    write_to(out);
    return M;
}
