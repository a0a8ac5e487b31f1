// Shared host/device definitions of the HCI library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hci.h"
#include "phase.h"

typedef uint64_t u64;
typedef uint32_t u32;
typedef uint16_t u16;
typedef int64_t i64;

#define HCI_WAVE 64

// ---------------------------------------------------------------- errors
struct HciError {
    int code;
    std::string msg;
};

void hci_set_error(const std::string& msg);

#define HIP_CHECK(expr)                                                               \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) {                                                       \
            throw HciError{HCI_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
        }                                                                             \
    } while (0)

#define HCI_REQUIRE(cond, code, text)                  \
    do {                                               \
        if (!(cond)) throw HciError{(code), (text)};   \
    } while (0)

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ int popc64(u64 x) { return __popcll(x); }
__device__ __forceinline__ int ctz64(u64 x) { return __builtin_ctzll(x); }
// Bit manipulation on 64-bit occupation words goes through 32-bit halves
// and shifts by less than 32 (well defined for every orbital index; the
// phase helpers in phase.h are checked against brute force on the CPU).
__device__ __forceinline__ u64 join32(u32 hi, u32 lo) { return ((u64)hi << 32) | (u64)lo; }
__device__ __forceinline__ u32 lo32(u64 x) { return (u32)x; }
__device__ __forceinline__ u32 hi32(u64 x) { return (u32)(x >> 32); }

// word with only bit p set (0 <= p < 64)
__device__ __forceinline__ u64 bit(int p) {
    const u32 one = 1u << (p & 31);
    return join32(p >= 32 ? one : 0u, p < 32 ? one : 0u);
}

// bit p of s (0 <= p < 64)
__device__ __forceinline__ bool test_bit(u64 s, int p) {
    const u32 w = p < 32 ? lo32(s) : hi32(s);
    return ((w >> (p & 31)) & 1u) != 0u;
}

// bits [0, k) set (0 <= k <= 64)
__device__ __forceinline__ u64 low_mask(int k) {
    return join32(phase_mask32(k > 32 ? k - 32 : 0), phase_mask32(k < 32 ? k : 32));
}

// byte b (0..7) of x
__device__ __forceinline__ u32 byte_of(u64 x, int b) {
    const u32 w = b < 4 ? lo32(x) : hi32(x);
    return (w >> (8 * (b & 3))) & 0xffu;
}

// Phases of excitations (host and device, checked on the CPU against a
// brute-force count of the bits between two orbitals).
__device__ __forceinline__ int rank_below(u64 s, int k) { return phase_rank_below(s, k); }
__device__ __forceinline__ int count_between(u64 s, int p, int q) { return phase_count_between(s, p, q); }
__device__ __forceinline__ double sign_between(u64 s, int p, int q) { return phase_sign_between(s, p, q); }
__device__ __forceinline__ double sign_double(u64 si, int p, int r, int q, int s) {
    return phase_sign_double(si, p, r, q, s);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ u64 ballot(bool p) { return __ballot(p); }

// number of set bits of m in the lanes below this one (mbcnt, no shifts)
__device__ __forceinline__ u32 rank_in(u64 m) {
    return __builtin_amdgcn_mbcnt_hi(hi32(m), __builtin_amdgcn_mbcnt_lo(lo32(m), 0u));
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ i64 wave_sum_i64(i64 v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ u64 wave_sum_u64(u64 v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block reduction (fixed tree) of one double per thread.
template <int BLOCK>
__device__ __forceinline__ double block_sum_f64(double v, double* lds /*[BLOCK/64]*/) {
    v = wave_sum_f64(v);
    const int w = threadIdx.x / 64;
    if (lane_id() == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < BLOCK / 64; ++k) t += lds[k];
    }
    __syncthreads();
    return t;  // valid in thread 0
}

// ---------------------------------------------------------------- memory
struct hci_ctx_s;

// A device allocation owned by a context (freed through the context's allocator).
struct DevMem {
    hci_ctx_s* ctx = nullptr;
    void* ptr = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    DevMem(DevMem&& o) noexcept { *this = std::move(o); }
    DevMem& operator=(DevMem&& o) noexcept;
    ~DevMem() { release(); }
    void release();
    template <class T>
    T* as() const { return reinterpret_cast<T*>(ptr); }
};

// ---------------------------------------------------------------- integrals
// Tables derived from h and g, all on the device.
struct Integrals {
    int n = 0;
    DevMem h;       // f64 [n][n]
    DevMem g;       // f64 [n]^4
    DevMem g32;     // f32 [n]^4
    DevMem jk;      // f64 [n][n][n]: jk[q][p][r] = (qp|rr) - (qr|rp)
    DevMem jj;      // f64 [n][n][n]: jj[q][p][r] = (qp|rr)
    DevMem jk32;    // f32 copies for the mixed recompute path
    DevMem jj32;
    DevMem h32;
    DevMem jdiag;   // f64 [n][n]: (pp|qq)
    DevMem kdiag;   // f64 [n][n]: (pq|qp)
    // heat-bath lists
    DevMem os_abs;  // f64 [n*n][(n-1)^2], |(rp|sq)| descending per (p,q)
    DevMem os_rs;   // u32 packed r | s << 8
    DevMem ss_abs;  // f64 [n(n-1)/2][(n-2)(n-3)/2] |(rp|sq)-(rq|sp)| descending per p<q
    DevMem ss_rs;
    DevMem single_bound;  // f64 [n][n] upper bound of |single element| for p->r
    int os_len = 0, ss_len = 0;
};

// Derived structure of one sorted determinant list V.
// Row chunks (bucket, first row, end row) of a persistent grid of P
// workgroups: workgroup p takes list[wptr[p] .. wptr[p + 1]) in that order.
// The assignment balances an estimated cost and depends only on the space.
struct RdmChunks {
    DevMem list;  // u32 [n][3]
    DevMem wptr;  // u32 [P + 1]
    int P = 0;
    int key = -1;  // what else the estimated costs depended on
};

struct Space {
    const u64* key_ptr = nullptr;  // caller's list address
    i64 N = 0;
    u64 hash = 0;
    DevMem alpha, beta;   // u64 [N]
    DevMem ia, ib;        // u32 [N]: index of the det's alpha / beta string
    DevMem ua, aoff;      // u64 [nua], u32 [nua+1]
    DevMem ub, boff;      // u64 [nub], u32 [nub+1]
    DevMem permb;         // u32 [N]: det indices in (beta, alpha) order
    DevMem as_ptr, as_idx;  // u32 [nua+1], u32 [..]: alpha strings one single apart
    DevMem bs_ptr, bs_idx;
    i64 nua = 0, nub = 0, n_as = 0, n_bs = 0;
    DevMem hdiag;         // f64 [N] (ecore excluded)
    DevMem c32;           // f32 [N] staging copy of the vector for mixed products
    bool have_diag = false;
    // stored Hamiltonian (off-diagonal part, CSR)
    DevMem rowptr;        // i64 [N+1]
    DevMem cols;          // u32 [nnz]
    DevMem vals64;        // f64 [nnz]
    DevMem vals32;        // f32 [nnz]
    i64 nnz_off = -1;     // off-diagonal connections
    i64 nnz_pad = 0;      // stored entries (rows padded to multiples of 4)
    bool have_csr64 = false, have_csr32 = false;
    // stored Hamiltonian, alpha-bucket-staged layout (staged.hip)
    int layout = 0;       // 0 undecided, 1 plain CSR, 2 staged
    u32 st_wlog = 0;      // window of 2^st_wlog entries of c staged in LDS
    i64 st_nchunk = 0;    // workgroups of one product
    DevMem st_xpos;       // u32 [nua + n_as]: start of each stage range
    DevMem st_len;        // u32 [nua]: stage length of each bucket
    DevMem st_nseg;       // u32 [nua]: windows + 1 (beta-group segment)
    DevMem st_cptr;       // u32 [nua + 1]: first workgroup of each bucket
    DevMem st_gcptr;      // u32 [nub + 1]: first workgroup of each beta group
    DevMem st_chunk;      // u32 [st_nchunk][3]: bucket, first row, end row of each workgroup
    DevMem st_gchunk;     // u32 [st_gnchunk][4]: rows [k0, k1), c slice [s0, s1) (beta-major)
    i64 st_gnchunk = 0;   // workgroups of the beta-group product
    i64 st_gmax = 0;      // largest beta group
    DevMem st_rsb;        // i64 [N + 1]: first segment slot of each row
    DevMem st_sstart;     // i64 [st_rsb[N]]: absolute start of every (row, segment)
    DevMem st_segcnt;     // u32 [st_rsb[N]]: entries of each segment before padding
    i64 st_nslots = 0;    // st_rsb[N]
    u32 st_abW = 0;       // beta-string bitmap words per neighbour (0: search instead)
    u32 st_abG = 0;       // alpha neighbours per bitmap pass
    DevMem st_cols;       // u16 [st_nnz]
    i64 st_nnz = 0;       // stored entries (segments padded to multiples of 4)
    DevMem st_vals32, st_vals64;
    DevMem cpb32, cpb64;  // c in beta-major order
    DevMem rc_chunk_a;    // u32 [rc_nch_a][3]: recomputed product, alpha-bucket chunks
    DevMem rc_chunk_b;    // u32 [rc_nch_b][3]: beta-bucket chunks (beta-major positions)
    i64 rc_nch_a = 0, rc_nch_b = 0;
    i64 rc_maxdeg = 0;    // largest alpha-single degree of a unique alpha string
    // density matrices: row chunks of the alpha buckets (same alpha string,
    // then alpha single x beta single) and of the beta buckets in beta-major
    // order, each list assigned to the workgroups of a persistent grid
    RdmChunks rdm_sa, rdm_nb, rdm_sb;
    DevMem alpha_b;       // u64 [N]: alpha word of each beta-major position (build, density matrices)
    bool st_have32 = false, st_have64 = false;
};

// Plain-pointer view of a Space for kernels.
struct SpaceView {
    int n;
    i64 N;
    const u64* alpha;
    const u64* beta;
    const u32* ia;
    const u32* ib;
    const u64* ua;
    const u32* aoff;
    const u64* ub;
    const u32* boff;
    const u32* permb;
    const u32* as_ptr;
    const u32* as_idx;
    const u32* bs_ptr;
    const u32* bs_idx;
    const u64* alpha_b;  // alpha word of each beta-major position (null until ensure_alpha_b)
};

struct IntView {
    int n;
    const double* h;
    const double* g;
    const double* jk;
    const double* jj;
    const double* jdiag;
    const double* kdiag;
    const float* g32;
    const float* jk32;
    const float* jj32;
    const float* h32;
};

struct KernelTimer {
    i64 launches = 0;
    double ms = 0.0;
};

struct PendingEvent {
    std::string name;
    hipEvent_t start, stop;
};

// The result of the last selection that did not fit its caller's capacity,
// kept for a retry with enough room on the same inputs (by content), so the
// retry copies it instead of walking again.
struct SelectKept {
    DevMem out;  // u64 [M][2], sorted unique V + C
    i64 M = 0, N = 0;
    u64 dets_hash = 0, c_hash = 0;
    double eps = 0.0;
};

struct hci_ctx_s {
    int n = 0, na = 0, nb = 0;
    int device = 0;
    double ecore = 0.0;
    hci_allocator alloc{};
    bool has_alloc = false;
    Integrals ints;
    Space* space = nullptr;
    SelectKept* sel_kept = nullptr;  // dropped with the space
    struct Pt2Frozen* frozen = nullptr;  // screened PT2 pairs frozen by hci_pt2_freeze
    i64 stored_budget = (i64)64 << 30;
    i64 pt2_budget = (i64)64 << 30;  // screened PT2 pairs held at once
    int stage_wlog = 14;  // log2 of the staged layout's window; 0 = plain CSR
    // pinned, coherent host words the Davidson reduction writes every
    // iteration (four scalars, then a sequence number the host polls)
    double* host_scal = nullptr;
    unsigned long long host_seq = 0;
    // pinned staging for small planner copies (grown on demand, only while
    // no copy through it is pending)
    unsigned char* host_stage = nullptr;
    size_t host_stage_bytes = 0;
    bool timing = false;
    std::map<std::string, KernelTimer> timers;
    std::vector<PendingEvent> pending;
    std::vector<hipEvent_t> event_pool;
};

// allocation through the context allocator
DevMem dev_alloc(hci_ctx_s* ctx, size_t bytes, hipStream_t stream);
// release a cached space
void drop_space(hci_ctx_s* ctx);
// Pinned host memory of at least bytes (the context's staging area; its
// previous contents are lost when it grows).
void* host_staging(hci_ctx_s* ctx, size_t bytes);
// release the frozen PT2 pair set
void drop_frozen(hci_ctx_s* ctx);

// kernel timing hooks (no-ops unless timing is on)
void timer_begin(hci_ctx_s* ctx, const char* name, hipStream_t s, PendingEvent* ev);
void timer_end(hci_ctx_s* ctx, PendingEvent* ev, hipStream_t s);

struct ScopedTimer {
    hci_ctx_s* ctx;
    hipStream_t s;
    PendingEvent ev;
    bool on;
    ScopedTimer(hci_ctx_s* c, const char* name, hipStream_t st) : ctx(c), s(st), on(c->timing) {
        if (on) timer_begin(ctx, name, s, &ev);
    }
    ~ScopedTimer() {
        if (on) timer_end(ctx, &ev, s);
    }
};

// The dispatch packet counts a grid in work-items as a 32-bit number: a
// larger grid would silently run only part of its workgroups, so it is an
// error here.  Kernels that may see more rows than one launch can cover loop
// over them (row_grid below).
inline bool launch_fits(i64 grid, i64 block) { return grid >= 0 && grid * block < ((i64)1 << 32); }
inline bool launch_fits(const dim3& grid, i64 block) {
    return (i64)grid.x * block < ((i64)1 << 32) && (i64)grid.y < ((i64)1 << 32) && (i64)grid.z < ((i64)1 << 32);
}
inline dim3 launch_dim(i64 grid) { return dim3((unsigned)grid); }
inline dim3 launch_dim(const dim3& grid) { return grid; }

#define HCI_LAUNCH(ctx, name, stream, kernel, grid, block, shmem, ...)             \
    do {                                                                          \
        const auto _grid = (grid);                                                \
        const i64 _block = (i64)(block);                                          \
        HCI_REQUIRE(launch_fits(_grid, _block), HCI_E_UNSUPPORTED,                \
                    std::string("launch of ") + (name) + " would exceed 2^32 work-items"); \
        ScopedTimer _st((ctx), (name), (stream));                                 \
        hipLaunchKernelGGL(kernel, launch_dim(_grid), dim3((unsigned)_block), (shmem), (stream), \
                           __VA_ARGS__);                                          \
        HIP_CHECK(hipGetLastError());                                             \
    } while (0)

inline i64 ceil_div(i64 a, i64 b) { return (a + b - 1) / b; }

// Workgroups for `rows` rows at `rows_per_block` per workgroup of `block`
// work-items, clamped below the 2^32 work-item limit of one launch (the
// kernel then strides over the rest).  HCI_ROW_GRID_CAP=<k> clamps to k
// workgroups instead, so that tests exercise the striding on small lists.
inline i64 row_grid(i64 rows, i64 rows_per_block, i64 block) {
    i64 cap = (((i64)1 << 32) - 1) / block;
    if (const char* e = std::getenv("HCI_ROW_GRID_CAP")) {
        const long long k = std::atoll(e);
        if (k > 0 && k < cap) cap = (i64)k;
    }
    const i64 g = ceil_div(rows, rows_per_block);
    return g < cap ? g : cap;
}

inline SpaceView space_view(const Space& s, int n) {
    SpaceView v;
    v.n = n;
    v.N = s.N;
    v.alpha = s.alpha.as<u64>();
    v.beta = s.beta.as<u64>();
    v.ia = s.ia.as<u32>();
    v.ib = s.ib.as<u32>();
    v.ua = s.ua.as<u64>();
    v.aoff = s.aoff.as<u32>();
    v.ub = s.ub.as<u64>();
    v.boff = s.boff.as<u32>();
    v.permb = s.permb.as<u32>();
    v.as_ptr = s.as_ptr.as<u32>();
    v.as_idx = s.as_idx.as<u32>();
    v.bs_ptr = s.bs_ptr.as<u32>();
    v.bs_idx = s.bs_idx.as<u32>();
    v.alpha_b = s.alpha_b.as<u64>();
    return v;
}

inline IntView int_view(const Integrals& I) {
    IntView v;
    v.n = I.n;
    v.h = I.h.as<double>();
    v.g = I.g.as<double>();
    v.jk = I.jk.as<double>();
    v.jj = I.jj.as<double>();
    v.jdiag = I.jdiag.as<double>();
    v.kdiag = I.kdiag.as<double>();
    v.g32 = I.g32.as<float>();
    v.jk32 = I.jk32.as<float>();
    v.jj32 = I.jj32.as<float>();
    v.h32 = I.h32.as<float>();
    return v;
}

// ---------------------------------------------------------------- primitives (prims.hip)
// Exclusive scan of n values; returns the total (synchronises when want_total).
void scan_u32_to_u32(hci_ctx_s* ctx, const u32* in, u32* out, i64 n, hipStream_t s);
void scan_u32_to_i64(hci_ctx_s* ctx, const u32* in, i64* out, i64 n, hipStream_t s);
void scan_i64(hci_ctx_s* ctx, const i64* in, i64* out, i64 n, hipStream_t s);
template <class T>
T read_scalar(const T* dptr, hipStream_t s) {
    T v;
    HIP_CHECK(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return v;
}

// Stable LSD radix sort of (hi, lo) 128-bit keys by (hi, lo) over the low
// `bits` bits of each word, with an optional u32 payload.  Results end in
// keys_hi/keys_lo/vals (the tmp buffers are scratch of the same size).
void radix_sort128(hci_ctx_s* ctx, u64* hi, u64* lo, u32* vals, u64* thi, u64* tlo, u32* tvals,
                   i64 n, int bits_hi, int bits_lo, hipStream_t s);
// Stable LSD radix sort of 64-bit keys by their bytes [byte_lo, byte_hi)
// (the lower bytes keep their input order among equal sort bytes); tmp is
// scratch of n words.
void radix_sort64_bytes(hci_ctx_s* ctx, u64* keys, u64* tmp, i64 n, int byte_lo, int byte_hi, hipStream_t s);
// Remove adjacent duplicates of sorted (hi, lo) keys; returns the unique
// count m and writes out_pairs [m][2] = {hi, lo} only when m <= cap.
i64 unique128_capped(hci_ctx_s* ctx, const u64* hi, const u64* lo, u64* out_pairs, i64 n, i64 cap,
                     hipStream_t s);

// ---------------------------------------------------------------- modules
void integrals_stage(hci_ctx_s* ctx, const double* h, const double* g, hipStream_t s);
Space* get_space(hci_ctx_s* ctx, const u64* dets, i64 n_var, hipStream_t s);
void ensure_diag(hci_ctx_s* ctx, Space* sp, hipStream_t s);
// sp->alpha_b: the alpha word of each beta-major position (cached with the space)
void ensure_alpha_b(hci_ctx_s* ctx, Space* sp, hipStream_t s);
void ensure_csr(hci_ctx_s* ctx, Space* sp, int precision, hipStream_t s);
i64 count_connections(hci_ctx_s* ctx, Space* sp, hipStream_t s);
void sigma_apply(hci_ctx_s* ctx, Space* sp, const double* c, double* sigma, int precision, int mode,
                 hipStream_t s);
int choose_mode(hci_ctx_s* ctx, Space* sp, int precision, int mode, hipStream_t s);
// staged layout (staged.hip): prepare returns false when the space does not
// fit the layout's limits (then the plain CSR is used)
bool staged_prepare(hci_ctx_s* ctx, Space* sp, hipStream_t s);
void staged_ensure_vals(hci_ctx_s* ctx, Space* sp, int precision, hipStream_t s);
// info[8] as documented for hci_layout_info (after the count pass)
void layout_info(hci_ctx_s* ctx, Space* sp, int64_t* info, hipStream_t s);
void staged_apply(hci_ctx_s* ctx, Space* sp, const double* c, double* sigma, int precision,
                  hipStream_t s);
// product with connections and elements regenerated on the fly (no storage)
void recompute_apply(hci_ctx_s* ctx, Space* sp, const double* c, double* sigma, int precision, hipStream_t s);
// lock: nlock orthonormal vectors [nlock][N] to deflate (the states below);
// generic_start: add a fixed pseudo-random 1e-3 component to the start vector
int davidson_run(hci_ctx_s* ctx, Space* sp, double* c, double* e_out, double tol, int max_iter,
                 int precision, int mode, int* iters_out, hipStream_t s, const double* lock = nullptr,
                 int nlock = 0, bool generic_start = false);
double heat_bath_max(hci_ctx_s* ctx, hipStream_t s);
i64 select_run(hci_ctx_s* ctx, const u64* dets, const double* c, i64 N, double eps, u64* out,
               i64 cap, hipStream_t s);
// <S^2> of c on the list (ecore-free, normalised by |c|^2)
double spin_square(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, hipStream_t s);
// union over the states (rows of C [nroots][N]) of the selected sets
i64 select_roots_run(hci_ctx_s* ctx, const u64* dets, const double* C, int nroots, i64 N, double eps,
                     u64* out, i64 cap, hipStream_t s);
void embed_run(hci_ctx_s* ctx, const u64* dets, i64 n, const double* c, const u64* dn, i64 nn,
               double* out, hipStream_t s);

// eps2-screened PT2 pieces of the relaxed gradient on a frozen (V, c, E0),
// in the same budgeted passes as pt2_energy: r = dE2/dc (device [N],
// overwritten), Gamma^{dc} added to dc1/dc2 (bra D_a weighted d_a, ket D_i
// weighted c_i, over the screened pairs) and Gamma^{dd} added to dd1/dd2
// (diagonal of the connected determinants, weights d_a^2); E2 and d.d on the
// host.
void pt2_relaxed_pieces(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, double e0, double eps2,
                        double* r, double* dc1, double* dc2, double* dd1, double* dd2, double* e2_out,
                        double* dd_out, i64* nconn, int* npasses, hipStream_t s);
// Freeze the screened pairs M = {(i, a): fl(|H_ai| |c_i|) > eps2} of (V, c) at
// the current integrals (one pass within the pt2 budget); returns |M|.
i64 pt2_freeze(hci_ctx_s* ctx, const u64* dets, i64 N, u64 hash, const double* c, double eps2, hipStream_t s);
// E2 over the frozen pairs with the current integrals, c and E0 (ecore-free)
double pt2_frozen_energy(hci_ctx_s* ctx, const u64* dets, i64 N, u64 hash, const double* c, double e0,
                         hipStream_t s);
// extrapolation to the full-CI limit: per level (host arrays) the determinant
// count, E_var (ecore included) and E2; fit = {E at E2 = 0, slope, error}
void extrapolate(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, double fraction, int levels,
                 double eps2, double tol, int precision, i64* nvar, double* evar, double* e2, double* fit,
                 hipStream_t s);
// orbital step (active-active rotations): grad = dE/dkappa (n x n), and the
// rotated integrals of the context's h, g under U
void orbital_gradient(hci_ctx_s* ctx, const double* rdm1, const double* rdm2, double* grad, hipStream_t s);
// the same gradient with its partial sums in a fixed device array (no
// allocation); orbital_scratch_setup resolves that array's address on a
// device (called once per device, with the device current, at set-up)
void orbital_gradient_noalloc(hci_ctx_s* ctx, const double* rdm1, const double* rdm2, double* grad,
                              hipStream_t s);
void orbital_scratch_setup(int device);
void rotate_integrals(hci_ctx_s* ctx, const double* U, double* h_out, double* g_out, hipStream_t s);
// device bytes per screened pair while a pass is processed (pairs, sort, segments)
constexpr i64 PT2_BYTES_PER_PAIR = 128;
// E2 of eq. pt_hci (and r = dE2/dc at fixed E0 when r != NULL) in passes over
// hash partitions of the connected determinants sized to ctx->pt2_budget.
double pt2_energy(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, double e0, double eps2,
                  double* r, i64* nconn, int* npasses, hipStream_t s);
// nb batches of nd draws each: sampled E2 estimates at eps2 and eps2_d (host
// arrays e2s, e2sd) from the uniforms u (device [nb][nd]).
void pt2_stochastic(hci_ctx_s* ctx, const u64* dets, i64 N, const double* c, double e0, double eps2,
                    double eps2_d, const double* u, i64 nd, i64 nb, double* e2s, double* e2sd,
                    hipStream_t s);
// Q (H - E) Q z = -Q r on c-perp by preconditioned conjugate gradients;
// returns the number of Hamiltonian products.
int zvector_solve(hci_ctx_s* ctx, Space* sp, const double* c, double e, const double* r, double* z,
                  double tol, int precision, int max_products, hipStream_t s);
// Density matrices of screened pairs (Gamma^{dc} of the PT2 pieces):
// rdm1/rdm2 += sum over the pairs t of w_t <D_a(t)| ops |D_i(t)>, with
// w_t = wa_t c_i(t), D_a = (a_hi, a_lo), i = idx.  The pairs of each pass are
// sorted by excitation class (type and orbitals) and reduced segment by
// segment in a fixed order into per-class tables, which one owner per
// density-matrix entry adds to rdm1/rdm2 at the end: no atomics, the result
// does not depend on scheduling.
struct PairRdm {
    DevMem dtab;  // [3][n^4]: alpha-beta, alpha-alpha, beta-beta doubles by orbitals
    DevMem stab;  // [2][n][n][2n + 1]: singles by (spin, u, v): spectator sums, then the plain sum
};
void pair_rdm_init(hci_ctx_s* ctx, PairRdm& A, hipStream_t s);
void pair_rdm_add(hci_ctx_s* ctx, PairRdm& A, const u64* a_hi, const u64* a_lo, const u32* idx, const double* wa,
                  i64 M, const u64* dets, const double* c, hipStream_t s);
void pair_rdm_finish(hci_ctx_s* ctx, PairRdm& A, double* rdm1, double* rdm2, hipStream_t s);
// rdm1/rdm2 += sum_k wa_k wb_k <D_k| ops |D_k> over the listed determinants
void rdm_add_diag(hci_ctx_s* ctx, const u64* alpha, const u64* beta, const double* wa,
                  const double* wb, i64 M, double* rdm1, double* rdm2, hipStream_t s);
void rdm_compute(hci_ctx_s* ctx, Space* sp, const double* bra, const double* ket, double* rdm1,
                 double* rdm2, hipStream_t s);
