// extern "C" entry points, context lifetime, allocation and kernel timing.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include <vector>
#include <limits>
#include <cmath>
#include "common.h"

namespace {
thread_local std::string g_last_error;

template <class F>
int guarded(F&& f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const HciError& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return HCI_E_NOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return HCI_E_HIP;
    } catch (...) {
        g_last_error = "unknown error";
        return HCI_E_HIP;
    }
}

__global__ void add_scalar_kernel(double* __restrict__ y, double a, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a;
}

__global__ void scale_kernel(const double* __restrict__ x, double a, double* __restrict__ y, i64 n) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

// dg[pqrs] = a * mean of G over the 8 index permutations that leave (pq|rs)
// unchanged for real orbitals
__global__ void sym8_kernel(const double* __restrict__ G, int n, double a, double* __restrict__ out) {
    const i64 n4 = (i64)n * n * n * n;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n4) return;
    const int s = (int)(t % n), r = (int)((t / n) % n), q = (int)((t / n / n) % n),
              p = (int)(t / n / n / n);
    auto at = [&](int a0, int a1, int a2, int a3) {
        return G[(((i64)a0 * n + a1) * n + a2) * n + a3];
    };
    const double v = at(p, q, r, s) + at(q, p, r, s) + at(p, q, s, r) + at(q, p, s, r) +
                     at(r, s, p, q) + at(s, r, p, q) + at(r, s, q, p) + at(s, r, q, p);
    out[t] = a * (v * 0.125);
}

// out[p][q] = a (x[p][q] + x[q][p]) / 2
__global__ void sym2_kernel(const double* __restrict__ x, int n, double a, double* __restrict__ out) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (i64)n * n) return;
    const int p = (int)(t / n), q = (int)(t % n);
    out[t] = a * (0.5 * (x[t] + x[(i64)q * n + p]));
}

// out = a0 A + a1 B + a2 C + a3 D (out may alias A)
__global__ void combine4_kernel(double a0, const double* A, double a1, const double* __restrict__ B,
                                double a2, const double* __restrict__ C, double a3,
                                const double* __restrict__ D, double* out, i64 m) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) out[t] = a0 * A[t] + a1 * B[t] + a2 * C[t] + a3 * D[t];
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

void hci_set_error(const std::string& msg) { g_last_error = msg; }

DevMem& DevMem::operator=(DevMem&& o) noexcept {
    if (this != &o) {
        release();
        ctx = o.ctx;
        ptr = o.ptr;
        bytes = o.bytes;
        o.ctx = nullptr;
        o.ptr = nullptr;
        o.bytes = 0;
    }
    return *this;
}

void DevMem::release() {
    if (ptr && ctx) {
        if (ctx->has_alloc) ctx->alloc.free(ptr, ctx->alloc.user);
        else (void)hipFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
}

DevMem dev_alloc(hci_ctx_s* ctx, size_t bytes, hipStream_t stream) {
    DevMem m;
    m.ctx = ctx;
    m.bytes = bytes ? bytes : 8;
    if (ctx->has_alloc) {
        m.ptr = ctx->alloc.alloc(m.bytes, (void*)stream, ctx->alloc.user);
        if (!m.ptr) throw HciError{HCI_E_NOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes"};
    } else {
        hipError_t e = hipMalloc(&m.ptr, m.bytes);
        if (e != hipSuccess) {
            m.ptr = nullptr;
            (void)hipGetLastError();
            throw HciError{HCI_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
        }
    }
    return m;
}

void* host_staging(hci_ctx_s* ctx, size_t bytes) {
    if (ctx->host_stage_bytes < bytes) {
        if (ctx->host_stage) HIP_CHECK(hipHostFree(ctx->host_stage));
        ctx->host_stage = nullptr;
        ctx->host_stage_bytes = 0;
        const size_t want = std::max<size_t>(bytes, (size_t)1 << 16);
        void* p = nullptr;
        HIP_CHECK(hipHostMalloc(&p, want, hipHostMallocDefault));
        ctx->host_stage = static_cast<unsigned char*>(p);
        ctx->host_stage_bytes = want;
    }
    return ctx->host_stage;
}

void drop_space(hci_ctx_s* ctx) {
    delete ctx->space;
    ctx->space = nullptr;
    delete ctx->sel_kept;
    ctx->sel_kept = nullptr;
}

static hipEvent_t take_event(hci_ctx_s* ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIP_CHECK(hipEventCreate(&e));
    return e;
}

void timer_begin(hci_ctx_s* ctx, const char* name, hipStream_t s, PendingEvent* ev) {
    ev->name = name;
    ev->start = take_event(ctx);
    ev->stop = take_event(ctx);
    HIP_CHECK(hipEventRecord(ev->start, s));
}

void timer_end(hci_ctx_s* ctx, PendingEvent* ev, hipStream_t s) {
    (void)hipEventRecord(ev->stop, s);
    ctx->pending.push_back(*ev);
}

static void timers_collect(hci_ctx_s* ctx) {
    for (auto& p : ctx->pending) {
        HIP_CHECK(hipEventSynchronize(p.stop));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, p.start, p.stop));
        KernelTimer& t = ctx->timers[p.name];
        t.launches += 1;
        t.ms += ms;
        ctx->event_pool.push_back(p.start);
        ctx->event_pool.push_back(p.stop);
    }
    ctx->pending.clear();
}

static void validate_integrals(int norb, const double* h, const double* g) {
    HCI_REQUIRE(h != nullptr && g != nullptr, HCI_E_ARG, "null integral pointer");
    (void)norb;
}

extern "C" {

const char* hci_last_error(void) { return g_last_error.c_str(); }

int hci_ctx_create(int norb, int nalpha, int nbeta, const double* h, const double* g, double ecore,
                   const hci_allocator* alloc, void* stream, hci_ctx* out) {
    return guarded([&]() -> int {
        HCI_REQUIRE(out != nullptr, HCI_E_ARG, "out is NULL");
        *out = nullptr;
        HCI_REQUIRE(norb >= 1 && norb <= 64, HCI_E_ARG, "norb must be in [1, 64]");
        HCI_REQUIRE(nalpha >= 0 && nalpha <= norb && nbeta >= 0 && nbeta <= norb, HCI_E_ARG,
                    "electron counts out of range");
        validate_integrals(norb, h, g);
        hci_ctx_s* ctx = new hci_ctx_s();
        ctx->n = norb;
        ctx->na = nalpha;
        ctx->nb = nbeta;
        ctx->ecore = ecore;
        if (alloc && alloc->alloc && alloc->free) {
            ctx->alloc = *alloc;
            ctx->has_alloc = true;
        }
        HIP_CHECK(hipGetDevice(&ctx->device));
        try {
            orbital_scratch_setup(ctx->device);
            integrals_stage(ctx, h, g, as_stream(stream));
            HIP_CHECK(hipStreamSynchronize(as_stream(stream)));
        } catch (...) {
            delete ctx;
            throw;
        }
        *out = ctx;
        return HCI_OK;
    });
}

int hci_ctx_update_integrals(hci_ctx ctx, const double* h, const double* g, double ecore,
                             void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr, HCI_E_ARG, "null context");
        validate_integrals(ctx->n, h, g);
        drop_space(ctx);
        ctx->ints = Integrals();
        ctx->ecore = ecore;
        integrals_stage(ctx, h, g, as_stream(stream));
        HIP_CHECK(hipStreamSynchronize(as_stream(stream)));
        return HCI_OK;
    });
}

int hci_ctx_destroy(hci_ctx ctx) {
    return guarded([&]() -> int {
        if (!ctx) return HCI_OK;
        (void)hipDeviceSynchronize();
        drop_space(ctx);
        drop_frozen(ctx);
        ctx->ints = Integrals();
        for (auto& p : ctx->pending) {
            (void)hipEventDestroy(p.start);
            (void)hipEventDestroy(p.stop);
        }
        for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
        if (ctx->host_scal) (void)hipHostFree(ctx->host_scal);
        if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
        delete ctx;
        return HCI_OK;
    });
}

int hci_ctx_release_cache(hci_ctx ctx) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr, HCI_E_ARG, "null context");
        (void)hipDeviceSynchronize();
        drop_space(ctx);
        return HCI_OK;
    });
}

int hci_ctx_set_stored_budget(hci_ctx ctx, int64_t bytes) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && bytes >= 0, HCI_E_ARG, "bad context or budget");
        ctx->stored_budget = bytes;
        return HCI_OK;
    });
}

int hci_ctx_set_stage_window(hci_ctx ctx, int log2_window) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr, HCI_E_ARG, "null context");
        HCI_REQUIRE(log2_window == 0 || (log2_window >= 6 && log2_window <= 16), HCI_E_ARG,
                    "stage window must be 0 or 2^6 .. 2^16");
        if (ctx->stage_wlog != log2_window) {
            (void)hipDeviceSynchronize();
            drop_space(ctx);
            ctx->stage_wlog = log2_window;
        }
        return HCI_OK;
    });
}

int hci_ctx_set_timing(hci_ctx ctx, int enable) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr, HCI_E_ARG, "null context");
        ctx->timing = enable != 0;
        return HCI_OK;
    });
}

int hci_ctx_kernel_time(hci_ctx ctx, const char* name, int64_t* launches, double* total_ms,
                        int reset) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && name != nullptr, HCI_E_ARG, "null argument");
        timers_collect(ctx);
        auto it = ctx->timers.find(name);
        if (launches) *launches = it == ctx->timers.end() ? 0 : it->second.launches;
        if (total_ms) *total_ms = it == ctx->timers.end() ? 0.0 : it->second.ms;
        if (reset) ctx->timers.clear();
        return HCI_OK;
    });
}

int hci_select(hci_ctx ctx, const uint64_t* dets, const double* c, int64_t n_var, double eps1,
               uint64_t* out_dets, int64_t cap, int64_t* n_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c && out_dets && n_out, HCI_E_ARG, "null argument");
        HCI_REQUIRE(n_var > 0 && cap >= 0, HCI_E_ARG, "bad sizes");
        HCI_REQUIRE(eps1 >= 0.0, HCI_E_ARG, "eps1 must be >= 0");
        HCI_REQUIRE((const void*)out_dets != (const void*)dets, HCI_E_ARG, "out_dets aliases dets");
        hipStream_t s = as_stream(stream);
        // validation shares the space builder's checks
        get_space(ctx, dets, n_var, s);
        const i64 m = select_run(ctx, dets, c, n_var, eps1, out_dets, cap, s);
        HIP_CHECK(hipStreamSynchronize(s));
        *n_out = m;
        if (m > cap) {
            g_last_error = "capacity " + std::to_string(cap) + " < required " + std::to_string(m);
            return HCI_E_CAPACITY;
        }
        return HCI_OK;
    });
}

int hci_select_roots(hci_ctx ctx, const uint64_t* dets, const double* c, int nroots, int64_t n_var,
                     double eps1, uint64_t* out_dets, int64_t cap, int64_t* n_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c && out_dets && n_out, HCI_E_ARG, "null argument");
        HCI_REQUIRE(n_var > 0 && cap >= 0, HCI_E_ARG, "bad sizes");
        HCI_REQUIRE(nroots >= 1 && nroots <= HCI_MAX_ROOTS, HCI_E_ARG, "nroots must be in [1, 31]");
        HCI_REQUIRE(eps1 >= 0.0, HCI_E_ARG, "eps1 must be >= 0");
        HCI_REQUIRE((const void*)out_dets != (const void*)dets, HCI_E_ARG, "out_dets aliases dets");
        hipStream_t s = as_stream(stream);
        get_space(ctx, dets, n_var, s);
        const i64 m = select_roots_run(ctx, dets, c, nroots, n_var, eps1, out_dets, cap, s);
        HIP_CHECK(hipStreamSynchronize(s));
        *n_out = m;
        if (m > cap) {
            g_last_error = "capacity " + std::to_string(cap) + " < required " + std::to_string(m);
            return HCI_E_CAPACITY;
        }
        return HCI_OK;
    });
}

int hci_embed(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c,
              const uint64_t* dets_new, int64_t n_new, double* c_new, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c && dets_new && c_new, HCI_E_ARG, "null argument");
        HCI_REQUIRE(n_var > 0 && n_new >= n_var, HCI_E_ARG, "bad sizes");
        embed_run(ctx, dets, n_var, c, dets_new, n_new, c_new, as_stream(stream));
        return HCI_OK;
    });
}

int hci_sigma(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double* sigma,
              int precision, int mode, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c && sigma, HCI_E_ARG, "null argument");
        HCI_REQUIRE(precision == HCI_FP64 || precision == HCI_FP32_MIXED, HCI_E_ARG, "bad precision");
        HCI_REQUIRE(mode >= 0 && mode <= 2, HCI_E_ARG, "bad mode");
        HCI_REQUIRE((const void*)c != (const void*)sigma, HCI_E_ARG, "c aliases sigma");
        hipStream_t s = as_stream(stream);
        Space* sp = get_space(ctx, dets, n_var, s);
        const int m = choose_mode(ctx, sp, precision, mode, s);
        sigma_apply(ctx, sp, c, sigma, precision, m, s);
        return HCI_OK;
    });
}

int hci_connections(hci_ctx ctx, const uint64_t* dets, int64_t n_var, int64_t* nnz_out,
                    void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && nnz_out, HCI_E_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        Space* sp = get_space(ctx, dets, n_var, s);
        *nnz_out = count_connections(ctx, sp, s);
        return HCI_OK;
    });
}

int hci_layout_info(hci_ctx ctx, const uint64_t* dets, int64_t n_var, int64_t* info,
                    void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && info, HCI_E_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        Space* sp = get_space(ctx, dets, n_var, s);
        (void)count_connections(ctx, sp, s);
        layout_info(ctx, sp, info, s);
        return HCI_OK;
    });
}

int hci_diagonal(hci_ctx ctx, const uint64_t* dets, int64_t n_var, double* hdiag, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && hdiag, HCI_E_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        Space* sp = get_space(ctx, dets, n_var, s);
        ensure_diag(ctx, sp, s);
        HIP_CHECK(hipMemcpyAsync(hdiag, sp->hdiag.ptr, sizeof(double) * n_var, hipMemcpyDeviceToDevice, s));
        if (ctx->ecore != 0.0)
            HCI_LAUNCH(ctx, "add_scalar", s, add_scalar_kernel, ceil_div(n_var, 256), 256, 0, hdiag,
                       ctx->ecore, (i64)n_var);
        return HCI_OK;
    });
}

int hci_davidson(hci_ctx ctx, const uint64_t* dets, int64_t n_var, double* c_inout, double* e_out,
                 double tol, int max_iter, int precision, int mode, int* iters_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c_inout && e_out, HCI_E_ARG, "null argument");
        HCI_REQUIRE(tol > 0.0 && max_iter > 0, HCI_E_ARG, "tol and max_iter must be positive");
        HCI_REQUIRE(precision == HCI_FP64 || precision == HCI_FP32_MIXED, HCI_E_ARG, "bad precision");
        HCI_REQUIRE(mode >= 0 && mode <= 2, HCI_E_ARG, "bad mode");
        hipStream_t s = as_stream(stream);
        Space* sp = get_space(ctx, dets, n_var, s);
        const int rc = davidson_run(ctx, sp, c_inout, e_out, tol, max_iter, precision, mode,
                                    iters_out, s);
        if (rc == HCI_E_NOCONV) g_last_error = "Davidson did not reach tol within max_iter products";
        return rc;
    });
}

int hci_davidson_roots(hci_ctx ctx, const uint64_t* dets, int64_t n_var, int nroots, double* c_inout,
                       double* e_out, double tol, int max_iter, int precision, int mode, int* iters_out,
                       void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c_inout && e_out, HCI_E_ARG, "null argument");
        HCI_REQUIRE(nroots >= 1 && nroots <= HCI_MAX_ROOTS, HCI_E_ARG, "nroots must be in [1, 31]");
        HCI_REQUIRE(nroots <= n_var, HCI_E_ARG, "nroots exceeds the number of determinants");
        HCI_REQUIRE(tol > 0.0 && max_iter > 0, HCI_E_ARG, "tol and max_iter must be positive");
        HCI_REQUIRE(precision == HCI_FP64 || precision == HCI_FP32_MIXED, HCI_E_ARG, "bad precision");
        HCI_REQUIRE(mode >= 0 && mode <= 2, HCI_E_ARG, "bad mode");
        hipStream_t s = as_stream(stream);
        Space* sp = get_space(ctx, dets, n_var, s);
        int worst = HCI_OK;
        for (int r = 0; r < nroots; ++r) {
            // state r: the lowest eigenpair in the complement of states 0..r-1
            const int rc = davidson_run(ctx, sp, c_inout + (i64)r * n_var, e_out + r, tol, max_iter, precision,
                                        mode, iters_out ? iters_out + r : nullptr, s, c_inout, r, true);
            if (rc != HCI_OK) worst = rc;
        }
        if (worst == HCI_E_NOCONV) g_last_error = "Davidson did not reach tol within max_iter products for a state";
        return worst;
    });
}

int hci_spin_square(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double* s2_out,
                    void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c && s2_out, HCI_E_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        get_space(ctx, dets, n_var, s);  // validates the list
        *s2_out = spin_square(ctx, dets, n_var, c, s);
        return HCI_OK;
    });
}

int hci_rdm12(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* bra, const double* ket,
              double* rdm1, double* rdm2, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && bra && ket && rdm1, HCI_E_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        Space* sp = get_space(ctx, dets, n_var, s);
        rdm_compute(ctx, sp, bra, ket, rdm1, rdm2, s);
        return HCI_OK;
    });
}

int hci_energy_backward(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double e,
                        double grad_e, const double* r, double eps2, double z_tol, int precision,
                        double* dh, double* dg, double* z_out, double* e2_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c && dh && dg, HCI_E_ARG, "null argument");
        HCI_REQUIRE(precision == HCI_FP64 || precision == HCI_FP32_MIXED, HCI_E_ARG, "bad precision");
        hipStream_t s = as_stream(stream);
        Space* sp = get_space(ctx, dets, n_var, s);
        const int n = ctx->n;
        const i64 n2 = (i64)n * n, n4 = n2 * n2;
        DevMem g1 = dev_alloc(ctx, sizeof(double) * n2, s);
        DevMem g2 = dev_alloc(ctx, sizeof(double) * n4, s);
        rdm_compute(ctx, sp, c, c, g1.as<double>(), g2.as<double>(), s);
        if (r == nullptr && !(eps2 > 0.0)) {
            // variational energy: unrelaxed density matrices (eq. vdedk2)
            HCI_LAUNCH(ctx, "bw_sym2", s, sym2_kernel, ceil_div(n2, 256), 256, 0, g1.as<double>(), n,
                       grad_e, dh);
            HCI_LAUNCH(ctx, "bw_sym8", s, sym8_kernel, ceil_div(n4, 256), 256, 0, g2.as<double>(), n,
                       0.5 * grad_e, dg);
            if (e2_out) *e2_out = 0.0;
            HIP_CHECK(hipStreamSynchronize(s));
            return HCI_OK;
        }
        HCI_REQUIRE(z_tol > 0.0, HCI_E_ARG, "z_tol must be positive");
        // relaxed gradient (eq. lambda with lambda_c = z/2 - (d.d) c/2):
        // (1 - d.d) G^cc + G^zc + 2 G^dc + G^dd
        DevMem p1 = dev_alloc(ctx, sizeof(double) * n2, s), p2 = dev_alloc(ctx, sizeof(double) * n4, s);
        DevMem q1 = dev_alloc(ctx, sizeof(double) * n2, s), q2 = dev_alloc(ctx, sizeof(double) * n4, s);
        HIP_CHECK(hipMemsetAsync(p1.ptr, 0, sizeof(double) * n2, s));
        HIP_CHECK(hipMemsetAsync(p2.ptr, 0, sizeof(double) * n4, s));
        HIP_CHECK(hipMemsetAsync(q1.ptr, 0, sizeof(double) * n2, s));
        HIP_CHECK(hipMemsetAsync(q2.ptr, 0, sizeof(double) * n4, s));
        const double* rr = r;
        double dd = 0.0, e2 = 0.0;
        DevMem rbuf;
        if (eps2 > 0.0) {
            // r, E2, d.d, Gamma^{dc} and Gamma^{dd} in the budgeted passes of the PT2
            rbuf = dev_alloc(ctx, sizeof(double) * n_var, s);
            pt2_relaxed_pieces(ctx, dets, n_var, c, e - ctx->ecore, eps2, rbuf.as<double>(), p1.as<double>(),
                               p2.as<double>(), q1.as<double>(), q2.as<double>(), &e2, &dd, nullptr, nullptr, s);
            rr = rbuf.as<double>();
        }
        DevMem zbuf;
        double* z = z_out;
        if (!z) {
            zbuf = dev_alloc(ctx, sizeof(double) * n_var, s);
            z = zbuf.as<double>();
        }
        const int prod = zvector_solve(ctx, sp, c, e, rr, z, z_tol, precision, 100000, s);
        DevMem t1 = dev_alloc(ctx, sizeof(double) * n2, s), t2 = dev_alloc(ctx, sizeof(double) * n4, s);
        rdm_compute(ctx, sp, z, c, t1.as<double>(), t2.as<double>(), s);
        HCI_LAUNCH(ctx, "bw_combine", s, combine4_kernel, ceil_div(n2, 256), 256, 0, 1.0 - dd,
                   g1.as<double>(), 1.0, t1.as<double>(), 2.0, p1.as<double>(), 1.0, q1.as<double>(),
                   g1.as<double>(), n2);
        HCI_LAUNCH(ctx, "bw_combine", s, combine4_kernel, ceil_div(n4, 256), 256, 0, 1.0 - dd,
                   g2.as<double>(), 1.0, t2.as<double>(), 2.0, p2.as<double>(), 1.0, q2.as<double>(),
                   g2.as<double>(), n4);
        HCI_LAUNCH(ctx, "bw_sym2", s, sym2_kernel, ceil_div(n2, 256), 256, 0, g1.as<double>(), n, grad_e,
                   dh);
        HCI_LAUNCH(ctx, "bw_sym8", s, sym8_kernel, ceil_div(n4, 256), 256, 0, g2.as<double>(), n,
                   0.5 * grad_e, dg);
        if (e2_out) *e2_out = e2;
        HIP_CHECK(hipStreamSynchronize(s));
        if (prod < 0) {
            g_last_error = "z-vector solve did not reach z_tol (outputs hold the last iterate)";
            return HCI_E_NOCONV;
        }
        return HCI_OK;
    });
}

int hci_pt2_freeze(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double eps2,
                   int64_t* n_pairs_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c, HCI_E_ARG, "null argument");
        HCI_REQUIRE(eps2 >= 0.0, HCI_E_ARG, "eps2 must be >= 0");
        hipStream_t s = as_stream(stream);
        Space* sp = get_space(ctx, dets, n_var, s);
        const i64 M = pt2_freeze(ctx, dets, n_var, sp->hash, c, eps2, s);
        HIP_CHECK(hipStreamSynchronize(s));
        if (n_pairs_out) *n_pairs_out = M;
        return HCI_OK;
    });
}

int hci_energy(hci_ctx ctx, const uint64_t* dets, int64_t n_var, double* c_inout, double tol, int max_iter,
               int precision, int mode, double eps2, int frozen, double* e_out, int* iters_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c_inout && e_out, HCI_E_ARG, "null argument");
        HCI_REQUIRE(tol > 0.0 && max_iter > 0, HCI_E_ARG, "tol and max_iter must be positive");
        HCI_REQUIRE(precision == HCI_FP64 || precision == HCI_FP32_MIXED, HCI_E_ARG, "bad precision");
        HCI_REQUIRE(mode >= 0 && mode <= 2, HCI_E_ARG, "bad mode");
        HCI_REQUIRE(eps2 >= 0.0, HCI_E_ARG, "eps2 must be >= 0");
        hipStream_t s = as_stream(stream);
        Space* sp = get_space(ctx, dets, n_var, s);
        const u64 hash = sp->hash;
        double evar = 0.0;
        const int rc = davidson_run(ctx, sp, c_inout, &evar, tol, max_iter, precision, mode, iters_out, s);
        double e2 = 0.0;
        if (frozen) {
            e2 = pt2_frozen_energy(ctx, dets, n_var, hash, c_inout, evar - ctx->ecore, s);
        } else if (eps2 > 0.0) {
            e2 = pt2_energy(ctx, dets, n_var, c_inout, evar - ctx->ecore, eps2, nullptr, nullptr, nullptr, s);
        }
        HIP_CHECK(hipStreamSynchronize(s));
        e_out[0] = evar;
        e_out[1] = e2;
        e_out[2] = evar + e2;
        if (rc == HCI_E_NOCONV) g_last_error = "Davidson did not reach tol within max_iter products";
        return rc;
    });
}

int hci_pt2(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double e0,
            double eps2, double* e2_out, double* r_out, int64_t* n_conn_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c && e2_out, HCI_E_ARG, "null argument");
        HCI_REQUIRE(eps2 >= 0.0, HCI_E_ARG, "eps2 must be >= 0");
        hipStream_t s = as_stream(stream);
        get_space(ctx, dets, n_var, s);  // validation
        i64 nc = 0;
        const double e2 = pt2_energy(ctx, dets, n_var, c, e0 - ctx->ecore, eps2, r_out, &nc, nullptr, s);
        HIP_CHECK(hipStreamSynchronize(s));
        *e2_out = e2;
        if (n_conn_out) *n_conn_out = nc;
        return HCI_OK;
    });
}

int hci_extrapolate(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double fraction,
                    int levels, double eps2, double tol, int precision, int64_t* nvar_out, double* evar_out,
                    double* e2_out, double* fit_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c && nvar_out && evar_out && e2_out && fit_out, HCI_E_ARG,
                    "null argument");
        HCI_REQUIRE(levels >= 2 && fraction > 0.0 && fraction < 1.0, HCI_E_ARG,
                    "need levels >= 2 and 0 < fraction < 1");
        HCI_REQUIRE(eps2 >= 0.0 && tol > 0.0, HCI_E_ARG, "need eps2 >= 0 and tol > 0");
        HCI_REQUIRE(precision == HCI_FP64 || precision == HCI_FP32_MIXED, HCI_E_ARG, "bad precision");
        hipStream_t s = as_stream(stream);
        get_space(ctx, dets, n_var, s);  // validation
        drop_space(ctx);
        static_assert(sizeof(int64_t) == sizeof(i64), "host counts");
        extrapolate(ctx, dets, n_var, c, fraction, levels, eps2, tol, precision, (i64*)nvar_out, evar_out,
                    e2_out, fit_out, s);
        HIP_CHECK(hipStreamSynchronize(s));
        return HCI_OK;
    });
}

int hci_orbital_gradient(hci_ctx ctx, const double* rdm1, const double* rdm2, double* grad, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && rdm1 && rdm2 && grad, HCI_E_ARG, "null argument");
        orbital_gradient(ctx, rdm1, rdm2, grad, as_stream(stream));
        return HCI_OK;
    });
}

int hci_orbital_gradient_noalloc(hci_ctx ctx, const double* rdm1, const double* rdm2, double* grad,
                                 void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && rdm1 && rdm2 && grad, HCI_E_ARG, "null argument");
        orbital_gradient_noalloc(ctx, rdm1, rdm2, grad, as_stream(stream));
        return HCI_OK;
    });
}

int hci_rotate_integrals(hci_ctx ctx, const double* U, double* h_out, double* g_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && U && h_out && g_out, HCI_E_ARG, "null argument");
        rotate_integrals(ctx, U, h_out, g_out, as_stream(stream));
        return HCI_OK;
    });
}

int hci_ctx_set_pt2_budget(hci_ctx ctx, int64_t bytes) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && bytes > 0, HCI_E_ARG, "bad context or budget");
        ctx->pt2_budget = bytes;
        return HCI_OK;
    });
}

int hci_pt2_stochastic(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double e0,
                       double eps2, double eps2_d, const double* u, int64_t n_samp, int64_t n_batch,
                       double* e2s_out, double* e2sd_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c && u && e2s_out && e2sd_out, HCI_E_ARG, "null argument");
        HCI_REQUIRE(eps2 >= 0.0 && eps2_d >= eps2, HCI_E_ARG, "need 0 <= eps2 <= eps2_d");
        HCI_REQUIRE(n_samp >= 2 && n_batch >= 1, HCI_E_ARG, "need n_samp >= 2 and n_batch >= 1");
        hipStream_t s = as_stream(stream);
        get_space(ctx, dets, n_var, s);  // validation
        pt2_stochastic(ctx, dets, n_var, c, e0 - ctx->ecore, eps2, eps2_d, u, n_samp, n_batch, e2s_out,
                       e2sd_out, s);
        HIP_CHECK(hipStreamSynchronize(s));
        return HCI_OK;
    });
}

int hci_pt2_semistochastic(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double e0,
                           double eps2, double eps2_d, const double* u, int64_t n_samp, int64_t n_batch,
                           double* e2_out, double* err_out, double* e2d_out, void* stream) {
    return guarded([&]() -> int {
        HCI_REQUIRE(ctx != nullptr && dets && c && u && e2_out, HCI_E_ARG, "null argument");
        HCI_REQUIRE(eps2 >= 0.0 && eps2_d >= eps2, HCI_E_ARG, "need 0 <= eps2 <= eps2_d");
        HCI_REQUIRE(n_samp >= 2 && n_batch >= 1, HCI_E_ARG, "need n_samp >= 2 and n_batch >= 1");
        hipStream_t s = as_stream(stream);
        get_space(ctx, dets, n_var, s);  // validation
        const double e0v = e0 - ctx->ecore;
        const double e2d = pt2_energy(ctx, dets, n_var, c, e0v, eps2_d, nullptr, nullptr, nullptr, s);
        std::vector<double> a(n_batch), b(n_batch);
        pt2_stochastic(ctx, dets, n_var, c, e0v, eps2, eps2_d, u, n_samp, n_batch, a.data(), b.data(), s);
        HIP_CHECK(hipStreamSynchronize(s));
        double mean = 0.0;
        for (int64_t k = 0; k < n_batch; ++k) mean += a[k] - b[k];
        mean /= (double)n_batch;
        double var = 0.0;
        for (int64_t k = 0; k < n_batch; ++k) var += (a[k] - b[k] - mean) * (a[k] - b[k] - mean);
        *e2_out = e2d + mean;
        if (err_out)
            *err_out = n_batch > 1 ? std::sqrt(var / (double)(n_batch - 1)) / std::sqrt((double)n_batch)
                                   : std::numeric_limits<double>::quiet_NaN();
        if (e2d_out) *e2d_out = e2d;
        return HCI_OK;
    });
}

}  // extern "C"
