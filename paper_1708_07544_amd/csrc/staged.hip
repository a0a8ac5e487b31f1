// Stored Hamiltonian in an alpha-bucket-staged layout, for the product
// sigma = H c inside the Davidson solver (Sec. "Variational Stage") over all
// single and double connections of V (Sec. "Computational Details").
//
// V is sorted by (alpha, beta), so each alpha string owns a contiguous bucket
// of rows.  A connection (i, j) of a row i in bucket A is either
//   S: j in A itself, or in a bucket A' one alpha single away from A (alpha
//      single with the same beta, or alpha single x beta single), or
//   G: an alpha double with the same beta string.
// The S buckets of A -- A, then its alpha-single neighbours in adjacency
// order -- are laid end to end; position P of j in that concatenation is
// stored as window P >> w and local column P & (2^w - 1) (u16).  A G entry
// stores the offset of j inside the row's beta group (u16), which is
// contiguous in the beta-major order.
//
// A workgroup owns up to 1024 rows of one bucket.  For each window it copies
// that slice of c into LDS (whole buckets are contiguous in c, so the copy
// streams), then its waves stream their rows' entries of the window and
// gather c_j from LDS.  G entries gather from a beta-major copy of c.  Each
// product therefore reads per entry only the value and a 2-byte column from
// HBM; the gathers that bound the plain CSR product (every row touches
// hundreds of distinct cache lines of c) move to LDS.
//
// Entries of a row are grouped by segment (windows in order, G last); the
// layout is built by a count pass, a scan, an integer column pass and a
// separate element pass per precision.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "slater.h"

namespace {


constexpr int ST_CPY = 8;          // window copy: gathers in flight per thread
constexpr int ST_ROW_BLOCK = 256;  // build passes: one wavefront per row
constexpr int ST_ROWS_PER_BLOCK = ST_ROW_BLOCK / HCI_WAVE;
constexpr int ST_BLOCK = 1024;     // product: 16 wavefronts
constexpr int ST_WAVES = ST_BLOCK / HCI_WAVE;

// LDS for a bucket's stage ranges in the product (two u32 per range; a
// bucket has at most N_alpha (n - N_alpha) alpha-single neighbours)
inline size_t st_range_lds(const hci_ctx_s* ctx) {
    return sizeof(u32) * 2 * (size_t)(1 + ctx->na * (ctx->n - ctx->na));
}
constexpr u32 ST_CHUNK = 64 * ST_WAVES;  // rows per workgroup (64 per wavefront)
constexpr int GT_BLOCK = 512;      // beta-group product: 8 wavefronts
constexpr int GT_WAVES = GT_BLOCK / HCI_WAVE;
constexpr u32 GT_CHUNK = 64 * GT_WAVES;
constexpr u32 ST_MAX_SEG = 64;           // segments per row (lane-held cursors)
constexpr u32 ST_MAX_GROUP = 65536;      // beta-group offsets are u16
constexpr u32 ST_VEC = 8;                // entries per lane per load; segments padded to it

struct StView {
    u32 wlog;
    i64 nua, nub;
    const u32* gcptr;
    const u32* xpos;
    const u32* len;
    const u32* nseg;
    const u32* cptr;
    const i64* rsb;
    const i64* sstart;  // absolute start of every (row, segment), padded to ST_VEC
    const u32* segcnt;  // entries of every (row, segment) before padding
    const u16* cols;
    const u32* chunk;   // [workgroups][3]: bucket, first row, end row
    const u32* gchunk;  // [beta-group workgroups][4]: rows [k0, k1) and c slice [s0, s1), beta-major
};

StView st_view(const Space& s) {
    StView v;
    v.wlog = s.st_wlog;
    v.nua = s.nua;
    v.nub = s.nub;
    v.gcptr = s.st_gcptr.as<u32>();
    v.xpos = s.st_xpos.as<u32>();
    v.len = s.st_len.as<u32>();
    v.nseg = s.st_nseg.as<u32>();
    v.cptr = s.st_cptr.as<u32>();
    v.rsb = s.st_rsb.as<i64>();
    v.sstart = s.st_sstart.as<i64>();
    v.segcnt = s.st_segcnt.as<u32>();
    v.cols = s.st_cols.as<u16>();
    v.chunk = s.st_chunk.as<u32>();
    v.gchunk = s.st_gchunk.as<u32>();
    return v;
}

// One thread per bucket: stage ranges, stage length, segment count and
// workgroup count; one thread per beta group: group size limit.  flags[0]
// counts buckets with too many segments, flags[1] oversized beta groups,
// flags[2] holds the largest stage length, flags[3] the largest beta group.
__global__ void st_meta_kernel(SpaceView S, u32 wlog, u32* __restrict__ xpos, u32* __restrict__ len,
                               u32* __restrict__ nseg, u32* __restrict__ nchunk,
                               u32* __restrict__ gnchunk, i64 nua, i64 nub,
                               unsigned long long* __restrict__ flags) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nua) {
        const u32 a = (u32)t;
        const u32 t0 = S.as_ptr[a], t1 = S.as_ptr[a + 1];
        const u32 xb = t0 + a;
        u32 pos = S.aoff[a + 1] - S.aoff[a];
        xpos[xb] = 0;
        for (u32 k = t0; k < t1; ++k) {
            xpos[xb + 1 + (k - t0)] = pos;
            const u32 a2 = S.as_idx[k];
            pos += S.aoff[a2 + 1] - S.aoff[a2];
        }
        len[a] = pos;
        const u32 ns = ((pos + (1u << wlog) - 1u) >> wlog) + 1u;
        nseg[a] = ns;
        nchunk[a] = (S.aoff[a + 1] - S.aoff[a] + ST_CHUNK - 1) / ST_CHUNK;
        if (ns > ST_MAX_SEG) atomicAdd(&flags[0], 1ull);
        atomicMax(&flags[2], (unsigned long long)pos);
    }
    if (t < nub) {
        const u32 gs = S.boff[t + 1] - S.boff[t];
        gnchunk[t] = (gs + GT_CHUNK - 1) / GT_CHUNK;
        atomicMax(&flags[3], (unsigned long long)gs);
        if (gs > ST_MAX_GROUP) atomicAdd(&flags[1], 1ull);
    }
}

// Chunk tables: for workgroup w of the staged kernels its bucket a and rows
// [r0, r1) (chunks of ST_CHUNK rows of one bucket); for workgroup w of the
// beta-group kernel its group b and positions [k0, k1) in beta-major order.
__global__ void st_chunk_table_kernel(const u32* __restrict__ cptr, const u32* __restrict__ off, i64 nbkt,
                                      u32 chunk, u32* __restrict__ table) {
    const i64 a = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nbkt) return;
    for (u32 w = cptr[a]; w < cptr[a + 1]; ++w) {
        const u32 r0 = off[a] + (w - cptr[a]) * chunk;
        table[3 * (i64)w] = (u32)a;
        table[3 * (i64)w + 1] = r0;
        table[3 * (i64)w + 2] = min(r0 + chunk, off[a + 1]);
    }
}

__global__ void st_row_nseg_kernel(const u32* __restrict__ ia, const u32* __restrict__ nseg, i64 N,
                                   u32* __restrict__ out) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) out[i] = nseg[ia[i]];
    if (i == N) out[i] = 0;
}

// Every j != i of V at excitation degree <= 2 from row i, with its segment
// and u16 column in the staged layout.  The whole wavefront calls this for
// one row; vis(ok, j, aj, bj, seg, col) is invoked wave-uniformly with each
// lane's own candidate.  Discovery order (deterministic): same-alpha bucket,
// same-beta group, then (AB) alpha-single neighbours in adjacency order.
template <bool AB, class Visitor>
__device__ __forceinline__ void enumerate_row_staged(const SpaceView& S, const u32* __restrict__ xpos,
                                                     u32 wlog, u32 gseg, u32 i, Visitor& vis) {
    const int lane = lane_id();
    const u32 wmask = (1u << wlog) - 1u;
    const u64 A = S.alpha[i], B = S.beta[i];
    const u32 a = S.ia[i], b = S.ib[i];
    const u32 t0 = S.as_ptr[a], t1 = S.as_ptr[a + 1];
    const u32 xb = t0 + a;
    {  // same alpha string: stage range 0
        const u32 lo = S.aoff[a], hi = S.aoff[a + 1];
        for (u32 base = lo; base < hi; base += HCI_WAVE) {
            const u32 j = base + lane;
            bool ok = j < hi && j != i;
            u64 bj = 0;
            if (ok) {
                bj = S.beta[j];
                ok = popc64(B ^ bj) <= 4;
            }
            const u32 P = j - lo;
            vis(ok, j, A, bj, P >> wlog, P & wmask);
        }
    }
    {  // same beta string: an alpha single lies in a staged neighbour bucket,
       // an alpha double goes to the beta-group segment
        const u32 lo = S.boff[b], hi = S.boff[b + 1];
        for (u32 base = lo; base < hi; base += HCI_WAVE) {
            const u32 k = base + lane;
            bool ok = k < hi;
            u32 j = 0, seg = gseg, col = k - lo;
            u64 aj = 0;
            if (ok) {
                aj = S.alpha_b[k];  // contiguous; the position j only for the hits
                const int d = popc64(A ^ aj);
                ok = d == 2 || d == 4;  // (d = 0 is the row itself: same alpha and beta)
                if (ok) {
                    j = S.permb[k];
                    if (d == 2) {
                        const u32 a2 = S.ia[j];
                        const u32 r = lower_bound_u32(S.as_idx + t0, t1 - t0, a2);
                        const u32 P = xpos[xb + 1 + r] + (j - S.aoff[a2]);
                        seg = P >> wlog;
                        col = P & wmask;
                    }
                }
            }
            vis(ok, j, aj, B, seg, col);
        }
    }
    if constexpr (AB) {  // one alpha and one beta excitation: stage ranges 1, 2, ...
        const u32 s0 = S.bs_ptr[b], s1 = S.bs_ptr[b + 1];
        const u32 nbs = s1 - s0;
        for (u32 t = t0; t < t1; ++t) {
            const u32 a2 = S.as_idx[t];
            const u64 A2 = S.ua[a2];
            const u32 lo = S.aoff[a2], hi = S.aoff[a2 + 1];
            const u32 len = hi - lo;
            const u32 P0 = xpos[xb + 1 + (t - t0)];
            if (len <= 4u * nbs) {
                for (u32 base = lo; base < hi; base += HCI_WAVE) {
                    const u32 j = base + lane;
                    bool ok = j < hi;
                    u64 bj = 0;
                    if (ok) {
                        bj = S.beta[j];
                        ok = popc64(B ^ bj) == 2;
                    }
                    const u32 P = P0 + (j - lo);
                    vis(ok, j, A2, bj, P >> wlog, P & wmask);
                }
            } else {
                for (u32 base = s0; base < s1; base += HCI_WAVE) {
                    const u32 k = base + lane;
                    bool ok = k < s1;
                    u32 j = 0;
                    u64 bj = 0;
                    if (ok) {
                        bj = S.ub[S.bs_idx[k]];
                        const u32 pos = lower_bound_u64(S.beta + lo, len, bj);
                        ok = pos < len && S.beta[lo + pos] == bj;
                        j = lo + pos;
                    }
                    const u32 P = P0 + (j - lo);
                    vis(ok, j, A2, bj, P >> wlog, P & wmask);
                }
            }
        }
    }
}

// Count pass: lane s of the wavefront holds the count of segment s.
struct StCountVis {
    u32 cnt = 0;
    __device__ __forceinline__ void operator()(bool ok, u32, u64, u64, u32 seg, u32) {
        u64 m = ballot(ok);
        while (m) {
            const u32 s = (u32)__shfl((int)seg, ctz64(m), HCI_WAVE);
            const u64 ms = ballot(ok && seg == s);
            if ((u32)lane_id() == s) cnt += (u32)__popcll(ms);
            m &= ~ms;
        }
    }
};

__device__ __forceinline__ u32 pad_vec(u32 x) { return (x + ST_VEC - 1u) & ~(ST_VEC - 1u); }

// Count pass: entries of every (row, segment) (without the alpha single x
// beta single part when AB is false: st_ab_kernel adds it).
template <bool AB>
__global__ void __launch_bounds__(ST_ROW_BLOCK) st_count_kernel(SpaceView S, StView T,
                                                                u32* __restrict__ segcnt) {
    const i64 i = (i64)blockIdx.x * ST_ROWS_PER_BLOCK + threadIdx.x / HCI_WAVE;
    if (i >= S.N) return;
    const u32 lane = (u32)lane_id();
    const u32 ns = T.nseg[S.ia[i]];
    StCountVis v;
    enumerate_row_staged<AB>(S, T.xpos, T.wlog, ns - 1u, (u32)i, v);
    if (lane < ns) segcnt[T.rsb[i] + lane] = v.cnt;
}

// Per row the padded totals of its windows (wtot) and of its beta-group
// segment (gtot).
__global__ void __launch_bounds__(ST_ROW_BLOCK) st_totals_kernel(SpaceView S, StView T,
                                                                 u32* __restrict__ wtot,
                                                                 u32* __restrict__ gtot) {
    const i64 i = (i64)blockIdx.x * ST_ROWS_PER_BLOCK + threadIdx.x / HCI_WAVE;
    if (i >= S.N) return;
    const u32 lane = (u32)lane_id();
    const u32 ns = T.nseg[S.ia[i]];
    const u32 cnt = lane < ns ? T.segcnt[T.rsb[i] + lane] : 0u;
    const u32 wsum = (u32)wave_sum_u64(lane + 1 < ns ? pad_vec(cnt) : 0u);
    const u32 g = (u32)__shfl((int)pad_vec(cnt), (int)ns - 1, HCI_WAVE);
    if (lane == 0) {
        wtot[i] = wsum;
        gtot[i] = g;
    }
}

// Window-major placement: a workgroup per chunk of rows writes, window by
// window, the rows' segment starts consecutively (so the product streams
// each window of a chunk as one contiguous region).
__global__ void __launch_bounds__(ST_BLOCK) st_place_kernel(SpaceView S, StView T,
                                                            const i64* __restrict__ wscan,
                                                            i64* __restrict__ sstart) {
    __shared__ u32 part[ST_WAVES];
    const u32 tid = threadIdx.x;
    // bucket and rows of this workgroup's chunk
    const u32* ce = T.chunk + 3 * (i64)blockIdx.x;
    const u32 a = ce[0], r0 = ce[1], r1 = ce[2];
    const u32 nw = T.nseg[a] - 1u;
    const u32 row = r0 + tid;
    const bool has = row < r1;
    const i64 sb = has ? T.rsb[row] : 0;
    i64 base = wscan[r0];  // windows of all earlier rows
    for (u32 g = 0; g < nw; ++g) {
        const u32 x = has ? pad_vec(T.segcnt[sb + g]) : 0u;
        // exclusive block scan of x in row order
        u32 incl = x;
#pragma unroll
        for (int off = 1; off < HCI_WAVE; off <<= 1) {
            const u32 y = (u32)__shfl_up((int)incl, off, HCI_WAVE);
            if ((int)lane_id() >= off) incl += y;
        }
        if (lane_id() == HCI_WAVE - 1) part[tid / HCI_WAVE] = incl;
        __syncthreads();
        u32 before = 0, total = 0;
        for (int q = 0; q < ST_WAVES; ++q) {
            const u32 pq = part[q];
            if (q < (int)(tid / HCI_WAVE)) before += pq;
            total += pq;
        }
        if (has) sstart[sb + g] = base + before + incl - x;
        base += total;
        __syncthreads();
    }
}

// Beta-group segments follow all windows, in beta-major row order.
__global__ void st_place_g_kernel(SpaceView S, StView T, const i64* __restrict__ gscan, i64 gbase,
                                  i64* __restrict__ sstart) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S.N) return;
    const u32 i = S.permb[k];
    sstart[T.rsb[i] + T.nseg[S.ia[i]] - 1] = gbase + gscan[k];
}

__global__ void st_gather_u32_kernel(const u32* __restrict__ src, const u32* __restrict__ perm, i64 n,
                                     u32* __restrict__ dst) {
    const i64 k = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[perm[k]];
    if (k == n) dst[k] = 0;
}

// Column pass: lane s holds the start and the cursor of segment s.
struct StFillVis {
    u16* cols;
    i64 so;
    u32 cur = 0;
    __device__ __forceinline__ void operator()(bool ok, u32, u64, u64, u32 seg, u32 col) {
        u64 m = ballot(ok);
        while (m) {
            const u32 s = (u32)__shfl((int)seg, ctz64(m), HCI_WAVE);
            const bool mine = ok && seg == s;
            const u64 ms = ballot(mine);
            const i64 at = __shfl(so + (i64)cur, (int)s, HCI_WAVE);
            if (mine) cols[at + rank_in(ms)] = (u16)col;
            if ((u32)lane_id() == s) cur += (u32)__popcll(ms);
            m &= ~ms;
        }
    }
};

template <bool AB>
__global__ void __launch_bounds__(ST_ROW_BLOCK) st_cols_kernel(SpaceView S, StView T,
                                                               u16* __restrict__ cols,
                                                               u32* __restrict__ fill) {
    const i64 i = (i64)blockIdx.x * ST_ROWS_PER_BLOCK + threadIdx.x / HCI_WAVE;
    if (i >= S.N) return;
    const u32 lane = (u32)lane_id();
    const u32 ns = T.nseg[S.ia[i]];
    const i64 sb = T.rsb[i];
    StFillVis v{cols, lane < ns ? T.sstart[sb + lane] : (i64)0};
    enumerate_row_staged<AB>(S, T.xpos, T.wlog, ns - 1u, (u32)i, v);
    if (lane < ns) fill[sb + lane] = v.cur;
}

// The fill must reproduce the count pass segment by segment; padding entries
// get column 0 (their element is 0).
__global__ void __launch_bounds__(ST_ROW_BLOCK) st_pad_kernel(SpaceView S, StView T,
                                                              const u32* __restrict__ fill,
                                                              u16* __restrict__ cols,
                                                              unsigned long long* __restrict__ bad) {
    const i64 i = (i64)blockIdx.x * ST_ROWS_PER_BLOCK + threadIdx.x / HCI_WAVE;
    if (i >= S.N) return;
    const u32 lane = (u32)lane_id();
    const u32 ns = T.nseg[S.ia[i]];
    if (lane >= ns) return;
    const i64 slot = T.rsb[i] + lane;
    const u32 cnt = T.segcnt[slot], cur = fill[slot];
    if (cur != cnt) {
        atomicAdd(bad, 1ull);
        return;
    }
    const i64 so = T.sstart[slot];
    for (i64 k = so + cur; k < so + pad_vec(cnt); ++k) cols[k] = 0;
}

// Alpha single x beta single connections of a chunk of rows (one alpha
// bucket A), G alpha neighbours at a time, through the LDS beta-string maps
// of build_beta_maps: every beta single of row i's beta string (adjacency
// order) resolves to its position in the neighbour bucket with two LDS reads
// instead of a search.  MODE 0 adds to the segment counts, MODE 1 continues
// the column cursors left by st_cols_kernel.
template <int MODE>
__global__ void __launch_bounds__(ST_BLOCK) st_ab_kernel(SpaceView S, StView T, u32 W, u32 G,
                                                         u32* __restrict__ segcnt, u32* __restrict__ fill,
                                                         u16* __restrict__ cols) {
    extern __shared__ __align__(16) unsigned char st_smem[];
    u32* bm = reinterpret_cast<u32*>(st_smem);
    u16* pre = reinterpret_cast<u16*>(bm + (size_t)G * W);
    const u32 tid = threadIdx.x;
    const u32 lane = (u32)lane_id();
    const u32 wave = tid / HCI_WAVE;
    // bucket and rows of this workgroup's chunk
    const u32* ce = T.chunk + 3 * (i64)blockIdx.x;
    const u32 a = ce[0], r0 = ce[1], r1 = ce[2];
    const u32 t0 = S.as_ptr[a], deg = S.as_ptr[a + 1] - t0;
    const u32 xb = t0 + a;
    const u32 ns = T.nseg[a];
    const u32 wmask = (1u << T.wlog) - 1u;
    for (u32 tg0 = 0; tg0 < deg; tg0 += G) {
        const u32 tg1 = min(tg0 + G, deg);
        __syncthreads();  // the previous maps are consumed
        build_beta_maps<ST_BLOCK>(S, t0, tg0, tg1, W, bm, pre, tid);
        for (u32 row = r0 + wave; row < r1; row += ST_WAVES) {
            const i64 sb = T.rsb[row];
            const u32 b = S.ib[row];
            const u32 s0 = S.bs_ptr[b], s1 = S.bs_ptr[b + 1];
            StCountVis vc;
            StFillVis vf{cols, 0, 0u};
            if constexpr (MODE == 1) {
                vf.so = lane < ns ? T.sstart[sb + lane] : (i64)0;
                vf.cur = lane < ns ? fill[sb + lane] : 0u;
            }
            // neighbour by neighbour, beta singles in adjacency order: the
            // discovery order of the search in enumerate_row_staged
            auto visit = [&](u32 t, bool has, u32 bp) {
                const u32 q = t - tg0;
                const u32 w = bp >> 5, bit = bp & 31u;
                const u32 word = has ? bm[q * W + w] : 0u;
                const bool ok = ((word >> bit) & 1u) != 0u;
                const u32 pos = ok ? (u32)pre[q * W + w] + (u32)__popc(word & ((1u << bit) - 1u)) : 0u;
                const u32 P = T.xpos[xb + 1 + t] + pos;
                if constexpr (MODE == 0) vc(ok, 0u, 0ull, 0ull, P >> T.wlog, P & wmask);
                else vf(ok, 0u, 0ull, 0ull, P >> T.wlog, P & wmask);
            };
            if (s1 - s0 <= (u32)HCI_WAVE) {
                const bool has = s0 + lane < s1;
                const u32 bp = has ? S.bs_idx[s0 + lane] : 0u;
                for (u32 t = tg0; t < tg1; ++t) visit(t, has, bp);
            } else {
                for (u32 t = tg0; t < tg1; ++t) {
                    for (u32 base = s0; base < s1; base += HCI_WAVE) {
                        const u32 k = base + lane;
                        const bool has = k < s1;
                        visit(t, has, has ? S.bs_idx[k] : 0u);
                    }
                }
            }
            if constexpr (MODE == 0) {
                if (lane < ns && vc.cnt) segcnt[sb + lane] += vc.cnt;
            } else {
                if (lane < ns) fill[sb + lane] = vf.cur;
            }
        }
    }
}

// Single excitations queued across the rows of a wavefront: lane l holds the
// l-th queued entry (its index, the bra's beta string and the ket), so the
// costly single elements are evaluated 64 at a time however few each row
// segment has (the bra's alpha string is the workgroup's bucket).
struct BraSinglesQueue {
    int n = 0;  // queued, wave-uniform
    i64 k = 0;
    u64 bi = 0, a = 0, b = 0;
    __device__ __forceinline__ bool full_for(u64 m) const { return n + popc64(m) > HCI_WAVE; }
    __device__ __forceinline__ void push(u64 m, i64 kk, u64 bra_b, u64 aa, u64 bb) {
        const int cnt = popc64(m);
        const int l = lane_id();
        const bool mine = l >= n && l < n + cnt;
        const int src = mine ? nth_set_bit(m, l - n) : l;
        const i64 sk = __shfl(kk, src, HCI_WAVE);
        const u64 sa = __shfl(aa, src, HCI_WAVE);
        const u64 sb = __shfl(bb, src, HCI_WAVE);
        if (mine) {
            k = sk;
            bi = bra_b;  // wave-uniform: the row being scanned
            a = sa;
            b = sb;
        }
        n += cnt;
    }
};

// Element pass: decode each stored column back to its determinant and
// evaluate H_ij in float64 (written rounded to float32 when OUT & 1, as
// float64 when OUT & 2; the float32-mixed solver refines with float64
// products, so it asks for both).  Workgroup = a chunk of rows of one alpha
// bucket, as the product, and window by window as the product: the window's
// beta strings are copied into LDS once, with the index of the stage range
// holding each position in the word's top 16 bits when n <= 48 (else a
// binary search over the bucket's ranges finds it), then every row of the
// chunk decodes its segment of that window from LDS.  A range other than the
// bucket's own is an alpha single A -> A' whose hole, particle and phase are
// fixed, so its alpha x beta doubles need only the beta part: sign_A sign_B
// (rp|sq) with the range's (r, p) offset into g kept in LDS.  The beta-group
// segments (same beta string) read the ket's alpha string from the
// beta-major copy of the alpha words.
constexpr u32 ST_NO_LINK = 0xffffffffu;
constexpr int ST_PACK_MAXN = 48;  // beta strings leave 16 bits for the range index

template <int OUT>
__global__ void __launch_bounds__(ST_BLOCK) st_vals_kernel(SpaceView S, IntView I, StView T,
                                                           float* __restrict__ v32,
                                                           double* __restrict__ v64) {
    extern __shared__ __align__(16) unsigned char st_smem[];
    const u32 tid = threadIdx.x;
    const u32 wave = tid / HCI_WAVE;
    const int lane = lane_id();
    const int n = I.n;
    const bool pk = n <= ST_PACK_MAXN;
    constexpr u64 LOW48 = (1ull << 48) - 1ull;
    // bucket and rows of this workgroup's chunk
    const u32* ce = T.chunk + 3 * (i64)blockIdx.x;
    const u32 a = ce[0], r0 = ce[1], r1 = ce[2];
    const u32 t0 = S.as_ptr[a];
    const u32 nr = 1u + S.as_ptr[a + 1] - t0;
    const u32 ns = T.nseg[a];
    const u32 slen = T.len[a];
    const u32 wsize = 1u << T.wlog;
    const u64 ai = S.ua[a];
    u64* sbeta = reinterpret_cast<u64*>(st_smem);  // [wsize] beta strings of the window
    u64* ralpha = sbeta + wsize;                    // [nr] alpha string of each range
    u32* rx = reinterpret_cast<u32*>(ralpha + nr);  // [nr] stage start of each range
    u32* rsrc = rx + nr;                            // [nr] first row of each range
    u32* rinfo = rsrc + nr;                         // [nr] g offset of (r, p) | sign bit
    for (u32 e = tid; e < nr; e += ST_BLOCK) {
        const u32 a2 = e == 0 ? a : S.as_idx[t0 + e - 1];
        const u64 A2 = S.ua[a2];
        ralpha[e] = A2;
        rx[e] = T.xpos[t0 + a + e];
        rsrc[e] = S.aoff[a2];
        u32 info = ST_NO_LINK;
        if (e > 0) {  // alpha single p -> r
            const u64 xa = ai ^ A2;
            const int p = ctz64(ai & xa), r = ctz64(A2 & xa);
            info = (u32)gidx(n, r, p, 0, 0) | (sign_between(ai, p, r) < 0.0 ? 0x80000000u : 0u);
        }
        rinfo[e] = info;
    }
    BraSinglesQueue q;
    auto flush = [&]() {
        if (lane < q.n) {
            const double v = hij_f64(I, ai, q.bi, q.a, q.b);
            if constexpr ((OUT & 1) != 0) v32[q.k] = (float)v;
            if constexpr ((OUT & 2) != 0) v64[q.k] = v;
        }
        q.n = 0;
    };
    // one row segment [k0, k0 + cnt) padded to ST_VEC; dec(k, col) -> (aj,
    // bj, the range's link info or ST_NO_LINK)
    auto segment = [&](u64 bi, i64 k0, u32 cnt, auto dec) {
        const i64 k1 = k0 + pad_vec(cnt);
        const i64 kr = k0 + cnt;
        // uniform trip count: the queue's ballots and shuffles need every lane
        for (i64 kb = k0; kb < k1; kb += HCI_WAVE) {
            const i64 k = kb + lane;
            double v = 0.0;
            bool single = false;
            u64 aj = 0, bj = 0;
            if (k < kr) {
                u32 info;
                dec(T.cols[k], aj, bj, info);
                const u64 xb = bi ^ bj;
                if (info != ST_NO_LINK) {  // alpha single, or alpha x beta double
                    single = xb == 0;
                    if (!single) {
                        const int qo = ctz64(bi & xb), so = ctz64(bj & xb);
                        const double sa = (info >> 31) ? -1.0 : 1.0;
                        v = (sa * sign_between(bi, qo, so)) * I.g[(i64)(info & 0x7fffffffu) + (i64)so * n + qo];
                    }
                } else {
                    single = popc64(ai ^ aj) + popc64(xb) == 2;
                    if (!single) v = hij_f64(I, ai, bi, aj, bj);
                }
            }
            if (!single && k < k1) {
                if constexpr ((OUT & 1) != 0) v32[k] = (float)v;
                if constexpr ((OUT & 2) != 0) v64[k] = v;
            }
            const u64 m = ballot(single);
            if (m) {
                if (q.full_for(m)) flush();
                q.push(m, k, bi, aj, bj);
            }
        }
    };
    for (u32 g = 0; g + 1 < ns; ++g) {
        __syncthreads();  // the previous window is consumed (and the ranges are in)
        const u32 wstart = g << T.wlog;
        const u32 wend = min(wstart + wsize, slen);
        u32 p = wstart + tid;
        if (p < wend) {
            // last range starting at or before p, then forward as p grows
            u32 e = 0, hi = nr - 1u;
            while (e < hi) {
                const u32 mid = (e + hi + 1u) >> 1;
                if (rx[mid] <= p) e = mid;
                else hi = mid - 1u;
            }
            for (; p < wend; p += ST_CPY * ST_BLOCK) {
                u32 sidx[ST_CPY], ej[ST_CPY];
#pragma unroll
                for (int j = 0; j < ST_CPY; ++j) {
                    const u32 pj = p + (u32)j * ST_BLOCK;
                    while (e + 1 < nr && rx[e + 1] <= pj) ++e;
                    sidx[j] = rsrc[e] + (pj - rx[e]);
                    ej[j] = e;
                }
                u64 v[ST_CPY];
#pragma unroll
                for (int j = 0; j < ST_CPY; ++j) v[j] = p + (u32)j * ST_BLOCK < wend ? S.beta[sidx[j]] : 0ull;
#pragma unroll
                for (int j = 0; j < ST_CPY; ++j) {
                    const u32 pj = p + (u32)j * ST_BLOCK;
                    if (pj < wend) sbeta[pj - wstart] = pk ? v[j] | ((u64)ej[j] << 48) : v[j];
                }
            }
        }
        __syncthreads();
        for (u32 i = r0 + wave; i < r1; i += ST_WAVES) {
            const i64 slot = T.rsb[i] + g;
            segment(S.beta[i], T.sstart[slot], T.segcnt[slot], [&](u32 col, u64& aj, u64& bj, u32& info) {
                const u64 w = sbeta[col];
                u32 lo;
                if (pk) {
                    lo = (u32)(w >> 48);
                    bj = w & LOW48;
                } else {
                    const u32 P = wstart + col;
                    u32 hi = nr - 1u;  // last range starting at or before P
                    lo = 0;
                    while (lo < hi) {
                        const u32 mid = (lo + hi + 1u) >> 1;
                        if (rx[mid] <= P) lo = mid;
                        else hi = mid - 1u;
                    }
                    bj = w;
                }
                aj = ralpha[lo];
                info = rinfo[lo];
            });
        }
    }
    for (u32 i = r0 + wave; i < r1; i += ST_WAVES) {
        const u64 bi = S.beta[i];
        const i64 slot = T.rsb[i] + ns - 1u;
        const u64* __restrict__ ga = S.alpha_b + S.boff[S.ib[i]];
        segment(bi, T.sstart[slot], T.segcnt[slot], [&](u32 col, u64& aj, u64& bj, u32& info) {
            aj = ga[col];
            bj = bi;
            info = ST_NO_LINK;
        });
    }
    if (q.n) flush();
}

__global__ void st_sum_kernel(const u32* __restrict__ x, i64 n, unsigned long long* __restrict__ out) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    u64 v = i < n ? (u64)x[i] : 0ull;
    v = wave_sum_u64(v);
    if (lane_id() == 0 && v) atomicAdd(out, (unsigned long long)v);
}

// Entries stored in each row's beta-group segment (last segment).
__global__ void st_gentries_kernel(SpaceView S, StView T, unsigned long long* __restrict__ out) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    u64 v = 0;
    if (i < S.N) v = pad_vec(T.segcnt[T.rsb[i] + T.nseg[S.ia[i]] - 1]);
    v = wave_sum_u64(v);
    if (lane_id() == 0 && v) atomicAdd(out, (unsigned long long)v);
}

// c (float64) -> the product's alpha-major and beta-major copies.
template <class CT>
__global__ void st_prep_kernel(const double* __restrict__ c, const u32* __restrict__ permb, i64 N,
                               CT* __restrict__ cx, CT* __restrict__ cpb) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (cx) cx[i] = (CT)c[i];
    cpb[i] = (CT)c[permb[i]];
}

// ST_VEC = 8 consecutive stored entries (aligned), kept as loaded: the eight
// u16 columns packed in one 128-bit word and the raw values; widened to
// float64 only in the multiply-add (fewer live registers per step in flight).
template <class VT>
struct Entries8;
template <>
struct Entries8<float> {
    uint4 c;
    float4 a, b;
    __device__ __forceinline__ void load(const u16* __restrict__ cols, const float* __restrict__ vals) {
        c = *reinterpret_cast<const uint4*>(cols);
        a = *reinterpret_cast<const float4*>(vals);
        b = *reinterpret_cast<const float4*>(vals + 4);
    }
    template <class CT>
    __device__ __forceinline__ double dot(const CT* __restrict__ x, double t) const {
        t += (double)a.x * (double)x[c.x & 0xffffu];
        t += (double)a.y * (double)x[c.x >> 16];
        t += (double)a.z * (double)x[c.y & 0xffffu];
        t += (double)a.w * (double)x[c.y >> 16];
        t += (double)b.x * (double)x[c.z & 0xffffu];
        t += (double)b.y * (double)x[c.z >> 16];
        t += (double)b.z * (double)x[c.w & 0xffffu];
        t += (double)b.w * (double)x[c.w >> 16];
        return t;
    }
};
template <>
struct Entries8<double> {
    uint4 c;
    double2 a, b, d, e;
    __device__ __forceinline__ void load(const u16* __restrict__ cols, const double* __restrict__ vals) {
        c = *reinterpret_cast<const uint4*>(cols);
        a = *reinterpret_cast<const double2*>(vals);
        b = *reinterpret_cast<const double2*>(vals + 2);
        d = *reinterpret_cast<const double2*>(vals + 4);
        e = *reinterpret_cast<const double2*>(vals + 6);
    }
    template <class CT>
    __device__ __forceinline__ double dot(const CT* __restrict__ x, double t) const {
        t += a.x * (double)x[c.x & 0xffffu];
        t += a.y * (double)x[c.x >> 16];
        t += b.x * (double)x[c.y & 0xffffu];
        t += b.y * (double)x[c.y >> 16];
        t += d.x * (double)x[c.z & 0xffffu];
        t += d.y * (double)x[c.z >> 16];
        t += e.x * (double)x[c.w & 0xffffu];
        t += e.y * (double)x[c.w >> 16];
        return t;
    }
};
static_assert(ST_VEC == 8, "the product kernels read entries in groups of 8");

// Sum of a value over groups of SUB consecutive lanes (result in every lane).
template <int SUB>
__device__ __forceinline__ double group_sum_f64(double v) {
#pragma unroll
    for (int off = SUB / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, HCI_WAVE);
    return v;
}

// Product kernel.  Workgroup = up to 1024 rows of one bucket; wavefront w owns
// rows r0 + w + 16 q (lane q holds that row's accumulator, so every wavefront
// has work even in small buckets); SUB lanes stream one row's segment at a
// time.
template <class VT, class CT, int SUB>
__global__ void __launch_bounds__(ST_BLOCK) st_spmv_kernel(SpaceView S, StView T,
                                                           const VT* __restrict__ vals,
                                                           const CT* __restrict__ cx,
                                                           const double* __restrict__ c,
                                                           const double* __restrict__ hd,
                                                           double* __restrict__ sigma) {
    extern __shared__ __align__(16) unsigned char st_smem[];
    CT* stage = reinterpret_cast<CT*>(st_smem);
    constexpr int GROUPS = HCI_WAVE / SUB;  // rows in flight per wavefront
    const u32 tid = threadIdx.x;
    const int lane = lane_id();
    const u32 wave = tid / HCI_WAVE;
    // bucket and rows of this workgroup's chunk
    const u32* ce = T.chunk + 3 * (i64)blockIdx.x;
    const u32 a = ce[0], r0 = ce[1], r1 = ce[2];
    const u32 t0 = S.as_ptr[a];
    const u32 nr = 1u + S.as_ptr[a + 1] - t0;
    const u32* xs = T.xpos + t0 + a;
    const u32 ns = T.nseg[a];
    const u32 slen = T.len[a];
    const u32 wsize = 1u << T.wlog;
    // rows r0 + wave + ST_WAVES q (q < 64) belong to this wavefront; lane q holds
    // row q's metadata and accumulator
    const u32 nrows = r1 - r0;
    const int nrw = wave < nrows ? (int)((nrows - wave + ST_WAVES - 1) / ST_WAVES) : 0;
    const u32 row = r0 + wave + ST_WAVES * (u32)lane;
    const bool has = lane < nrw;
    const i64 sb = has ? T.rsb[row] : 0;
    // the bucket's stage ranges (start within the slice, first row of the
    // range's bucket) in LDS after the window, read once per workgroup
    u32* rx = reinterpret_cast<u32*>(st_smem + (sizeof(CT) << T.wlog));
    u32* rsrc = rx + nr;
    for (u32 e = tid; e < nr; e += ST_BLOCK) {
        rx[e] = xs[e];
        rsrc[e] = S.aoff[e == 0 ? a : S.as_idx[t0 + e - 1]];
    }
    double acc = 0.0;
    for (u32 g = 0; g + 1 < ns; ++g) {
        __syncthreads();  // the previous window is consumed (and the ranges are in)
        const u32 wstart = g << T.wlog;
        const u32 wend = min(wstart + wsize, slen);
        u32 p = wstart + tid;
        if (p < wend) {
            // last range starting at or before p
            u32 e = 0, hi = nr - 1u;
            while (e < hi) {
                const u32 mid = (e + hi + 1u) >> 1;
                if (rx[mid] <= p) e = mid;
                else hi = mid - 1u;
            }
            // ST_CPY independent gathers in flight per thread, then the stores
            for (; p < wend; p += ST_CPY * ST_BLOCK) {
                u32 sidx[ST_CPY];
#pragma unroll
                for (int j = 0; j < ST_CPY; ++j) {
                    const u32 pj = p + (u32)j * ST_BLOCK;
                    while (e + 1 < nr && rx[e + 1] <= pj) ++e;
                    sidx[j] = rsrc[e] + (pj - rx[e]);
                }
                CT v[ST_CPY];
#pragma unroll
                for (int j = 0; j < ST_CPY; ++j) v[j] = p + (u32)j * ST_BLOCK < wend ? cx[sidx[j]] : (CT)0;
#pragma unroll
                for (int j = 0; j < ST_CPY; ++j) {
                    const u32 pj = p + (u32)j * ST_BLOCK;
                    if (pj < wend) stage[pj - wstart] = v[j];
                }
            }
        }
        __syncthreads();
        const i64 mk0 = has ? T.sstart[sb + g] : (i64)0;
        const i64 mk1 = mk0 + (has ? pad_vec(T.segcnt[sb + g]) : 0u);
        for (int qb = 0; qb < nrw; qb += GROUPS) {
            const int q = qb + lane / SUB;
            const int sl = lane % SUB;
            const i64 k0 = __shfl(mk0, q, HCI_WAVE);
            const i64 k1s = __shfl(mk1, q, HCI_WAVE);
            const i64 k1 = q < nrw ? k1s : k0;
            double t = 0.0;
            // two steps per trip: both loads in flight before the first use
            for (i64 k = k0 + ST_VEC * sl; k < k1; k += 2 * ST_VEC * SUB) {
                Entries8<VT> e1, e2;
                const i64 k2 = k + ST_VEC * SUB;
                const bool two = k2 < k1;
                e1.load(T.cols + k, vals + k);
                if (two) e2.load(T.cols + k2, vals + k2);
                t = e1.dot(stage, t);
                if (two) t = e2.dot(stage, t);
            }
            t = group_sum_f64<SUB>(t);
            const double v = __shfl(t, ((lane - qb) * SUB) & (HCI_WAVE - 1), HCI_WAVE);
            if (lane >= qb && lane < qb + GROUPS) acc += v;
        }
    }
    if (has) sigma[row] = hd[row] * c[row] + acc;
}

// Beta-group product: in beta-major order the alpha doubles with the same
// beta string form diagonal blocks, one per beta group.  A workgroup owns up
// to GT_CHUNK rows of one group, copies the group's slice of the beta-major c
// into LDS when it fits the window (else gathers it from global memory) and
// adds each row's G segment to sigma (after the staged kernel).
template <class VT, class CT, int SUB, bool LDS>
__device__ __forceinline__ double g_rows(const StView& T, const VT* __restrict__ vals,
                                         const CT* __restrict__ src, i64 mk0, i64 mk1, u32 base,
                                         int nrw, int lane) {
    constexpr int GROUPS = HCI_WAVE / SUB;
    double acc = 0.0;
    for (int qb = 0; qb < nrw; qb += GROUPS) {
        const int q = qb + lane / SUB;
        const int sl = lane % SUB;
        const i64 k0 = __shfl(mk0, q, HCI_WAVE);
        const i64 k1s = __shfl(mk1, q, HCI_WAVE);
        const i64 k1 = q < nrw ? k1s : k0;
        // the row's group starts base entries into the slice
        const CT* __restrict__ rsrc = src + (u32)__shfl((int)base, q, HCI_WAVE);
        double t = 0.0;
        for (i64 k = k0 + ST_VEC * sl; k < k1; k += 2 * ST_VEC * SUB) {
            Entries8<VT> e1, e2;
            const i64 k2 = k + ST_VEC * SUB;
            const bool two = k2 < k1;
            e1.load(T.cols + k, vals + k);
            if (two) e2.load(T.cols + k2, vals + k2);
            t = e1.dot(rsrc, t);
            if (two) t = e2.dot(rsrc, t);
        }
        t = group_sum_f64<SUB>(t);
        const double v = __shfl(t, ((lane - qb) * SUB) & (HCI_WAVE - 1), HCI_WAVE);
        if (lane >= qb && lane < qb + GROUPS) acc += v;
    }
    return acc;
}

template <class VT, class CT, int SUB>
__global__ void __launch_bounds__(GT_BLOCK) st_spmv_g_kernel(SpaceView S, StView T,
                                                             const VT* __restrict__ vals,
                                                             const CT* __restrict__ cpb, u32 cap,
                                                             double* __restrict__ sigma) {
    extern __shared__ __align__(16) unsigned char st_smem[];
    CT* stage = reinterpret_cast<CT*>(st_smem);
    const u32 tid = threadIdx.x;
    const int lane = lane_id();
    const u32 wave = tid / HCI_WAVE;
    // rows [k0, k1) (beta-major order) of this workgroup and the slice
    // [s0, s1) of the beta-major c they read: whole small groups packed
    // together, or part of a large group with the whole group's slice
    const u32* ce = T.gchunk + 4 * (i64)blockIdx.x;
    const u32 k0 = ce[0], k1 = ce[1], s0 = ce[2], s1 = ce[3];
    const u32 slen = s1 - s0;
    const bool in_lds = slen <= cap;
    if (in_lds) {
        for (u32 p = tid; p < slen; p += GT_BLOCK) stage[p] = cpb[s0 + p];
    }
    __syncthreads();
    const u32 nrows = k1 - k0;
    const int nrw = wave < nrows ? (int)((nrows - wave + GT_WAVES - 1) / GT_WAVES) : 0;
    const bool has = lane < nrw;
    const u32 i = has ? S.permb[k0 + wave + GT_WAVES * (u32)lane] : 0u;
    i64 mk0 = 0, mk1 = 0;
    u32 base = 0;
    if (has) {
        const i64 slot = T.rsb[i] + T.nseg[S.ia[i]] - 1;
        mk0 = T.sstart[slot];
        mk1 = mk0 + pad_vec(T.segcnt[slot]);
        base = S.boff[S.ib[i]] - s0;
    }
    const double acc = in_lds ? g_rows<VT, CT, SUB, true>(T, vals, stage, mk0, mk1, base, nrw, lane)
                              : g_rows<VT, CT, SUB, false>(T, vals, cpb + s0, mk0, mk1, base, nrw, lane);
    if (has) sigma[i] += acc;
}

constexpr int ST_SUB = 32;

template <class VT, class CT>
void launch_spmv(hci_ctx_s* ctx, Space* sp, const char* name, const char* gname, const VT* vals,
                 const CT* cx, const CT* cpb, const double* c, double* sigma, hipStream_t s) {
    const size_t shmem = (sizeof(CT) << sp->st_wlog) + st_range_lds(ctx);
    // the beta-group kernel stages whole groups up to the largest one (groups
    // beyond the window gather from global memory)
    const u32 cap = (u32)std::min<i64>((i64)1 << sp->st_wlog, std::max<i64>(sp->st_gmax, GT_CHUNK));
    const size_t gshmem = sizeof(CT) * (cap > 0 ? cap : 1);
    auto kern = st_spmv_kernel<VT, CT, ST_SUB>;
    // beta-group rows are short (a few hundred entries): 16 lanes per row
    auto gkern = st_spmv_g_kernel<VT, CT, 16>;
    HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
    HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(gkern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)gshmem));
    HCI_LAUNCH(ctx, name, s, kern, sp->st_nchunk, ST_BLOCK, shmem, space_view(*sp, ctx->n),
               st_view(*sp), vals, cx, c, sp->hdiag.as<double>(), sigma);
    HCI_LAUNCH(ctx, gname, s, gkern, sp->st_gnchunk, GT_BLOCK, gshmem, space_view(*sp, ctx->n),
               st_view(*sp), vals, cpb, cap, sigma);
}

size_t ab_lds(const Space& sp) { return (size_t)6 * sp.st_abW * sp.st_abG; }

size_t vals_lds(const hci_ctx_s* ctx, u32 wlog) {
    // window of beta strings, then 20 B per range (alpha string, stage start,
    // first row, link info)
    return (sizeof(u64) << wlog) + st_range_lds(ctx) / 8 * 20;
}

}  // namespace

bool staged_prepare(hci_ctx_s* ctx, Space* sp, hipStream_t s) {
    const int wlog = ctx->stage_wlog;
    if (wlog == 0 || sp->N < 1) return false;
    int dev = 0, max_shared = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&max_shared, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if ((i64)vals_lds(ctx, (u32)wlog) > (i64)max_shared) return false;
    const i64 N = sp->N, nua = sp->nua, nub = sp->nub;
    // the build passes take one wavefront per row in one launch
    if (ceil_div(N, ST_ROWS_PER_BLOCK) * ST_ROW_BLOCK >= ((i64)1 << 32)) return false;
    ensure_alpha_b(ctx, sp, s);  // the same-beta scans read the alpha words in beta-major order
    SpaceView S = space_view(*sp, ctx->n);
    sp->st_wlog = (u32)wlog;
    sp->st_xpos = dev_alloc(ctx, sizeof(u32) * (nua + sp->n_as), s);
    sp->st_len = dev_alloc(ctx, sizeof(u32) * nua, s);
    sp->st_nseg = dev_alloc(ctx, sizeof(u32) * nua, s);
    DevMem nchunk = dev_alloc(ctx, sizeof(u32) * (nua + 1), s);
    DevMem gnchunk = dev_alloc(ctx, sizeof(u32) * (nub + 1), s);
    HIP_CHECK(hipMemsetAsync(gnchunk.as<u32>() + nub, 0, sizeof(u32), s));
    DevMem flags = dev_alloc(ctx, sizeof(u64) * 4, s);
    HIP_CHECK(hipMemsetAsync(flags.ptr, 0, sizeof(u64) * 4, s));
    HIP_CHECK(hipMemsetAsync(nchunk.as<u32>() + nua, 0, sizeof(u32), s));
    const i64 m = nua > nub ? nua : nub;
    HCI_LAUNCH(ctx, "st_meta", s, st_meta_kernel, ceil_div(m, 256), 256, 0, S, (u32)wlog,
               sp->st_xpos.as<u32>(), sp->st_len.as<u32>(), sp->st_nseg.as<u32>(), nchunk.as<u32>(),
               gnchunk.as<u32>(), nua, nub, (unsigned long long*)flags.as<u64>());
    u64 fl[4];
    HIP_CHECK(hipMemcpyAsync(fl, flags.ptr, sizeof(fl), hipMemcpyDeviceToHost, s));
    sp->st_gmax = (i64)fl[3];
    HIP_CHECK(hipStreamSynchronize(s));
    if (fl[0] != 0 || fl[1] != 0) {
        sp->st_xpos.release();
        sp->st_len.release();
        sp->st_nseg.release();
        return false;
    }
    sp->st_cptr = dev_alloc(ctx, sizeof(u32) * (nua + 1), s);
    scan_u32_to_u32(ctx, nchunk.as<u32>(), sp->st_cptr.as<u32>(), nua + 1, s);
    sp->st_nchunk = read_scalar(sp->st_cptr.as<u32>() + nua, s);
    sp->st_gcptr = dev_alloc(ctx, sizeof(u32) * (nub + 1), s);
    scan_u32_to_u32(ctx, gnchunk.as<u32>(), sp->st_gcptr.as<u32>(), nub + 1, s);
    sp->st_gnchunk = read_scalar(sp->st_gcptr.as<u32>() + nub, s);
    sp->st_chunk = dev_alloc(ctx, sizeof(u32) * 3 * (sp->st_nchunk > 0 ? sp->st_nchunk : 1), s);
    HCI_LAUNCH(ctx, "st_meta", s, st_chunk_table_kernel, ceil_div(nua, 256), 256, 0, sp->st_cptr.as<u32>(),
               sp->aoff.as<u32>(), nua, (u32)ST_CHUNK, sp->st_chunk.as<u32>());
    {
        // beta-group workgroups, in beta-major order: consecutive groups of at
        // most GT_CHUNK rows together packed into one workgroup (their slices
        // of the beta-major c are contiguous); a larger group in parts of
        // GT_CHUNK rows, each with the whole group's slice
        std::vector<u32> boff((size_t)nub + 1);
        HIP_CHECK(hipMemcpyAsync(boff.data(), sp->boff.ptr, sizeof(u32) * (nub + 1), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        std::vector<u32> tab;
        for (i64 b = 0; b < nub;) {
            if (boff[b + 1] - boff[b] > GT_CHUNK) {
                for (u32 k0 = boff[b]; k0 < boff[b + 1]; k0 += GT_CHUNK)
                    tab.insert(tab.end(), {k0, std::min<u32>(k0 + GT_CHUNK, boff[b + 1]), boff[b], boff[b + 1]});
                ++b;
                continue;
            }
            i64 e = b + 1;
            while (e < nub && boff[e + 1] - boff[b] <= GT_CHUNK) ++e;
            tab.insert(tab.end(), {boff[b], boff[e], boff[b], boff[e]});
            b = e;
        }
        sp->st_gnchunk = (i64)(tab.size() / 4);
        sp->st_gchunk = dev_alloc(ctx, sizeof(u32) * (tab.empty() ? 4 : tab.size()), s);
        if (!tab.empty())
            HIP_CHECK(hipMemcpyAsync(sp->st_gchunk.ptr, tab.data(), sizeof(u32) * tab.size(),
                                     hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));  // tab leaves scope
    }
    // segment slots per row
    DevMem rn = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    HCI_LAUNCH(ctx, "st_row_nseg", s, st_row_nseg_kernel, ceil_div(N + 1, 256), 256, 0,
               sp->ia.as<u32>(), sp->st_nseg.as<u32>(), N, rn.as<u32>());
    sp->st_rsb = dev_alloc(ctx, sizeof(i64) * (N + 1), s);
    scan_u32_to_i64(ctx, rn.as<u32>(), sp->st_rsb.as<i64>(), N + 1, s);
    const i64 nslots = read_scalar(sp->st_rsb.as<i64>() + N, s);
    sp->st_nslots = nslots;
    sp->st_sstart = dev_alloc(ctx, sizeof(i64) * (nslots > 0 ? nslots : 1), s);
    sp->st_segcnt = dev_alloc(ctx, sizeof(u32) * (nslots > 0 ? nslots : 1), s);
    // LDS beta-string bitmaps for the alpha single x beta single part: u32
    // words + u16 prefix counts per neighbour, within 64 KB per workgroup
    sp->st_abW = 0;
    sp->st_abG = 0;
    const char* force_search = std::getenv("HCI_AB_SEARCH");  // "1": always search (tests)
    if (nub <= 65535 && !(force_search && force_search[0] == '1')) {
        const i64 W = ceil_div(nub, 32);
        const i64 dmax = (i64)ctx->na * (ctx->n - ctx->na);
        const i64 G = std::min<i64>((std::min<i64>(65536, max_shared) - 1024) / (6 * W), std::max<i64>(dmax, 1));
        if (G >= 1) {
            sp->st_abW = (u32)W;
            sp->st_abG = (u32)G;
        }
    }
    const i64 rgrid = ceil_div(N, ST_ROWS_PER_BLOCK);
    // count pass: per (row, segment) entries, per row padded window / group totals
    if (sp->st_abW) {
        HCI_LAUNCH(ctx, "conn_count", s, st_count_kernel<false>, rgrid, ST_ROW_BLOCK, 0, S, st_view(*sp),
                   sp->st_segcnt.as<u32>());
        HCI_LAUNCH(ctx, "conn_count", s, st_ab_kernel<0>, sp->st_nchunk, ST_BLOCK, ab_lds(*sp), S,
                   st_view(*sp), sp->st_abW, sp->st_abG, sp->st_segcnt.as<u32>(), (u32*)nullptr,
                   (u16*)nullptr);
    } else {
        HCI_LAUNCH(ctx, "conn_count", s, st_count_kernel<true>, rgrid, ST_ROW_BLOCK, 0, S, st_view(*sp),
                   sp->st_segcnt.as<u32>());
    }
    DevMem wtot = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    DevMem gtot = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    HIP_CHECK(hipMemsetAsync(wtot.as<u32>() + N, 0, sizeof(u32), s));
    HCI_LAUNCH(ctx, "conn_count", s, st_totals_kernel, rgrid, ST_ROW_BLOCK, 0, S, st_view(*sp),
               wtot.as<u32>(), gtot.as<u32>());
    // windows: chunk by chunk in row order, window-major inside each chunk
    DevMem wscan = dev_alloc(ctx, sizeof(i64) * (N + 1), s);
    scan_u32_to_i64(ctx, wtot.as<u32>(), wscan.as<i64>(), N + 1, s);
    const i64 wtotal = read_scalar(wscan.as<i64>() + N, s);
    HCI_LAUNCH(ctx, "st_place", s, st_place_kernel, sp->st_nchunk, ST_BLOCK, 0, S, st_view(*sp),
               wscan.as<i64>(), sp->st_sstart.as<i64>());
    // beta-group segments after them, in beta-major row order
    DevMem gperm = dev_alloc(ctx, sizeof(u32) * (N + 1), s);
    HCI_LAUNCH(ctx, "st_place", s, st_gather_u32_kernel, ceil_div(N + 1, 256), 256, 0, gtot.as<u32>(),
               sp->permb.as<u32>(), N, gperm.as<u32>());
    DevMem gscan = dev_alloc(ctx, sizeof(i64) * (N + 1), s);
    scan_u32_to_i64(ctx, gperm.as<u32>(), gscan.as<i64>(), N + 1, s);
    const i64 gtotal = read_scalar(gscan.as<i64>() + N, s);
    HCI_LAUNCH(ctx, "st_place", s, st_place_g_kernel, ceil_div(N, 256), 256, 0, S, st_view(*sp),
               gscan.as<i64>(), wtotal, sp->st_sstart.as<i64>());
    sp->st_nnz = wtotal + gtotal;
    // connections without padding: sum of the segment counts
    DevMem total = dev_alloc(ctx, sizeof(u64), s);
    HIP_CHECK(hipMemsetAsync(total.ptr, 0, sizeof(u64), s));
    HCI_LAUNCH(ctx, "conn_total", s, st_sum_kernel, ceil_div(nslots, 256), 256, 0,
               sp->st_segcnt.as<u32>(), nslots, (unsigned long long*)total.as<u64>());
    sp->nnz_off = (i64)read_scalar(total.as<u64>(), s);
    sp->layout = 2;
    return true;
}

void staged_ensure_vals(hci_ctx_s* ctx, Space* sp, int precision, hipStream_t s) {
    const bool f32 = precision == HCI_FP32_MIXED;
    if (f32 ? sp->st_have32 : sp->st_have64) return;
    const i64 nnz = sp->st_nnz;
    ensure_alpha_b(ctx, sp, s);
    SpaceView S = space_view(*sp, ctx->n);
    const i64 grid = ceil_div(sp->N, ST_ROWS_PER_BLOCK);
    if (!sp->st_cols.ptr) {
        sp->st_cols = dev_alloc(ctx, sizeof(u16) * (nnz > 0 ? nnz : 1), s);
        DevMem fill = dev_alloc(ctx, sizeof(u32) * (sp->st_nslots > 0 ? sp->st_nslots : 1), s);
        DevMem bad = dev_alloc(ctx, sizeof(u64), s);
        HIP_CHECK(hipMemsetAsync(bad.ptr, 0, sizeof(u64), s));
        if (sp->st_abW) {
            HCI_LAUNCH(ctx, "csr_cols", s, st_cols_kernel<false>, grid, ST_ROW_BLOCK, 0, S, st_view(*sp),
                       sp->st_cols.as<u16>(), fill.as<u32>());
            HCI_LAUNCH(ctx, "csr_cols", s, st_ab_kernel<1>, sp->st_nchunk, ST_BLOCK, ab_lds(*sp), S,
                       st_view(*sp), sp->st_abW, sp->st_abG, (u32*)nullptr, fill.as<u32>(),
                       sp->st_cols.as<u16>());
        } else {
            HCI_LAUNCH(ctx, "csr_cols", s, st_cols_kernel<true>, grid, ST_ROW_BLOCK, 0, S, st_view(*sp),
                       sp->st_cols.as<u16>(), fill.as<u32>());
        }
        HCI_LAUNCH(ctx, "csr_cols", s, st_pad_kernel, grid, ST_ROW_BLOCK, 0, S, st_view(*sp),
                   (const u32*)fill.as<u32>(), sp->st_cols.as<u16>(), (unsigned long long*)bad.as<u64>());
        const u64 nbad = read_scalar(bad.as<u64>(), s);
        HCI_REQUIRE(nbad == 0, HCI_E_HIP,
                    "internal: " + std::to_string(nbad) + " row segments disagree with the count pass");
    }
    IntView I = int_view(ctx->ints);
    // element pass per row chunk; LDS: the window's beta strings, then the
    // alpha string, stage start and first row of each of the bucket's ranges
    // (at most 1 + N_alpha (n - N_alpha))
    const size_t vlds = vals_lds(ctx, sp->st_wlog);
    for (const void* k : {reinterpret_cast<const void*>(st_vals_kernel<1>),
                          reinterpret_cast<const void*>(st_vals_kernel<2>),
                          reinterpret_cast<const void*>(st_vals_kernel<3>)})
        HIP_CHECK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)vlds));
    if (f32 && !sp->st_have64 && nnz * (i64)(2 + 4 + 8) <= ctx->stored_budget) {
        sp->st_vals32 = dev_alloc(ctx, sizeof(float) * (nnz > 0 ? nnz : 1), s);
        sp->st_vals64 = dev_alloc(ctx, sizeof(double) * (nnz > 0 ? nnz : 1), s);
        HCI_LAUNCH(ctx, "csr_vals_f32", s, st_vals_kernel<3>, sp->st_nchunk, ST_BLOCK, vlds, S, I,
                   st_view(*sp), sp->st_vals32.as<float>(), sp->st_vals64.as<double>());
        sp->st_have32 = true;
        sp->st_have64 = true;
    } else if (f32) {
        sp->st_vals32 = dev_alloc(ctx, sizeof(float) * (nnz > 0 ? nnz : 1), s);
        HCI_LAUNCH(ctx, "csr_vals_f32", s, st_vals_kernel<1>, sp->st_nchunk, ST_BLOCK, vlds, S, I,
                   st_view(*sp), sp->st_vals32.as<float>(), (double*)nullptr);
        sp->st_have32 = true;
    } else {
        sp->st_vals64 = dev_alloc(ctx, sizeof(double) * (nnz > 0 ? nnz : 1), s);
        HCI_LAUNCH(ctx, "csr_vals_f64", s, st_vals_kernel<2>, sp->st_nchunk, ST_BLOCK, vlds, S, I,
                   st_view(*sp), (float*)nullptr, sp->st_vals64.as<double>());
        sp->st_have64 = true;
    }
}

void staged_apply(hci_ctx_s* ctx, Space* sp, const double* c, double* sigma, int precision,
                  hipStream_t s) {
    staged_ensure_vals(ctx, sp, precision, s);
    const i64 N = sp->N;
    if (precision == HCI_FP32_MIXED) {
        if (!sp->c32.ptr) sp->c32 = dev_alloc(ctx, sizeof(float) * N, s);
        if (!sp->cpb32.ptr) sp->cpb32 = dev_alloc(ctx, sizeof(float) * N, s);
        HCI_LAUNCH(ctx, "c_to_f32", s, st_prep_kernel<float>, ceil_div(N, 256), 256, 0, c,
                   sp->permb.as<u32>(), N, sp->c32.as<float>(), sp->cpb32.as<float>());
        launch_spmv<float, float>(ctx, sp, "sigma_stored_f32", "sigma_stored_f32_g",
                                  sp->st_vals32.as<float>(),
                                  sp->c32.as<float>(), sp->cpb32.as<float>(), c, sigma, s);
    } else {
        if (!sp->cpb64.ptr) sp->cpb64 = dev_alloc(ctx, sizeof(double) * N, s);
        HCI_LAUNCH(ctx, "c_perm_f64", s, st_prep_kernel<double>, ceil_div(N, 256), 256, 0, c,
                   sp->permb.as<u32>(), N, (double*)nullptr, sp->cpb64.as<double>());
        launch_spmv<double, double>(ctx, sp, "sigma_stored_f64", "sigma_stored_f64_g",
                                    sp->st_vals64.as<double>(), c,
                                    sp->cpb64.as<double>(), c, sigma, s);
    }
}

void layout_info(hci_ctx_s* ctx, Space* sp, int64_t* info, hipStream_t s) {
    for (int k = 0; k < 8; ++k) info[k] = 0;
    info[0] = sp->layout;
    info[1] = sp->nnz_off;
    if (sp->layout != 2) {
        info[2] = sp->nnz_pad;
        return;
    }
    info[2] = sp->st_nnz;
    info[3] = sp->st_wlog;
    info[6] = sp->st_nchunk;
    info[7] = sp->st_gnchunk;
    DevMem total = dev_alloc(ctx, sizeof(u64), s);
    HIP_CHECK(hipMemsetAsync(total.ptr, 0, sizeof(u64), s));
    HCI_LAUNCH(ctx, "st_gentries", s, st_gentries_kernel, ceil_div(sp->N, 256), 256, 0,
               space_view(*sp, ctx->n), st_view(*sp), (unsigned long long*)total.as<u64>());
    info[4] = (i64)read_scalar(total.as<u64>(), s);
    // entries of c staged by the product kernel: every workgroup of a bucket
    // copies the bucket's whole stage list
    const i64 nua = sp->nua;
    std::vector<u32> len(nua), cptr(nua + 1);
    HIP_CHECK(hipMemcpyAsync(len.data(), sp->st_len.ptr, sizeof(u32) * nua, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(cptr.data(), sp->st_cptr.ptr, sizeof(u32) * (nua + 1),
                             hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    i64 staged = 0;
    for (i64 a = 0; a < nua; ++a) staged += (i64)(cptr[a + 1] - cptr[a]) * len[a];
    info[5] = staged;
}
