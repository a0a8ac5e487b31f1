/*
 * CPU oracle for the Heat-bath CI variational step -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct reference arithmetic that the GPU library is
 * checked against.  It shares no code, header or table with the GPU library
 * and is loaded only by the test suite, the smoke check and the benchmark's
 * CPU-baseline leg.  Every loop follows a definition written out in the
 * comments; nothing is blocked, fused or reordered for speed (independent
 * rows may run on several OpenMP threads, which changes no arithmetic).
 *
 * Conventions (chosen where the paper is silent; see the oracle README):
 *   determinant = (alpha word, beta word), orbital p <-> bit p, n <= 64;
 *   Jordan-Wigner order: all alpha creators left of all beta creators, each
 *   spin in ascending orbital order;
 *   integrals: h[p][q] symmetric, g[p][q][r][s] = (pq|rs) chemist notation;
 *   H = sum_{pq,s} h_pq a+_ps a_qs + 1/2 sum_{pqrs,st} (pq|rs) a+_ps a+_rt a_st a_qs.
 *
 * Build: gcc -O2 -fPIC -shared -fopenmp -ffp-contract=off
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;

#define G(p, q, r, s) g[((((size_t)(p) * n + (q)) * n + (r)) * n) + (s)]
#define H1(p, q) h[(size_t)(p) * n + (q)]

static int popc(u64 x) { return __builtin_popcountll(x); }

static int lowest_bit(u64 x) { return __builtin_ctzll(x); }

/* (-1)^(number of occupied orbitals of `s` strictly between p and q). */
static double sign_between(u64 s, int p, int q) {
    int lo = p < q ? p : q, hi = p < q ? q : p;
    int cnt = 0;
    for (int k = lo + 1; k < hi; ++k)
        if ((s >> k) & 1ULL) cnt++;
    return (cnt & 1) ? -1.0 : 1.0;
}

int orc_abi_version(void) { return 3; }

/* <D|H|D>: sum of occupied one-body energies plus, over every unordered pair
 * of occupied spin orbitals, Coulomb minus (same-spin) exchange. */
double orc_diag(int n, const double* h, const double* g, u64 a, u64 b) {
    double e = 0.0;
    for (int p = 0; p < n; ++p) {
        if ((a >> p) & 1ULL) e += H1(p, p);
        if ((b >> p) & 1ULL) e += H1(p, p);
    }
    double two = 0.0;
    for (int p = 0; p < n; ++p) {
        for (int q = 0; q < n; ++q) {
            int pa = (a >> p) & 1, pb = (b >> p) & 1, qa = (a >> q) & 1, qb = (b >> q) & 1;
            if (pa && qa) two += G(p, p, q, q) - G(p, q, q, p);
            if (pb && qb) two += G(p, p, q, q) - G(p, q, q, p);
            if (pa && qb) two += G(p, p, q, q);
            if (pb && qa) two += G(p, p, q, q);
        }
    }
    return e + 0.5 * two;
}

/* Matrix element of a single excitation p -> q in the string `same` (spin s),
 * `other` the opposite-spin string of the ket.  Sum order: one-body term, then
 * occupied same-spin r ascending (Coulomb minus exchange), then occupied
 * opposite-spin r ascending (Coulomb). */
static double single_value(int n, const double* h, const double* g, u64 same, u64 other,
                           int p, int q) {
    double v = H1(q, p);
    for (int r = 0; r < n; ++r)
        if ((same >> r) & 1ULL) v += (G(q, p, r, r) - G(q, r, r, p));
    for (int r = 0; r < n; ++r)
        if ((other >> r) & 1ULL) v += G(q, p, r, r);
    return v;
}

/* <D_j|H|D_i> by the Slater-Condon rules (excitation degree <= 2). */
double orc_hij(int n, const double* h, const double* g, u64 ai, u64 bi, u64 aj, u64 bj) {
    int da = popc(ai ^ aj) / 2, db = popc(bi ^ bj) / 2;
    if (da + db == 0) return orc_diag(n, h, g, ai, bi);
    if (da + db > 2) return 0.0;
    if (da == 1 && db == 0) {
        int p = lowest_bit(ai & ~aj), q = lowest_bit(aj & ~ai);
        return sign_between(ai, p, q) * single_value(n, h, g, ai, bi, p, q);
    }
    if (da == 0 && db == 1) {
        int p = lowest_bit(bi & ~bj), q = lowest_bit(bj & ~bi);
        return sign_between(bi, p, q) * single_value(n, h, g, bi, ai, p, q);
    }
    if (da == 1 && db == 1) {
        int p = lowest_bit(ai & ~aj), r = lowest_bit(aj & ~ai);
        int q = lowest_bit(bi & ~bj), s = lowest_bit(bj & ~bi);
        return sign_between(ai, p, r) * sign_between(bi, q, s) * G(r, p, s, q);
    }
    /* same-spin double: holes p < q, particles r < s; phase of p->r then q->s */
    u64 si = da == 2 ? ai : bi, sj = da == 2 ? aj : bj;
    u64 holes = si & ~sj, parts = sj & ~si;
    int p = lowest_bit(holes), q = lowest_bit(holes & (holes - 1));
    int r = lowest_bit(parts), s = lowest_bit(parts & (parts - 1));
    double sg = sign_between(si, p, r);
    u64 mid = si ^ (1ULL << p) ^ (1ULL << r);
    sg *= sign_between(mid, q, s);
    return sg * (G(r, p, s, q) - G(r, q, s, p));
}

/* Every determinant reachable from (a,b) by one single or double excitation,
 * each exactly once: alpha singles, beta singles, alpha-alpha doubles,
 * beta-beta doubles, alpha-beta doubles.  Writes up to `cap` pairs into out
 * (may be NULL) and returns the total count. */
long orc_excitations(int n, u64 a, u64 b, u64* out, long cap) {
    long k = 0;
#define EMIT(x, y)                          \
    do {                                    \
        if (out && k < cap) {               \
            out[2 * k] = (x);               \
            out[2 * k + 1] = (y);           \
        }                                   \
        k++;                                \
    } while (0)
    for (int spin = 0; spin < 2; ++spin) {
        u64 s = spin ? b : a;
        for (int p = 0; p < n; ++p) {
            if (!((s >> p) & 1ULL)) continue;
            for (int r = 0; r < n; ++r) {
                if ((s >> r) & 1ULL) continue;
                u64 t = s ^ (1ULL << p) ^ (1ULL << r);
                if (spin) EMIT(a, t); else EMIT(t, b);
            }
        }
    }
    for (int spin = 0; spin < 2; ++spin) {
        u64 s = spin ? b : a;
        for (int p = 0; p < n; ++p) {
            if (!((s >> p) & 1ULL)) continue;
            for (int q = p + 1; q < n; ++q) {
                if (!((s >> q) & 1ULL)) continue;
                for (int r = 0; r < n; ++r) {
                    if ((s >> r) & 1ULL) continue;
                    for (int t2 = r + 1; t2 < n; ++t2) {
                        if ((s >> t2) & 1ULL) continue;
                        u64 t = s ^ (1ULL << p) ^ (1ULL << q) ^ (1ULL << r) ^ (1ULL << t2);
                        if (spin) EMIT(a, t); else EMIT(t, b);
                    }
                }
            }
        }
    }
    for (int p = 0; p < n; ++p) {
        if (!((a >> p) & 1ULL)) continue;
        for (int r = 0; r < n; ++r) {
            if ((a >> r) & 1ULL) continue;
            u64 ta = a ^ (1ULL << p) ^ (1ULL << r);
            for (int q = 0; q < n; ++q) {
                if (!((b >> q) & 1ULL)) continue;
                for (int s = 0; s < n; ++s) {
                    if ((b >> s) & 1ULL) continue;
                    EMIT(ta, b ^ (1ULL << q) ^ (1ULL << s));
                }
            }
        }
    }
#undef EMIT
    return k;
}

/* Index of (a,b) in the (alpha, beta)-sorted list V, or -1. */
long orc_find(const u64* V, long nv, u64 a, u64 b) {
    long lo = 0, hi = nv;
    while (lo < hi) {
        long mid = lo + (hi - lo) / 2;
        u64 ma = V[2 * mid], mb = V[2 * mid + 1];
        if (ma < a || (ma == a && mb < b)) lo = mid + 1;
        else hi = mid;
    }
    if (lo < nv && V[2 * lo] == a && V[2 * lo + 1] == b) return lo;
    return -1;
}

static long max_excitations(int n, u64 a, u64 b) { return orc_excitations(n, a, b, NULL, 0); }

/* Heat-bath selection by its definition: for every i in V and every single or
 * double excitation a of D_i that is not in V, keep a when
 * fl(|H_ai| * |c_i|) > eps (strict).  Duplicates are written as found (the
 * caller takes the unique set).  Returns the number of hits; writes at most
 * `cap` of them. */
long orc_select(int n, const double* h, const double* g, const u64* V, long nv,
                const double* c, double eps, u64* out, long cap) {
    long total = 0;
    u64* buf = NULL;
    long bufcap = 0;
    for (long i = 0; i < nv; ++i) {
        u64 a = V[2 * i], b = V[2 * i + 1];
        long m = max_excitations(n, a, b);
        if (m > bufcap) {
            free(buf);
            bufcap = m;
            buf = (u64*)malloc(sizeof(u64) * 2 * bufcap);
        }
        orc_excitations(n, a, b, buf, m);
        double ci = fabs(c[i]);
        for (long k = 0; k < m; ++k) {
            u64 xa = buf[2 * k], xb = buf[2 * k + 1];
            if (orc_find(V, nv, xa, xb) >= 0) continue;
            double hai = orc_hij(n, h, g, a, b, xa, xb);
            double prod = fabs(hai) * ci;
            if (prod > eps) {
                if (out && total < cap) {
                    out[2 * total] = xa;
                    out[2 * total + 1] = xb;
                }
                total++;
            }
        }
    }
    free(buf);
    return total;
}

/* sigma_i = sum_j H_ij c_j for the listed rows i (all of V when rows == NULL),
 * with j running over i itself and every excitation of D_i found in V.
 * pairs (may be NULL) receives the number of j of each row. */
void orc_sigma_rows(int n, const double* h, const double* g, const u64* V, long nv,
                    const double* c, const long* rows, long nrows, double* out, long* pairs) {
    long cnt = rows ? nrows : nv;
#pragma omp parallel
    {
        u64* buf = NULL;
        long bufcap = 0;
#pragma omp for schedule(dynamic, 16)
        for (long k = 0; k < cnt; ++k) {
            long i = rows ? rows[k] : k;
            u64 a = V[2 * i], b = V[2 * i + 1];
            long m = max_excitations(n, a, b);
            if (m > bufcap) {
                free(buf);
                bufcap = m;
                buf = (u64*)malloc(sizeof(u64) * 2 * bufcap);
            }
            orc_excitations(n, a, b, buf, m);
            double s = orc_diag(n, h, g, a, b) * c[i];
            long found = 1;
            for (long e = 0; e < m; ++e) {
                long j = orc_find(V, nv, buf[2 * e], buf[2 * e + 1]);
                if (j < 0) continue;
                s += orc_hij(n, h, g, V[2 * j], V[2 * j + 1], a, b) * c[j];
                found++;
            }
            out[k] = s;
            if (pairs) pairs[k] = found;
        }
        free(buf);
    }
}

/* Number of connected (i,j) pairs per row (diagonal included). */
void orc_row_counts(int n, const u64* V, long nv, long* counts) {
#pragma omp parallel
    {
        u64* buf = NULL;
        long bufcap = 0;
#pragma omp for schedule(dynamic, 16)
        for (long i = 0; i < nv; ++i) {
            u64 a = V[2 * i], b = V[2 * i + 1];
            long m = max_excitations(n, a, b);
            if (m > bufcap) {
                free(buf);
                bufcap = m;
                buf = (u64*)malloc(sizeof(u64) * 2 * bufcap);
            }
            orc_excitations(n, a, b, buf, m);
            long k = 1;
            for (long e = 0; e < m; ++e)
                if (orc_find(V, nv, buf[2 * e], buf[2 * e + 1]) >= 0) k++;
            counts[i] = k;
        }
        free(buf);
    }
}

/* Full Hamiltonian on V as CSR (rows in V order, columns ascending within a
 * row, diagonal included).  rowptr has nv+1 entries from orc_row_counts. */
void orc_csr_fill(int n, const double* h, const double* g, const u64* V, long nv,
                  const long* rowptr, long* cols, double* vals) {
#pragma omp parallel
    {
        u64* buf = NULL;
        long bufcap = 0;
#pragma omp for schedule(dynamic, 16)
        for (long i = 0; i < nv; ++i) {
            u64 a = V[2 * i], b = V[2 * i + 1];
            long m = max_excitations(n, a, b);
            if (m > bufcap) {
                free(buf);
                bufcap = m;
                buf = (u64*)malloc(sizeof(u64) * 2 * bufcap);
            }
            orc_excitations(n, a, b, buf, m);
            long k = rowptr[i];
            cols[k] = i;
            vals[k] = orc_diag(n, h, g, a, b);
            k++;
            for (long e = 0; e < m; ++e) {
                long j = orc_find(V, nv, buf[2 * e], buf[2 * e + 1]);
                if (j < 0) continue;
                cols[k] = j;
                vals[k] = orc_hij(n, h, g, a, b, V[2 * j], V[2 * j + 1]);
                k++;
            }
            /* insertion sort of the row by column */
            for (long x = rowptr[i] + 1; x < rowptr[i + 1]; ++x) {
                long cc = cols[x];
                double vv = vals[x];
                long y = x - 1;
                while (y >= rowptr[i] && cols[y] > cc) {
                    cols[y + 1] = cols[y];
                    vals[y + 1] = vals[y];
                    y--;
                }
                cols[y + 1] = cc;
                vals[y + 1] = vv;
            }
        }
        free(buf);
    }
}

/* ---- second quantisation on spin-orbital words (Jordan-Wigner order) ---- */
/* A determinant as one 128-bit occupation: spin-orbital k < n is alpha k,
 * k >= n is beta (k - n).  Operators return 0 when they annihilate the state
 * and otherwise the sign picked up passing the occupied modes to the left. */
typedef struct { u64 lo, hi; } so_t; /* alpha word, beta word */

static int so_test(const so_t* d, int n, int k) {
    return k < n ? (int)((d->lo >> k) & 1ULL) : (int)((d->hi >> (k - n)) & 1ULL);
}
static void so_flip(so_t* d, int n, int k) {
    if (k < n) d->lo ^= (1ULL << k); else d->hi ^= (1ULL << (k - n));
}
static int so_count_below(const so_t* d, int n, int k) {
    int c = 0;
    for (int m = 0; m < k; ++m) c += so_test(d, n, m);
    return c;
}
static int so_annihilate(so_t* d, int n, int k) {
    if (!so_test(d, n, k)) return 0;
    int s = (so_count_below(d, n, k) & 1) ? -1 : 1;
    so_flip(d, n, k);
    return s;
}
static int so_create(so_t* d, int n, int k) {
    if (so_test(d, n, k)) return 0;
    int s = (so_count_below(d, n, k) & 1) ? -1 : 1;
    so_flip(d, n, k);
    return s;
}

/* Spin-traced density matrices by applying the operators to every ket
 * determinant:  rdm1[p][q] = sum_s <bra| a+_ps a_qs |ket>,
 * rdm2[p][q][r][s] = sum_{s,t} <bra| a+_ps a+_rt a_st a_qs |ket>.
 * Outputs are overwritten. */
void orc_rdm12(int n, const u64* V, long nv, const double* bra, const double* ket,
               double* rdm1, double* rdm2) {
    size_t n2 = (size_t)n * n, n4 = n2 * n2;
    memset(rdm1, 0, sizeof(double) * n2);
    memset(rdm2, 0, sizeof(double) * n4);
    int ns = 2 * n;
    for (long j = 0; j < nv; ++j) {
        if (ket[j] == 0.0) continue;
        so_t d0 = {V[2 * j], V[2 * j + 1]};
        for (int qs = 0; qs < ns; ++qs) {
            for (int ps = 0; ps < ns; ++ps) {
                if ((qs < n) != (ps < n)) continue; /* spin conserved */
                so_t d = d0;
                int s1 = so_annihilate(&d, n, qs);
                if (!s1) continue;
                int s2 = so_create(&d, n, ps);
                if (!s2) continue;
                long i = orc_find(V, nv, d.lo, d.hi);
                if (i < 0) continue;
                rdm1[(size_t)(ps % n) * n + (qs % n)] += bra[i] * ket[j] * s1 * s2;
            }
        }
        for (int qs = 0; qs < ns; ++qs) {
            so_t d1 = d0;
            int s1 = so_annihilate(&d1, n, qs);
            if (!s1) continue;
            for (int ss = 0; ss < ns; ++ss) {
                so_t d2 = d1;
                int s2 = so_annihilate(&d2, n, ss);
                if (!s2) continue;
                for (int rs = 0; rs < ns; ++rs) {
                    if ((ss < n) != (rs < n)) continue;
                    so_t d3 = d2;
                    int s3 = so_create(&d3, n, rs);
                    if (!s3) continue;
                    for (int ps = 0; ps < ns; ++ps) {
                        if ((qs < n) != (ps < n)) continue;
                        so_t d = d3;
                        int s4 = so_create(&d, n, ps);
                        if (!s4) continue;
                        long i = orc_find(V, nv, d.lo, d.hi);
                        if (i < 0) continue;
                        int p = ps % n, q = qs % n, r = rs % n, s = ss % n;
                        rdm2[(((size_t)p * n + q) * n + r) * n + s] +=
                            bra[i] * ket[j] * (double)(s1 * s2 * s3 * s4);
                    }
                }
            }
        }
    }
}

/* One element of each density matrix by the same operator application,
 * for sampled checks on spaces too large for the full loops above. */
double orc_rdm2_element(int n, const u64* V, long nv, const double* bra, const double* ket,
                        int p, int q, int r, int s) {
    double acc = 0.0;
    for (int sg = 0; sg < 2; ++sg) {
        for (int tu = 0; tu < 2; ++tu) {
            int ps = p + sg * n, qs = q + sg * n, rs = r + tu * n, ss = s + tu * n;
            double part = 0.0;
#pragma omp parallel for reduction(+ : part) schedule(static)
            for (long j = 0; j < nv; ++j) {
                so_t d = {V[2 * j], V[2 * j + 1]};
                int s1 = so_annihilate(&d, n, qs);
                if (!s1) continue;
                int s2 = so_annihilate(&d, n, ss);
                if (!s2) continue;
                int s3 = so_create(&d, n, rs);
                if (!s3) continue;
                int s4 = so_create(&d, n, ps);
                if (!s4) continue;
                long i = orc_find(V, nv, d.lo, d.hi);
                if (i < 0) continue;
                part += bra[i] * ket[j] * (double)(s1 * s2 * s3 * s4);
            }
            acc += part;
        }
    }
    return acc;
}

double orc_rdm1_element(int n, const u64* V, long nv, const double* bra, const double* ket,
                        int p, int q) {
    double acc = 0.0;
    for (int sg = 0; sg < 2; ++sg) {
        int ps = p + sg * n, qs = q + sg * n;
        for (long j = 0; j < nv; ++j) {
            so_t d = {V[2 * j], V[2 * j + 1]};
            int s1 = so_annihilate(&d, n, qs);
            if (!s1) continue;
            int s2 = so_create(&d, n, ps);
            if (!s2) continue;
            long i = orc_find(V, nv, d.lo, d.hi);
            if (i < 0) continue;
            acc += bra[i] * ket[j] * (double)(s1 * s2);
        }
    }
    return acc;
}

/* H|D> by applying every operator term of H to the determinant (no
 * Slater-Condon rules).  Fills parallel arrays of result determinants and
 * amplitudes (duplicates allowed, the caller sums them); returns the count. */
long orc_apply_h(int n, const double* h, const double* g, u64 a, u64 b,
                 u64* out_dets, double* out_amp, long cap) {
    long k = 0;
    int ns = 2 * n;
    so_t d0 = {a, b};
    for (int qs = 0; qs < ns; ++qs) {
        for (int ps = 0; ps < ns; ++ps) {
            if ((qs < n) != (ps < n)) continue;
            so_t d = d0;
            int s1 = so_annihilate(&d, n, qs);
            if (!s1) continue;
            int s2 = so_create(&d, n, ps);
            if (!s2) continue;
            if (k < cap) {
                out_dets[2 * k] = d.lo;
                out_dets[2 * k + 1] = d.hi;
                out_amp[k] = H1(ps % n, qs % n) * (double)(s1 * s2);
            }
            k++;
        }
    }
    for (int qs = 0; qs < ns; ++qs) {
        for (int ss = 0; ss < ns; ++ss) {
            for (int rs = 0; rs < ns; ++rs) {
                if ((ss < n) != (rs < n)) continue;
                for (int ps = 0; ps < ns; ++ps) {
                    if ((qs < n) != (ps < n)) continue;
                    so_t d = d0;
                    int s1 = so_annihilate(&d, n, qs);
                    if (!s1) continue;
                    int s2 = so_annihilate(&d, n, ss);
                    if (!s2) continue;
                    int s3 = so_create(&d, n, rs);
                    if (!s3) continue;
                    int s4 = so_create(&d, n, ps);
                    if (!s4) continue;
                    if (k < cap) {
                        out_dets[2 * k] = d.lo;
                        out_dets[2 * k + 1] = d.hi;
                        out_amp[k] = 0.5 * G(ps % n, qs % n, rs % n, ss % n) *
                                     (double)(s1 * s2 * s3 * s4);
                    }
                    k++;
                }
            }
        }
    }
    return k;
}

/* ---- eps2-screened second-order pieces (eq. pt_hci) ---- */
/* Every pair (i, a) with D_a outside V reached from D_i by one single or
 * double excitation and fl(|H_ai| * |c_i|) > eps2 (the screening mask),
 * listed in i order then excitation order.  Writes up to cap entries of
 * (a alpha, a beta), i and H_ai; returns the total. */
long orc_pt2_pairs(int n, const double* h, const double* g, const u64* V, long nv,
                   const double* c, double eps2, u64* out_a, long* out_i, double* out_h, long cap) {
    long total = 0;
    u64* buf = NULL;
    long bufcap = 0;
    for (long i = 0; i < nv; ++i) {
        /* |H_ai| * 0 > eps2 never holds (eps2 >= 0): such a row has no pairs */
        if (c[i] == 0.0 && eps2 >= 0.0) continue;
        u64 a = V[2 * i], b = V[2 * i + 1];
        long m = max_excitations(n, a, b);
        if (m > bufcap) {
            free(buf);
            bufcap = m;
            buf = (u64*)malloc(sizeof(u64) * 2 * bufcap);
        }
        orc_excitations(n, a, b, buf, m);
        double ci = fabs(c[i]);
        for (long k = 0; k < m; ++k) {
            u64 xa = buf[2 * k], xb = buf[2 * k + 1];
            if (orc_find(V, nv, xa, xb) >= 0) continue;
            double hai = orc_hij(n, h, g, a, b, xa, xb);
            double prod = fabs(hai) * ci;
            if (prod > eps2) {
                if (total < cap) {
                    out_a[2 * total] = xa;
                    out_a[2 * total + 1] = xb;
                    out_i[total] = i;
                    out_h[total] = hai;
                }
                total++;
            }
        }
    }
    free(buf);
    return total;
}

/* rdm1/rdm2 += w * <D_x| ops |D_y> for one pair of determinants, by applying
 * every operator of the spin-traced definitions to D_y (x may equal y). */
void orc_pair_rdm_add(int n, u64 xa, u64 xb, u64 ya, u64 yb, double w, double* rdm1, double* rdm2) {
    int ns = 2 * n;
    so_t d0 = {ya, yb};
    for (int qs = 0; qs < ns; ++qs)
        for (int ps = 0; ps < ns; ++ps) {
            if ((qs < n) != (ps < n)) continue;
            so_t d = d0;
            int s1 = so_annihilate(&d, n, qs);
            if (!s1) continue;
            int s2 = so_create(&d, n, ps);
            if (!s2) continue;
            if (d.lo != xa || d.hi != xb) continue;
            rdm1[(size_t)(ps % n) * n + (qs % n)] += w * s1 * s2;
        }
    if (!rdm2) return;
    /* a+_p a+_r a_s a_q |y>: after the two annihilations the remaining
     * orbitals must all be occupied in x, and each creation must fill an
     * orbital occupied in x, or the result cannot be x (those branches
     * contribute exactly zero and are skipped) */
    so_t xt = {xa, xb};
    for (int qs = 0; qs < ns; ++qs) {
        so_t d1 = d0;
        int s1 = so_annihilate(&d1, n, qs);
        if (!s1) continue;
        for (int ss = 0; ss < ns; ++ss) {
            so_t d2 = d1;
            int s2 = so_annihilate(&d2, n, ss);
            if (!s2) continue;
            if ((d2.lo & ~xa) || (d2.hi & ~xb)) continue;
            for (int rs = 0; rs < ns; ++rs) {
                if ((ss < n) != (rs < n)) continue;
                if (!so_test(&xt, n, rs)) continue;
                so_t d3 = d2;
                int s3 = so_create(&d3, n, rs);
                if (!s3) continue;
                for (int ps = 0; ps < ns; ++ps) {
                    if ((qs < n) != (ps < n)) continue;
                    if (!so_test(&xt, n, ps)) continue;
                    so_t d = d3;
                    int s4 = so_create(&d, n, ps);
                    if (!s4) continue;
                    if (d.lo != xa || d.hi != xb) continue;
                    int p = ps % n, q = qs % n, r = rs % n, s = ss % n;
                    rdm2[(((size_t)p * n + q) * n + r) * n + s] += w * (double)(s1 * s2 * s3 * s4);
                }
            }
        }
    }
}
