/*
 * hci.h -- C ABI of the MI355X (gfx950) Heat-bath CI variational step.
 *
 * Method: Smith, Mussard, Holmes, Sharma, "Cheap and near exact CASSCF with
 * large active spaces" (arXiv:1708.07544).  The library takes active-space
 * integrals in and returns the variational energy, the wavefunction, the
 * one- and two-particle density matrices and the energy's derivatives with
 * respect to the integrals (the quantities an orbital optimiser consumes:
 * Sec. "HCI self-consistent field", eq. vdedk2 and eq. lambda).
 *
 * Conventions used by every entry point:
 *   - A determinant is two 64-bit occupation words {alpha, beta}; orbital p
 *     is bit p (norb <= 64).  Fermion signs follow Jordan-Wigner order with
 *     all alpha creators to the left of all beta creators, ascending orbital
 *     index within a spin.
 *   - Determinant lists are uint64_t[n][2] = {alpha, beta}, strictly
 *     ascending in (alpha, beta) lexicographic order, every row with
 *     popcount(alpha) == nalpha and popcount(beta) == nbeta.
 *   - Integrals: h[p][q] (symmetric) and g[p][q][r][s] = (pq|rs) in chemist
 *     notation, 8-fold symmetric, both float64 row-major.
 *   - H = ecore + sum_{pq,s} h_pq a+_ps a_qs
 *         + 1/2 sum_{pqrs,st} (pq|rs) a+_ps a+_rt a_st a_qs.
 *   - Density matrices are spin-traced:
 *       rdm1[p][q]       = sum_s  <bra| a+_ps a_qs |ket>
 *       rdm2[p][q][r][s] = sum_st <bra| a+_ps a+_rt a_st a_qs |ket>
 *     so that E = ecore + sum h_pq rdm1_pq + 1/2 sum (pq|rs) rdm2_pqrs
 *     (the paper's Gamma_ijkl = <a+_i a+_j a_k a_l> with indices reordered).
 *
 * Memory and streams:
 *   - Every pointer argument marked "device" is a caller-owned device buffer
 *     on the context's GPU; "host" pointers are ordinary host memory.  The
 *     library never frees caller memory.
 *   - Scratch and cached structures are allocated through the context's
 *     allocator (or hipMalloc when none is given) and released by
 *     hci_ctx_destroy.  The context caches, for the most recently used
 *     determinant list, its bucket/adjacency structure and the stored
 *     Hamiltonian; the cache is keyed by the list's length and a content
 *     hash computed on the GPU (not its address), so editing a list in place
 *     is safe and an equal list in another buffer reuses the structure.
 *   - All work is enqueued on `stream` (a hipStream_t; NULL = default
 *     stream).  Calls that return host scalars synchronise that stream.
 *
 * Sizes: a list holds at most 2^32 - 2 determinants, and the
 * single-excitation links between its unique alpha (beta) strings plus their
 * number stay below 2^32 (HCI_E_UNSUPPORTED otherwise, before any work).
 * One launch covers at most 2^32 work-items: the row kernels of the
 * selection walk, the connection count and the recomputed product stride
 * over the rows of a clamped grid (so any list size works there); the
 * stored-Hamiltonian builds take one wavefront per row in one launch, so
 * HCI_SIGMA_AUTO recomputes lists of more than about 67 million
 * determinants, and any launch that would exceed the limit fails with
 * HCI_E_UNSUPPORTED instead of running in part.  HCI_ROW_GRID_CAP=<k> in the
 * environment clamps the striding kernels to k workgroups (for tests).
 *
 * Errors: every entry point returns an hci_status.  No C++ exception crosses
 * the ABI.  hci_last_error() returns a thread-local message for the last
 * failing call.  A context must not be used by two threads at once.
 */
#ifndef HCI_MI355X_H
#define HCI_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HCI_OK = 0,
    HCI_E_ARG = -1,         /* invalid argument or malformed determinant list */
    HCI_E_NOMEM = -2,       /* an allocation failed */
    HCI_E_CAPACITY = -3,    /* output capacity too small; required size reported */
    HCI_E_NOCONV = -4,      /* iterative solver hit max_iter; best result written */
    HCI_E_HIP = -5,         /* a HIP runtime call failed */
    HCI_E_UNSUPPORTED = -6  /* option not available */
} hci_status;

typedef enum { HCI_FP64 = 0, HCI_FP32_MIXED = 1 } hci_precision;

/* Largest number of states of one determinant space (hci_select_roots,
 * hci_davidson_roots). */
#define HCI_MAX_ROOTS 31

typedef enum {
    HCI_SIGMA_AUTO = 0,      /* stored when the Hamiltonian fits the memory budget */
    HCI_SIGMA_STORED = 1,    /* build the sparse Hamiltonian once, then stream it */
    HCI_SIGMA_RECOMPUTE = 2  /* regenerate connections and elements every product */
} hci_sigma_mode;

typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* user); /* NULL on failure */
    void (*free)(void* ptr, void* user);
    void* user;
} hci_allocator;

typedef struct hci_ctx_s* hci_ctx;

/* ------------------------------------------------------------------ context
 * Stage the integrals on the GPU and build the heat-bath tables: for every
 * occupied pair the double-excitation magnitudes |H| sorted in descending
 * order, computed once per integral set (Sec. "Variational Stage": the
 * magnitudes depend on the orbitals only and are sorted before the run;
 * Fig. 1b).
 *   norb in [1,64]; 0 <= nalpha, nbeta <= norb.
 *   h: device float64 [norb][norb]; g: device float64 [norb]^4; both are
 *   copied, the caller may free them after the call returns.
 *   alloc: optional; copied by value.  stream: hipStream_t for the set-up.
 *   out: receives the new context.  Errors: HCI_E_ARG, HCI_E_NOMEM, HCI_E_HIP. */
int hci_ctx_create(int norb, int nalpha, int nbeta, const double* h, const double* g,
                   double ecore, const hci_allocator* alloc, void* stream, hci_ctx* out);

/* Replace the integrals (same norb) and rebuild the tables; drops the cached
 * Hamiltonian.  Same argument rules as hci_ctx_create. */
int hci_ctx_update_integrals(hci_ctx ctx, const double* h, const double* g, double ecore,
                             void* stream);

/* Release everything the context owns.  NULL is accepted. */
int hci_ctx_destroy(hci_ctx ctx);

/* Release the cached structure of the last determinant list (buckets,
 * adjacency, stored Hamiltonian, a selection result kept for a capacity
 * retry).  The next call on any list rebuilds it.  Two small pinned host
 * buffers the context allocates on first use (the Davidson iteration's
 * scalars, the density-matrix planner's staging) stay until
 * hci_ctx_destroy. */
int hci_ctx_release_cache(hci_ctx ctx);

/* Memory budget (bytes) for the stored Hamiltonian in HCI_SIGMA_AUTO mode
 * (default: 64 GiB). */
int hci_ctx_set_stored_budget(hci_ctx ctx, int64_t bytes);

/* Layout of the stored Hamiltonian (Sec. "Variational Stage": the matrix of
 * the Davidson products).  log2_window > 0 selects the alpha-bucket-staged
 * layout: for each alpha string, its bucket and the buckets one alpha single
 * away are read into on-chip memory 2^log2_window entries of c at a time and
 * columns are stored as 16-bit offsets (6 bytes per float32 entry).  0
 * selects the plain CSR layout (32-bit columns).  Valid values: 0 or 6..16
 * (default 14); spaces outside the staged layout's limits use plain CSR.
 * Changing the layout releases the cached structure.  HCI_E_ARG otherwise.
 * The alpha single x beta single connections of the staged layout (and of
 * the density matrices) are found through on-chip bitmaps of the beta
 * strings of each neighbour bucket when the space has at most 65535 unique
 * beta strings, else by searching the bucket; the environment variable
 * HCI_AB_SEARCH=1, read when a layout is built, forces the search (both give
 * the same entries in the same order). */
int hci_ctx_set_stage_window(hci_ctx ctx, int log2_window);

/* Per-kernel timing with HIP events on the launch stream (off by default).
 * When enabled, every library kernel launch is bracketed by events and its
 * duration accumulated under the kernel's name. */
int hci_ctx_set_timing(hci_ctx ctx, int enable);

/* Accumulated launches and milliseconds for a kernel name since the last
 * reset (synchronises the context's recorded events).  Unknown names give
 * count 0.  reset != 0 clears all counters after reading. */
int hci_ctx_kernel_time(hci_ctx ctx, const char* name, int64_t* launches, double* total_ms,
                        int reset);

/* Thread-local description of the last error ("" if none). */
const char* hci_last_error(void);

/* ---------------------------------------------------------------- selection
 * One HCI selection step (Sec. "Variational Stage", eq. criteria with the
 * HCI importance function): C(eps1) is the set of determinants D_a not in V
 * for which |H_ai c_i| > eps1 for at least one D_i in V; the routine writes
 * V + C(eps1), sorted and unique, to out_dets.  Doubles are found by walking
 * the pre-sorted heat-bath lists of each occupied pair of D_i only while the
 * magnitude can still pass (Fig. 1b); singles are evaluated exactly.  The
 * test is fl(|H_ai| * |c_i|) > eps1 in float64 (strict), identical on every
 * path.
 *   dets: device [n_var][2] sorted unique list V; c: device float64 [n_var].
 *   out_dets: device [cap][2]; may not alias dets.  n_out (host) receives the
 *   size of V + C; on HCI_E_CAPACITY it holds the required capacity and
 *   out_dets is unspecified.  Such a refused call keeps its result in the
 *   context (up to 2^28 determinants, 16 B each, when the memory is there):
 *   the next selection call with the same dets and c by content, the same
 *   eps1 and room for it copies the kept list instead of walking again.  Any
 *   other selection call, a change of cached space, hci_ctx_release_cache and
 *   hci_ctx_update_integrals drop it.  Synchronises the stream. */
int hci_select(hci_ctx ctx, const uint64_t* dets, const double* c, int64_t n_var,
               double eps1, uint64_t* out_dets, int64_t cap, int64_t* n_out, void* stream);

/* Selection for several states of one space at once.  The paper selects
 * for one state per calculation (its excited states are the lowest states of
 * other spin projections, N_alpha != N_beta, which every entry point here
 * accepts); for several states of one space the set taken is the union of
 * the single-state sets: D_a enters when fl(|H_ai| * |c_i|) > eps1 for some
 * D_i in V and some state.  One walk with the weights max over the states of
 * |c_i| gives exactly that union (the float64 product is non-decreasing in
 * its second factor).
 *   c: device float64 [nroots][n_var] (state r in row r), 1 <= nroots <=
 *   HCI_MAX_ROOTS.  Every other argument, the output and the errors as in
 *   hci_select. */
int hci_select_roots(hci_ctx ctx, const uint64_t* dets, const double* c, int nroots,
                     int64_t n_var, double eps1, uint64_t* out_dets, int64_t cap,
                     int64_t* n_out, void* stream);

/* Carry a vector from V to a superset V' (both sorted unique lists), as the
 * warm start of the next Davidson solve after V' = V + C (Fig. 1a):
 * c_new[k'] = c[k] where V'[k'] == V[k], and 0 on the determinants of V'
 * that are not in V.
 *   dets, c: device [n_var][2], [n_var]; dets_new, c_new: device
 *   [n_new][2], [n_new].  HCI_E_ARG if a member of V is missing from V'. */
int hci_embed(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c,
              const uint64_t* dets_new, int64_t n_new, double* c_new, void* stream);

/* --------------------------------------------------------------------- sigma
 * sigma = H c on V (the product inside Davidson, Sec. "Variational Stage";
 * all single and double connections between members of V, Sec.
 * "Computational Details").  precision HCI_FP64 evaluates and accumulates in
 * float64; HCI_FP32_MIXED multiplies float32 off-diagonal elements by a
 * float32 copy of c and accumulates each row in float64, with the float64
 * diagonal term added in float64.
 *   dets: device [n_var][2]; c, sigma: device float64 [n_var], no aliasing.
 *   mode: hci_sigma_mode.  Asynchronous unless a cache rebuild is needed. */
int hci_sigma(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c,
              double* sigma, int precision, int mode, void* stream);

/* Number of ordered pairs (i,j) in V x V with excitation degree <= 2,
 * diagonal included (host int64 out).  Synchronises the stream. */
int hci_connections(hci_ctx ctx, const uint64_t* dets, int64_t n_var, int64_t* nnz_out,
                    void* stream);

/* Statistics of the stored Hamiltonian of V (Sec. "Variational Stage": the
 * matrix of the Davidson products), for memory planning and traffic
 * accounting; runs the count pass if needed and synchronises the stream.
 * info (host int64 [8]):
 *   [0] layout: 1 plain CSR, 2 alpha-bucket-staged
 *   [1] off-diagonal connections
 *   [2] stored entries (staged: segments padded to multiples of 8)
 *   [3] log2 of the stage window (0 for plain CSR)
 *   [4] stored entries of the beta-group segments (alpha doubles, same beta)
 *   [5] entries of c copied into on-chip memory per staged product
 *   [6] workgroups of the staged product, [7] of the beta-group product
 * HCI_E_ARG on null arguments or an invalid list. */
int hci_layout_info(hci_ctx ctx, const uint64_t* dets, int64_t n_var, int64_t* info,
                    void* stream);

/* Diagonal H_ii (float64, device [n_var]), ecore included. */
int hci_diagonal(hci_ctx ctx, const uint64_t* dets, int64_t n_var, double* hdiag, void* stream);

/* ------------------------------------------------------------------ Davidson
 * Lowest eigenpair of H on V by the Davidson method, which minimises
 * <Psi|H|Psi> - E(<Psi|Psi> - 1) over the coefficients (eq. variational).
 *   c_inout: device float64 [n_var], the start vector (need not be
 *   normalised; a zero vector selects the lowest-diagonal determinant); on
 *   return the normalised eigenvector, signed so that its first entry whose
 *   magnitude is within 1e-6 (relative) of the largest is > 0 (entries
 *   equal by symmetry tie whatever rounding the solve leaves in them, so
 *   the sign does not depend on rounding).
 *   e_out (host): eigenvalue + ecore.  tol: float64 residual norm
 *   ||H c - E c|| at which to stop.  precision HCI_FP32_MIXED iterates with
 *   the mixed product, then refines with float64 products until the float64
 *   residual meets tol.  iters_out (host, may be NULL): products performed.
 *   HCI_E_NOCONV when max_iter products did not reach tol (c and E hold the
 *   best iterate).  The start vector is used as given: one confined to a
 *   symmetry sector of H (see hci_davidson_roots) gives the lowest state of
 *   that sector, as a warm start from the previous state of the same
 *   symmetry intends.  Each iteration's convergence scalars reach the host
 *   through pinned memory the context owns (the host polls them for up to
 *   HCI_DAVIDSON_POLL_MS milliseconds, default 200, then waits on the
 *   stream), so one context must not run two Davidson solves at once.
 *   Synchronises the stream. */
int hci_davidson(hci_ctx ctx, const uint64_t* dets, int64_t n_var, double* c_inout,
                 double* e_out, double tol, int max_iter, int precision, int mode,
                 int* iters_out, void* stream);

/* The nroots lowest eigenpairs of H on V (several states of one space; the
 * paper's stationarity condition eq. variational for each state), by
 * deflation: state r is the lowest eigenpair of Q H Q on the complement of
 * states 0..r-1 (Q = 1 - sum_l c_l c_l^T), found by the solver of
 * hci_davidson with every new direction orthogonalised against the earlier
 * states and every product projected by Q.  Every start vector first gets a
 * fixed pseudo-random component of about 1e-3 of its norm (splitmix64 of
 * the determinant index), so that each solve reaches the lowest state of its
 * complement whatever its symmetry: a start vector confined to one symmetry
 * sector of H (even or odd under the exchange of alpha and beta strings when
 * N_alpha = N_beta and V is closed under it, as selected spaces of such
 * states are) would otherwise converge inside that sector and skip lower
 * states of the other.  States come out in ascending order.
 *   c_inout: device float64 [nroots][n_var]: row r is the start of state r
 *   (a zero row, or one inside the span of the earlier states, selects the
 *   lowest-diagonal determinant that the earlier states hold less than half
 *   of); on return the orthonormal eigenvectors, each with its
 *   sign fixed as in hci_davidson.  e_out: host float64 [nroots], eigenvalues
 *   + ecore.  iters_out: host int [nroots] (may be NULL), products per
 *   state.  1 <= nroots <= min(HCI_MAX_ROOTS, n_var).  tol, max_iter (per
 *   state), precision and mode as in hci_davidson.  HCI_E_NOCONV when some
 *   state missed tol (every state is still written).  Synchronises the
 *   stream. */
int hci_davidson_roots(hci_ctx ctx, const uint64_t* dets, int64_t n_var, int nroots,
                       double* c_inout, double* e_out, double tol, int max_iter,
                       int precision, int mode, int* iters_out, void* stream);

/* <S^2> of the state c on V, to tell which spin state a solve found (the
 * paper's excited states are the lowest of given spin; the determinant space
 * fixes only S_z = (N_alpha - N_beta)/2, so a state of any S >= |S_z| can be
 * the lowest): <S^2> = S_z (S_z + 1) + |S_+ c|^2 / |c|^2 with the spin
 * raising operator S_+ = sum_p a+_{p,alpha} a_{p,beta}, whose images are
 * summed per target determinant in a fixed order.
 *   c: device float64 [n_var], need not be normalised (HCI_E_ARG if zero).
 *   s2_out: host.  Synchronises the stream. */
int hci_spin_square(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c,
                    double* s2_out, void* stream);

/* ---------------------------------------------------------------------- RDMs
 * Spin-traced transition density matrices between bra and ket on V (the
 * Gamma^{x,y} of Sec. "Computational Details"; accumulated by looping over
 * the same single and double connections as sigma).
 *   bra, ket: device float64 [n_var] (may be the same pointer).
 *   rdm1: device float64 [norb][norb]; rdm2: device float64 [norb]^4 (layout
 *   in the header comment); both overwritten.  rdm2 may be NULL.
 * Every sum is taken in an order fixed by the determinant list (no
 * floating-point atomics) and by the device's CU count, so the result is
 * the same bit for bit on every call on a given GPU model; so are the relaxed
 * density matrices of hci_energy_backward. */
int hci_rdm12(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* bra,
              const double* ket, double* rdm1, double* rdm2, void* stream);

/* ----------------------------------------------------------------- backward
 * Derivatives of the energy with respect to the integrals, scaled by grad_e.
 *
 * r == NULL and eps2 <= 0 (variational energy, eq. vdedk2):
 *   dh = grad_e * rdm1(c,c);  dg = grad_e * 1/2 * rdm2(c,c) averaged over the
 *   8 permutations that leave (pq|rs) unchanged.
 *
 * eps2 > 0 (variational + eps2-screened PT2 energy, eq. pt_hci, with the
 * Lagrangian of eq. lagd/eq. lagc and the relaxed gradient eq. lambda): the
 * library builds the first-order vector d on C(eps2), E2, r = dE2/dc, solves
 * Q(H - E)Q z = -Q r (Q = 1 - c c^T) by preconditioned conjugate gradients
 * with float64 residual refinement to z_tol, and assembles
 *   dh, dg from (1 - d.d) Gamma^{cc} + sym Gamma^{zc} + 2 sym Gamma^{dc} + Gamma^{dd}.
 *   e2_out (host, may be NULL) receives E2.
 *
 * r != NULL (caller-supplied dF/dc for some F(c)): as above with the
 *   caller's r and no PT2 pieces: relaxed density (1)Gamma^{cc} + sym Gamma^{zc}.
 *
 *   c: device float64 [n_var] normalised eigenvector; e: its eigenvalue
 *   (ecore included).  dh: device [norb][norb]; dg: device [norb]^4
 *   (overwritten).  z_out: device [n_var] or NULL.  precision applies to the
 *   inner products of the linear solve.  Synchronises the stream. */
int hci_energy_backward(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c,
                        double e, double grad_e, const double* r, double eps2, double z_tol,
                        int precision, double* dh, double* dg, double* z_out, double* e2_out,
                        void* stream);

/* eps2-screened second-order energy and its pieces on a frozen V, c, E0
 * (eq. h0, eq. pt_hci; Hylleraas minimiser d_a = N_a / (E0 - H_aa)).
 *   e2_out (host): E2.  r_out: device float64 [n_var] = dE2/dc at fixed E0,
 *   or NULL.  n_conn_out (host, may be NULL): |C(eps2)|.
 *   Synchronises the stream. */
int hci_pt2(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double e0,
            double eps2, double* e2_out, double* r_out, int64_t* n_conn_out, void* stream);

/* Freeze the screened pair set of the second-order energy at the current
 * integrals: M = {(i, a): D_a outside V, one excitation from D_i,
 * fl(|H_ai| |c_i|) > eps2} (eq. pt_hci's screening), kept in the context
 * for hci_energy(..., frozen = 1).  The energy E_var + E2 is then a smooth
 * function of the integrals on the frozen V and M, whose derivative is the
 * relaxed density matrix of hci_energy_backward at the same point (eq.
 * lambda); re-screening at perturbed integrals would make it jump.  The set
 * survives hci_ctx_update_integrals and is replaced by the next freeze.
 *   dets, c: device, as hci_pt2.  n_pairs_out (host, may be NULL): |M|.
 *   HCI_E_NOMEM if the pairs exceed the pt2 budget (a frozen set is held in
 *   one pass).  Synchronises the stream. */
int hci_pt2_freeze(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double eps2,
                   int64_t* n_pairs_out, void* stream);

/* The energy E = E_var + E2 of a frozen determinant list (eq. variational,
 * eq. pt_hci): the lowest eigenpair by hci_davidson from c_inout (tol,
 * max_iter, precision, mode as there), then E2 of that eigenpair: over the
 * pair set of hci_pt2_freeze (frozen != 0; HCI_E_ARG if the set belongs to
 * another list or none exists), else re-screened at eps2 (eps2 = 0: E2 = 0).
 *   c_inout: device float64 [n_var], start vector in, eigenvector out.
 *   e_out: host [3] = {E_var, E2, E_var + E2} (ecore included).
 *   iters_out: host or NULL.  HCI_E_NOCONV as hci_davidson (energies of the
 *   best iterate written).  Synchronises the stream. */
int hci_energy(hci_ctx ctx, const uint64_t* dets, int64_t n_var, double* c_inout, double tol, int max_iter,
               int precision, int mode, double eps2, int frozen, double* e_out, int* iters_out, void* stream);

/* Extrapolation to the full-CI limit (Sec. "Results and discussion": the
 * procedure of the butadiene calculations).  Starting from the largest
 * calculation (dets, c), level k keeps the m_k most important determinants
 * (one ranking by decreasing |c_i|, ties by increasing index, so the levels
 * are nested; m_0 = n_var, m_k = max(1, ceil(m_{k-1} (1 - fraction)))),
 * solves for its lowest eigenpair (Davidson from c restricted to the level,
 * tolerance tol, precision as hci_davidson) and its screened E2 at eps2
 * (as hci_pt2).  A least-squares line E_var + E2 = a + b E2 over the levels
 * gives the full-CI estimate a.
 *   c: device float64 [n_var], the largest calculation's eigenvector (not
 *   modified).  levels >= 2, 0 < fraction < 1 (the paper uses 0.33),
 *   eps2 >= 0, tol > 0 (else HCI_E_ARG).
 *   nvar_out, evar_out, e2_out: host [levels]: m_k, E_var (ecore included),
 *   E2.  fit_out: host [3]: a, b, and the error estimate
 *   0.25 |a - (E_var + E2)_0|.  HCI_E_NOCONV when a level's Davidson does
 *   not converge.  Synchronises the stream. */
int hci_extrapolate(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double fraction,
                    int levels, double eps2, double tol, int precision, int64_t* nvar_out, double* evar_out,
                    double* e2_out, double* fit_out, void* stream);

/* Orbital gradient for active-active rotations (Sec. "HCI self-consistent
 * field": eq. vdedk2 with the variational density matrices, eq. lambda with
 * the relaxed ones).  For orbitals rotated by U = exp(kappa), kappa
 * antisymmetric (h' = U^T h U, (pq|rs)' = sum U_ap U_bq U_cr U_ds (ab|cd)),
 * the energy E = sum h_pq gamma_pq + 1/2 sum (pq|rs) Gamma_pqrs of fixed
 * density matrices has dE/dkappa_xy = 2 (F_xy - F_yx) at kappa = 0, with
 * F = h gamma + G, G_xy = sum_qrs (xq|rs) Gamma_yqrs (the integrals of the
 * context).
 *   rdm1: device float64 [n][n] gamma; rdm2: device float64 [n]^4 Gamma, both
 *   with the index symmetries of a real state (gamma symmetric,
 *   Gamma_pqrs = Gamma_rspq = Gamma_qpsr), as hci_rdm12 (bra = ket) returns
 *   them, or gamma = dh and Gamma = 2 dg of hci_energy_backward.
 *   grad: device float64 [n][n], antisymmetric (overwritten).
 *   Asynchronous on the stream. */
int hci_orbital_gradient(hci_ctx ctx, const double* rdm1, const double* rdm2, double* grad, void* stream);

/* hci_orbital_gradient for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result, bit for bit, with the partial sums held in a
 * fixed device array of 16 MiB per GPU (512 tiles of 64 x 64 float64, enough
 * for every norb <= 64), whose address the library resolves once per device
 * in hci_ctx_create; the array stays allocated until the process ends.  The
 * call allocates nothing (no hipMalloc, no allocator callback).  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (two
 * streams, two threads, two contexts) race and must be serialised by the
 * caller.  Arguments as hci_orbital_gradient; HCI_E_UNSUPPORTED if the split
 * would need more tiles than the array holds.  Asynchronous on the stream. */
int hci_orbital_gradient_noalloc(hci_ctx ctx, const double* rdm1, const double* rdm2, double* grad,
                                 void* stream);

/* Integrals of the context's h, g in rotated orbitals phi'_p = sum_a phi_a U_ap:
 * h_out = U^T h U, g_out_pqrs = sum_abcd U_ap U_bq U_cr U_ds (ab|cd) (the
 * active-space integral transformation of the orbital step).  U: device
 * float64 [n][n] (row a, column p), normally orthogonal (not checked).
 * h_out: device [n][n]; g_out: device [n]^4 (overwritten; not aliasing the
 * context's copies).  Hand them to hci_ctx_update_integrals to continue with
 * the rotated orbitals.  Scratch: 2 n^4 float64.  Asynchronous on the stream. */
int hci_rotate_integrals(hci_ctx ctx, const double* U, double* h_out, double* g_out, void* stream);

/* Device memory (bytes) the screened PT2 pairs may hold at once (default
 * 64 GiB, about 128 B per pair).  hci_pt2 and the deterministic part of
 * hci_pt2_semistochastic take the pairs in several passes over a hash
 * partition of the connected determinants when they exceed it (the memory
 * bottleneck of eq. pt_hci); so does hci_energy_backward with eps2 > 0,
 * which accumulates r, Gamma^{dc} and Gamma^{dd} pass by pass.  The passes
 * are sized from a count pass before any pair is stored.  bytes <= 0:
 * HCI_E_ARG. */
int hci_ctx_set_pt2_budget(hci_ctx ctx, int64_t bytes);

/* Sampled estimates of the screened second-order energy of eq. pt_hci, the
 * stochastic terms of eq. semistoc, at two thresholds from the same draws.
 * Batch b draws n_samp rows of V with replacement: row i has probability
 * p_i = q_i / Q with integer weights q_i = max(1, round(2^31 |c_i| / max|c|))
 * (0 for c_i = 0), and draw k picks the row whose cumulative weight range
 * holds min(Q - 1, floor(u[b][k] Q)).  With multiplicities w_i and
 * x_ai = H_ai c_i over the screened pairs of the drawn rows,
 *   E2^S = sum_a [S1^2 - S2 + (n_samp - 1) S3] / (n_samp (n_samp - 1) (E0 - H_aa)),
 *   S1 = sum w x / p, S2 = sum (w x / p)^2, S3 = sum w x^2 / p,
 * an unbiased estimate of E2(eps) (the paper defers the estimator to its
 * reference; this is the reading used).
 *   dets, c: as hci_pt2; e0: variational energy (ecore included).
 *   u: device float64 [n_batch][n_samp], the caller's uniforms in [0, 1)
 *   (a value outside: HCI_E_ARG).  e2s_out, e2sd_out: host [n_batch],
 *   E2^S(eps2) and E2^S(eps2_d) of each batch.  Needs 0 <= eps2 <= eps2_d,
 *   n_samp >= 2, n_batch >= 1 and c != 0 (else HCI_E_ARG).
 *   Synchronises the stream. */
int hci_pt2_stochastic(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double e0,
                       double eps2, double eps2_d, const double* u, int64_t n_samp, int64_t n_batch,
                       double* e2s_out, double* e2sd_out, void* stream);

/* Semistochastic second-order energy, eq. semistoc:
 *   E2 = E2^D(eps2_d) + mean_b [E2^S_b(eps2) - E2^S_b(eps2_d)],
 * E2^D by hci_pt2 at eps2_d (in passes when over the pt2 budget), the
 * batches as hci_pt2_stochastic.  e2_out (host): E2.  err_out (host, may be
 * NULL): standard error of the mean over batches (NaN for one batch).
 * e2d_out (host, may be NULL): E2^D(eps2_d).  Arguments and errors as
 * hci_pt2_stochastic.  Synchronises the stream. */
int hci_pt2_semistochastic(hci_ctx ctx, const uint64_t* dets, int64_t n_var, const double* c, double e0,
                           double eps2, double eps2_d, const double* u, int64_t n_samp, int64_t n_batch,
                           double* e2_out, double* err_out, double* e2d_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HCI_MI355X_H */
