/*
 * dmrg.h -- C ABI of libdmrg, the MI355X (gfx950) superblock H*psi library.
 *
 * The library applies the DMRG superblock Hamiltonian of a grown system S'
 * and a grown environment E' (paper Sec. 1 and Sec. 3.1, Fig. 2 steps (c)-(f))
 *
 *     y = ( H_S' (x) I + I (x) H_E' + sum_k c_k A_k (x) B_k ) psi
 *
 * without ever forming the superblock matrix (Sec. 3.3: the S'(x)E' product is
 * a basis only; its Hamiltonian is applied on the fly from the S' and E'
 * operators).  psi lives only in the targeted symmetry sector (Sec. 3.3:
 * only the blocks with the targeted quantum numbers are diagonalised) and is
 * stored block-sparse by effective quantum number (Sec. 3.2).  Every term is
 * evaluated per symmetry block as Y_q += c_k A_k[q<-q'] Psi_q' B_k^T.
 *
 * Conventions common to all entry points
 * --------------------------------------
 * - Every function returns dmrg_status; none throws, aborts or prints.  On an
 *   error the outputs are left untouched and dmrg_last_error() (per host
 *   thread) describes the failure.
 * - "_h" pointers are host memory, "_d" pointers are device memory on the
 *   context's device.  Device buffers passed in are owned by the caller and
 *   must stay valid until the work queued on the context's stream is done.
 * - All device work is queued on the stream given to dmrg_ctx_create.
 *   dmrg_hpsi and dmrg_hpsi_adjoint's psi gradient are asynchronous; the
 *   calls that return host scalars synchronise that stream.
 * - Precision: operator blocks and vectors cross the boundary in FP64.  The
 *   block products run in the precision chosen at build time (FP64, FP32 on
 *   the matrix cores, or BF16 hi/lo split x3); Lanczos vectors,
 *   reorthogonalisation, the tridiagonal eigen-solve and the density-matrix
 *   eigen-solve are always FP64.
 */
#ifndef DMRG_H
#define DMRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DMRG_OK = 0,
  DMRG_E_ARG = 1,          /* null pointer, negative size, bad enum value        */
  DMRG_E_QN = 2,           /* quantum numbers inconsistent, or empty target      */
  DMRG_E_SHAPE = 3,        /* a block's size disagrees with its sectors          */
  DMRG_E_NOMEM = 4,        /* device or host allocation failed / over the cap    */
  DMRG_E_DEVICE = 5,       /* HIP runtime error, or no device for this call      */
  DMRG_E_NOCONV = 6,       /* Lanczos hit its iteration cap (partial result out) */
  DMRG_E_UNSUPPORTED = 7   /* a term shape the fused kernel does not handle      */
} dmrg_status;

typedef enum {
  DMRG_FP64 = 0,        /* FP64 matrix-core grouped kernel                          */
  DMRG_FP32 = 1,        /* FP32 matrix-core grouped kernel, FP32 accumulate         */
  DMRG_BF16X3 = 2,      /* BF16 hi/lo split, hi*hi + hi*lo + lo*hi, FP32 accumulate */
  DMRG_FP64_PLAIN = 3   /* one launch per (term, symmetry block), FP64 FMA; the
                           straightforward baseline                                 */
} dmrg_prec;

typedef struct dmrg_ctx_s* dmrg_ctx;   /* a device, a stream, workspace        */
typedef struct dmrg_sb_s* dmrg_sb;     /* one superblock: plan + staged blocks */

/* A basis split into symmetry sectors (Sec. 3.2: the effective quantum
 * numbers in increasing order and the partition into equal-q runs).
 *   nsec  number of sectors (>= 1)
 *   q     [nsec] effective quantum numbers, strictly increasing
 *   dim   [nsec] states per sector, each >= 1                                  */
typedef struct {
  int32_t nsec;
  const int64_t* q;
  const int32_t* dim;
} dmrg_basis;

/* A block-sparse operator on one basis.  Quantum numbers add under products
 * (Sec. 3.2), so an operator shifts q by a fixed delta: block (r, c) may be
 * present only if q[r] - q[c] == delta, and each row sector at most once.
 *   delta    q(row) - q(col)
 *   nblk     number of stored blocks
 *   row_sec  [nblk] row sector index
 *   col_sec  [nblk] column sector index
 *   blk      [nblk] host FP64, row-major dim[row_sec] x dim[col_sec]
 * Blocks whose rows hold at most one nonzero each (operators of the newest
 * site, I (x) o) are stored by the library as a gather (index + scale); all
 * others as dense blocks.  The caller's arrays are copied during
 * dmrg_build_superblock and may be freed on return.                         */
typedef struct {
  int64_t delta;
  int32_t nblk;
  const int32_t* row_sec;
  const int32_t* col_sec;
  const double* const* blk;
} dmrg_op;

/* One term c * A (x) B of the superblock Hamiltonian (Sec. 3.3: the
 * system part, the environment part and the system-environment connection;
 * the connection is split into one term per bond operator product).
 * A acts on S', B on E'; NULL means the identity.  delta(A) + delta(B) must
 * be 0.  group is a free label carried for the caller (e.g. which coupling
 * the term belongs to).                                                      */
typedef struct {
  double c;
  const dmrg_op* A;
  const dmrg_op* B;
  int32_t group;
} dmrg_term;

/* Result of dmrg_rho_truncate (library-owned; valid until the next
 * dmrg_rho_truncate on the same superblock or dmrg_sb_destroy).
 *   trunc_err   sum of the discarded eigenvalues (Sec. 1, eps_tr)
 *   kept        number of kept states
 *   straddle    1 if the cut fell inside a cluster of tied eigenvalues
 *   lambda      [kept] kept eigenvalues in selection order
 *   lambda_sec  [kept] sector of each kept eigenvalue
 *   nsec        sectors of the truncated side's basis
 *   kept_per_sec[nsec] kept states per sector
 *   W           [nsec] row-major dim[s] x kept_per_sec[s] eigenvector blocks,
 *               columns in decreasing eigenvalue order (NULL if none kept)
 *   W_all       the same blocks back to back in sector order (W[s] points
 *               into it), W_total doubles, so a caller can copy them at once */
typedef struct {
  double trunc_err;
  int32_t kept;
  int32_t straddle;
  const double* lambda;
  const int32_t* lambda_sec;
  int32_t nsec;
  const int32_t* kept_per_sec;
  const double* const* W;
  const double* W_all;
  int64_t W_total;
} dmrg_trunc;

/* ---------------------------------------------------------------------- */

/* Create a context on HIP device `device`, queueing work on `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  One context per host
 * thread.                                                                  */
dmrg_status dmrg_ctx_create(int device, void* hip_stream, dmrg_ctx* out);
void dmrg_ctx_destroy(dmrg_ctx ctx);

/* Set the stream later work is queued on (e.g. the caller's current stream). */
dmrg_status dmrg_ctx_set_stream(dmrg_ctx ctx, void* hip_stream);

/* Device-memory cap (failure injection and budgeting; not a paper
 * passage).  dmrg_ctx_set_mem_cap(ctx, bytes): the device memory the
 * library holds on the context's device -- every context and superblock on
 * that device together: staged operators, tile images, Lanczos and
 * density-matrix workspaces -- may not exceed `bytes` (0: no cap, the
 * default).  An allocation that would pass it fails, and the call that
 * needed it returns DMRG_E_NOMEM (as it does when the device itself is out
 * of memory) with nothing half-built: the superblock or context stays
 * usable and the call can be repeated after the cap is raised.  A cap below
 * what is already held frees nothing; it refuses further growth.
 * DMRG_E_ARG for bytes < 0.  dmrg_ctx_mem: bytes held and the cap (either
 * pointer may be NULL).  Memory the caller allocates (vectors passed in) and
 * the fixed scratch array of dmrg_hpsi_noalloc are not counted.            */
dmrg_status dmrg_ctx_set_mem_cap(dmrg_ctx ctx, int64_t bytes);
dmrg_status dmrg_ctx_mem(dmrg_ctx ctx, int64_t* used, int64_t* cap);

/* Timing of the product kernels.  dmrg_ctx_set_timing(ctx, every): with
 * every >= 1, every every-th product launch the library makes on this
 * context (dmrg_hpsi and the products inside dmrg_lanczos_ground, counted
 * in launch order) is bracketed by HIP events on the context's stream, and
 * all product launches are counted; every = 0 turns both off.  A stride
 * above 1 keeps the events' own cost out of the timed work while the
 * sampled launches still give the average kernel time.
 * dmrg_ctx_timing synchronises on the last event and returns, for
 * precision `prec` (a dmrg_prec value), the summed event time (ms) and the
 * number of timed launches, and in *products (if not null) the number of
 * all launches made while timing was on; reset != 0 then forgets all of
 * them.  Negative `every` is DMRG_E_ARG.                                    */
dmrg_status dmrg_ctx_set_timing(dmrg_ctx ctx, int32_t every);
dmrg_status dmrg_ctx_timing(dmrg_ctx ctx, int32_t prec, double* ms_total, int64_t* launches,
                            int64_t* products, int32_t reset);

/* Message describing the last failure on this host thread ("" if none).   */
const char* dmrg_last_error(void);

/* Library version string.                                                   */
const char* dmrg_version(void);

/* Build a superblock: validate the quantum-number algebra (Sec. 3.2), match
 * S' sector q with E' sector q_target - q (the target pairs, ordered by S'
 * sector), lay out psi, classify blocks (dense / gather), build and
 * cost-balance the work-tile schedule, and stage the operators on the device
 * in `prec` (plus FP64 copies, used for FP64 refinement).
 *   ctx may be NULL: then only the host plan is built (layout and statistics
 *   can be queried; every device entry point returns DMRG_E_DEVICE).
 * Errors: DMRG_E_QN (q not increasing, block breaks delta, term not
 * q-neutral, no target pair), DMRG_E_SHAPE, DMRG_E_UNSUPPORTED (a term with
 * dense blocks on both sides), DMRG_E_NOMEM, DMRG_E_DEVICE.              */
dmrg_status dmrg_build_superblock(dmrg_ctx ctx, const dmrg_basis* S, const dmrg_basis* E,
                                  int64_t q_target, int32_t nterms, const dmrg_term* terms,
                                  dmrg_prec prec, dmrg_sb* out);
void dmrg_sb_destroy(dmrg_sb sb);

/* An operator between two target sectors (for spectral functions, Eq. (5):
 * c_i maps the ground state's sector to one with an electron less): inputs
 * live in the q_in sector, outputs in q_out, both laid out as
 * dmrg_build_superblock would lay them out for that target; every term must
 * shift q by q_out - q_in (DMRG_E_QN otherwise).  dmrg_hpsi and
 * dmrg_hpsi_adjoint work on it; the Lanczos and density-matrix calls need
 * q_in == q_out (DMRG_E_ARG).                                               */
dmrg_status dmrg_build_operator(dmrg_ctx ctx, const dmrg_basis* S, const dmrg_basis* E,
                                int64_t q_in, int64_t q_out, int32_t nterms,
                                const dmrg_term* terms, dmrg_prec prec, dmrg_sb* out);

/* Input and output vector lengths of a superblock or operator.             */
dmrg_status dmrg_sb_dims(dmrg_sb sb, int64_t* D_in, int64_t* D_out);

/* psi layout (Eq. (1) restricted to the target): npairs blocks; block p is
 * the row-major dim_S[s_sec[p]] x dim_E[e_sec[p]] matrix Psi_p starting at
 * element off[p]; D = total length.  Arrays are library-owned.            */
dmrg_status dmrg_sb_layout(dmrg_sb sb, int64_t* D, int32_t* npairs, const int64_t** off,
                           const int32_t** s_sec, const int32_t** e_sec);

/* Work statistics of one H*psi: algorithmic flops (dense blocks at their
 * stored size, gathers at 2 flops per element touched), flops the matrix
 * cores issue (padded tiles), algorithmic bytes (operators once in the
 * compute precision, psi read once and y written once in FP64; a product
 * with beta != 0 also reads y, 8 bytes per element more), and the number of
 * work tiles.  Any pointer may be NULL.                                      */
dmrg_status dmrg_sb_stats(dmrg_sb sb, double* flops_alg, double* flops_exec,
                          double* bytes_alg, int32_t* ntiles);

/* Replace the term coefficients c_k (nterms values, host) without a rebuild. */
dmrg_status dmrg_sb_set_coeffs(dmrg_sb sb, const double* c_h);

/* Select the block-product precision used by dmrg_hpsi (the superblock
 * stages FP64 copies always, and `prec`'s copies if it was built with it
 * or if this call stages them).                                            */
dmrg_status dmrg_sb_set_prec(dmrg_sb sb, dmrg_prec prec);

/* Tile-shape autotuner for the FP32 and BF16 products: times every variant
 * of the product on this superblock (reps launches each, on zeroed device
 * vectors the call allocates and frees) and keeps the fastest for later
 * products.  Variant 0: 32 x 32 output tiles, the sixteen waves of a
 * workgroup splitting a tile's contraction, one tile list per compute unit.
 * Variant 1: 64 x 64 output tiles whose two operand panels are staged once
 * in LDS for four waves; all tiles' contraction stages dealt out in equal
 * shares to the workgroups (a tile may be cut between workgroups, whose
 * partial sums a second kernel adds in a fixed order).  Both are
 * deterministic and within the same rounding bound; their results differ
 * in the last bits (different summation orders).  *variant (may be NULL) receives the choice; FP64 and
 * the plain baseline have one variant (0).  Synchronous.                    */
dmrg_status dmrg_sb_autotune(dmrg_sb sb, int32_t reps, int32_t* variant);

/* Pin the product variant for the current precision (0 or 1, as
 * dmrg_sb_autotune reports it); DMRG_E_ARG for an unknown variant.  FP64
 * products ignore it.  Variant 1's plan and padded operator pool are built
 * and uploaded the first time variant 1 is pinned or the autotuner runs
 * (synchronous, allocates; DMRG_E_NOMEM possible), not when the FP32
 * operators are staged.                                                     */
dmrg_status dmrg_sb_set_variant(dmrg_sb sb, int32_t variant);

/* Reorthogonalisation of dmrg_lanczos_ground's basis (paper Sec. 3.3 gives
 * the recursion, not a scheme).  mode 0 (the default): after each restart
 * cycle's first step, the local three-term recurrence at every step and one
 * Gram-Schmidt pass against the whole basis on every other step, which keeps
 * the basis semi-orthogonal (overlaps of order 1e-7 with reduced-precision
 * products); small dimensions always take mode 1.  mode 1: classical
 * Gram-Schmidt twice against the whole basis at every step (orthogonal to
 * working precision, about twice the passes over the basis).  DMRG_E_ARG
 * for another mode.                                                          */
dmrg_status dmrg_sb_set_reorth(dmrg_sb sb, int32_t mode);

/* Launch batching of dmrg_lanczos_ground (Sec. 3.3's recursion, one product
 * and its orthogonalisation per step).  enable 1: the steps between two of
 * the host's convergence checks (every fourth step) are captured into a HIP
 * graph the first time their position in a restart cycle is reached, on a
 * non-blocking stream the context owns, and replayed on the context's
 * stream at that position in every later cycle and solve on this
 * superblock; a restart cycle's first step and the steps near the end of a
 * cycle or of the product cap run as ordinary launches.  Results are the
 * same bits as with enable 0 (the same kernels with the same arguments in
 * the same order).  Products inside the graphs take no timing events
 * (dmrg_ctx_set_timing still counts them).  The graphs hold the context's
 * Lanczos buffers and the superblock's staged operators at the time of
 * capture; a solve that finds any of them moved, or another precision,
 * kernel variant or reorthogonalisation mode, captures afresh.  enable 0
 * (the default) synchronises the context's stream and frees the graphs.
 * DMRG_E_ARG for another value or a superblock without a device context.
 * dmrg_sb_graph_stats: the number of captures and of graph launches so far
 * (either pointer may be NULL).                                             */
dmrg_status dmrg_sb_set_graphs(dmrg_sb sb, int32_t enable);
dmrg_status dmrg_sb_graph_stats(dmrg_sb sb, int64_t* captures, int64_t* replays);

/* y_d = alpha * H psi_d + beta * y_d (paper Sec. 3.3: the Lanczos solver's
 * only need, x += H y, with alpha = beta = 1).  psi_d and y_d are device FP64
 * arrays of length D in the dmrg_sb_layout order and must not overlap.
 * Asynchronous on the context's stream.                                    */
dmrg_status dmrg_hpsi(dmrg_sb sb, const double* psi_d, double* y_d, double alpha, double beta);

/* The product of dmrg_hpsi for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments and result, but every temporary (the
 * FP32 copy of psi that the FP32 and BF16 products read, and the partial
 * tiles of the macro-tile variant) lives in a fixed device scratch array of
 * 2^24 floats (64 MiB) that the library holds on each device from the first
 * dmrg_ctx_create there until the process ends; the call makes no
 * allocation and takes no timing events.  DMRG_E_NOMEM if D_in + 16 exceeds
 * 2^24; when the macro-tile variant is selected but its partial tiles do
 * not fit beside psi, the 32 x 32 tile variant runs.  Calls on one device
 * share the scratch: calls that
 * overlap on one GPU (other host threads, other streams) race; calls queued
 * on one stream do not.  Asynchronous on the context's stream.            */
dmrg_status dmrg_hpsi_noalloc(dmrg_sb sb, const double* psi_d, double* y_d, double alpha, double beta);

/* Adjoint of the product, for differentiation:
 *   gpsi_d = H^T g_d                 (device, length D, overwritten)
 *   gc_h[k] = < g, (A_k (x) B_k) psi >  (host, nterms values; may be NULL)
 * Synchronises the stream when gc_h is not NULL.                          */
dmrg_status dmrg_hpsi_adjoint(dmrg_sb sb, const double* psi_d, const double* g_d,
                              double* gpsi_d, double* gc_h);

/* Lowest eigenpair of H in the target sector by Lanczos (Sec. 3.3), with
 * FP64 vectors reorthogonalised as dmrg_sb_set_reorth selects (by default
 * semi-orthogonally: the local recurrence at every step, one Gram-Schmidt
 * pass against the whole basis on every other step).  When the
 * superblock computes in reduced precision, each restart cycle begins with
 * one FP64 product (Rayleigh quotient and residual in FP64) and continues in
 * the reduced precision; cycles repeat until the FP64 residual
 * || H psi - E psi || <= tol.
 *   psi0_d    device FP64 [D] start vector (not modified; normalised inside)
 *   max_iter  cap on the total number of products
 *   E0_h      the FP64 Rayleigh quotient of the returned vector
 *   psi_d     device FP64 [D] normalised ground state (may alias psi0_d)
 *   iters_h   products used;  resid_h  final FP64 residual norm
 * Returns DMRG_E_NOCONV (outputs still written) if the cap is reached.
 * Synchronises the stream.                                                 */
dmrg_status dmrg_lanczos_ground(dmrg_sb sb, const double* psi0_d, int32_t max_iter, double tol,
                                double* E0_h, double* psi_d, int32_t* iters_h, double* resid_h);

/* The Lanczos recursion (Sec. 3.3) from an arbitrary start vector, for the
 * continued fraction of a spectral function (the paper's LDOS, Eq. (5),
 * computed from H's tridiagonal form on c_i|psi>).  v0_d (device, length D)
 * is normalised inside; *norm0_h = ||v0||.  nsteps products with full FP64
 * reorthogonalisation; alpha_h[k], beta_h[k] (host, nsteps each) receive the
 * diagonal and the coupling of step k to k+1; *steps_h the number of steps
 * before the recursion broke down (an invariant subspace), at most nsteps.
 * Synchronises the stream.                                                  */
dmrg_status dmrg_lanczos_tridiag(dmrg_sb sb, const double* v0_d, int32_t nsteps, double* alpha_h,
                                 double* beta_h, int32_t* steps_h, double* norm0_h);

/* Reduced density matrix of S' (side 0, Eq. (2): rho_S = Psi Psi^T) or E'
 * (side 1, Eq. (3): rho_E = Psi^T Psi), formed per symmetry block on the
 * device in FP64, diagonalised per block in FP64 on the host, eigenvalues
 * ordered decreasingly with ties (relative gap <= 1e-6; values < 1e-13
 * counted as 0) broken by (q ascending, in-sector index ascending); the first
 * m are kept, all if m >= dimension (Sec. 1).  no_split != 0 extends the cut
 * to the end of a straddled nonzero tie cluster.  Synchronises the stream. */
dmrg_status dmrg_rho_truncate(dmrg_sb sb, const double* psi_d, int32_t side, int32_t m,
                              int32_t no_split, dmrg_trunc* out);

/* One block of a basis change (Eq. (4) with (w)^-1 read as W^T, a truncated W
 * having orthonormal columns):  out = Wr^T O Wc, where
 *   O    rows x cols, row stride o_ld (0: cols), at O_d + o_off
 *   Wr   rows x kr,   row-major, at W_d + wr_off  (kept eigenvectors of the row sector)
 *   Wc   cols x kc,   row-major, at W_d + wc_off  (kept eigenvectors of the column sector)
 *   out  kr x kc,     row stride out_ld (0: kc), at out_d + out_off
 * (The strides let O be a column slice of a larger block and out a slice of
 * a psi block, as the wave-function transformation between DMRG steps
 * needs.)                                                                    */
typedef struct {
  int64_t o_off;
  int32_t rows, cols;
  int64_t wr_off;
  int32_t kr;
  int64_t wc_off;
  int32_t kc;
  int64_t out_off;
  int32_t o_ld, out_ld;
} dmrg_tblock;

/* Change the basis of block operators and truncate them (Sec. 1: H_S' and
 * the other operators in the kept density-matrix eigenvectors; Eq. (4)),
 * all blocks in two FP64 matrix-core launches (U = O^T Wr, out = U^T Wc).
 * O_d, W_d, out_d are device FP64 buffers owned by the caller; blocks[] is
 * host memory.  Asynchronous on the context's stream.  DMRG_E_ARG on a
 * negative size or null pointer.                                             */
dmrg_status dmrg_transform_blocks(dmrg_ctx ctx, int32_t nblk, const dmrg_tblock* blocks,
                                  const double* O_d, const double* W_d, double* out_d);

/* ---------------------------------------------------------------------- */
/* Host utilities (no device needed): the FP64 eigen-solvers the library   */
/* uses for the Lanczos tridiagonal matrix and the density-matrix blocks.  */

/* All eigenpairs of the symmetric n x n row-major matrix a (host): w[n]
 * receives the eigenvalues in ascending order, column c of a the
 * eigenvector of w[c] (Householder tridiagonalisation, implicit QR with
 * Wilkinson shifts).  DMRG_E_NOCONV if the sweeps do not converge.        */
dmrg_status dmrg_host_sym_eigen(int32_t n, double* a, double* w);

/* Local density of states of Eq. (5) from Lanczos coefficients of H on
 * phi = c|psi> (host): out[k] = 2 weight Im f(E0 - omega[k] - i eta), with
 * f(z) = 1/(z - a_0 - b_0^2/(z - a_1 - b_1^2/(...))) over n steps and
 * weight = ||phi||^2; i.e. 2 pi sum_n |<n|c|psi>|^2 L_eta(omega - (E0 - E_n))
 * with L_eta a unit-area Lorentzian of half-width eta.                      */
dmrg_status dmrg_host_ldos(int32_t n, const double* alpha, const double* beta, double weight,
                           double e0, int32_t nomega, const double* omega, double eta, double* out);

/* Lowest eigenpair of the symmetric tridiagonal matrix with diagonal
 * alpha[n] and off-diagonal beta[n-1] (Sturm bisection + inverse
 * iteration); u[n] normalised, first nonzero component positive.          */
dmrg_status dmrg_host_tridiag_lowest(int32_t n, const double* alpha, const double* beta,
                                     double* theta, double* u);

#ifdef __cplusplus
}
#endif

#endif /* DMRG_H */
