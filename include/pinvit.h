/*
 * pinvit.h -- C ABI of the MI355X block-sparse PINVIT library (libpinvit.so).
 *
 * The library computes the lowest eigenvalue of a second-quantised fermionic
 * Hamiltonian restricted to N particles (Section 1.1, eqs. hamil and Hevp),
 *     H = sum_ij h_ij a_i^* a_j + sum_ijkl v_ijkl a_i^* a_j^* a_k a_l ,
 * with the state held as a particle-number block-sparse matrix product state
 * (Section 2.3) and iterated by preconditioned inverse iteration with rank
 * truncation (Algorithm 2, "perturbed inverse (inner) iteration"), using the
 * exponential-sum preconditioner of Section 4 (Cor. lrprecond).
 *
 * Conventions
 * -----------
 * - Orbitals are 0-based: orbital i of the paper is index i-1 here.
 * - h: L*L doubles, row-major, h[i*L+j] multiplies a_i^* a_j.
 * - v: L^4 doubles, row-major, v[((i*L+j)*L+k)*L+l] multiplies a_i^* a_j^* a_k a_l
 *   (the paper's one-half is already inside).  Only the antisymmetrised combination
 *   enters, as in the paper's sum.
 * - gamma: shift; the library works with H_gamma = H + gamma (Section 3.1), applied
 *   as gamma/N added to every h_ii, which equals H + gamma on the N-particle space.
 * - Block table rho: an (L+1) x (N+1) int32 array, row-major, rho[k*(N+1)+n] is the
 *   dimension of sector n on bond k (n = number of particles among orbitals 1..k).
 *   Entries outside K_k = {max(0,N-L+k)..min(N,k)} are 0; rho[0][0] = rho[L][N] = 1.
 * - A joint MPS (several columns, pv_run_subspace_joint) has rho[L][N] = D, the column
 *   index; its last blocks have D columns.
 * - MPS data layout (export and import): sites k = 1..L in order; inside a site,
 *   left sectors n in K_{k-1} ascending; for each, the unoccupied block U_{k,n}
 *   (rho[k-1][n] x rho[k][n], present when n is in K_k) followed by the occupied
 *   block O_{k,n} (rho[k-1][n] x rho[k][n+1], present when n+1 is in K_k)
 *   (eq. blockstructure); each block column-major (rows = left bond), float64.
 * - MPS handles are small integers owned by a context; every operation that produces
 *   an MPS returns a new handle.  pv_mps_free releases one.
 * - Host pointers are owned by the caller and are only read or written during the
 *   call.  The context owns all device memory and one HIP stream (or uses the caller's,
 *   see pv_create); all calls on a context are synchronous with respect to the host on
 *   return.
 * - A context is used by one thread at a time.  Errors never throw across the ABI:
 *   every call returns a pv_status and pv_last_error() describes the last failure of
 *   the calling thread.
 */
#ifndef PINVIT_H
#define PINVIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pv_ctx pv_ctx;

typedef enum {
  PV_OK = 0,
  PV_EINVAL = -1,    /* invalid argument (sizes, handles, non-finite input) */
  PV_ENOMEM = -2,    /* device allocation failed */
  PV_EDEVICE = -3,   /* HIP runtime error or no device */
  PV_ENOTSPD = -4,   /* t_min <= 0 (D not positive) or 2x2 Ritz pencil not definite */
  PV_ENOCONV = -5,   /* iteration limit reached before the tolerance (pv_run only) */
  PV_ESTATE = -6     /* call out of order (e.g. no Hamiltonian set) */
} pv_status;

/* Parameters of Algorithm 2 (Section 5.3-5.4, Section 7.1.3). */
typedef struct {
  int rank_cap;     /* maximal total rank per bond after every truncation (>= 1) */
  int m_zip;        /* intermediate rank cap of the H application; <= 0: exact */
  int max_iter;     /* iteration limit */
  double tau;       /* stop when the eigenvector error bound (eq. everrbound) <= tau */
  double c0;        /* exponential-sum accuracy (Thm. expsum), the paper uses 0.1 */
  double c;         /* spectral-equivalence constant of A (eq. specequivA) */
  double delta;     /* gap constant delta >= lambda_2/(lambda_2-lambda_1) */
  double eps_num;   /* residual accuracy; <= 0 selects (1-c)/2 (Section 7.1.3) */
  double t_eig;     /* Rayleigh-quotient truncation slack, the paper uses 1/2 */
  double c_lower;   /* C_lower of eq. lowerupper (enters alpha_0 only); <= 0: 1 */
  double c_upper;   /* C_upper of eq. lowerupper; <= 0: 1 */
  int max_retries;  /* limit of the residual-tolerance reductions per iteration */
  int precision;    /* 0: float64 everywhere; 1: the operator contractions of H psi and of
                     *    the two Ritz sandwiches run on float32 MFMA (operands rounded to
                     *    float32, float32 accumulation), while truncations, norms, the
                     *    Rayleigh quotient lambda and the residual stay float64; 2: the
                     *    same contractions with operands rounded to bfloat16 (float32
                     *    accumulation on bfloat16 MFMA); other values give PV_EINVAL */
  int truncation;   /* 0: sequential TT-SVD truncation (eq. ttsvdquasiopt), two-pass Gram
                     *    factorisations; 1: simultaneous truncation of all bonds from Gram
                     *    matrices (tolerance eps/sqrt(L-1) per bond), see pv_set_truncation */
  /* Resume state from a previous pv_run (pv_result fields eta_res, s_last, s_prev);
   * resume_s <= 0 starts afresh with a trial residual for the first tolerance. */
  double resume_eta, resume_s, resume_s2;
} pv_params;

/* One row of the iteration history. */
typedef struct {
  double lambda;      /* Rayleigh quotient of H_gamma (eq. exactrq) */
  double energy;      /* lambda - gamma */
  double rho;         /* residual bound rho^n (eq. rhobound) */
  double bound;       /* eigenvector error bound (eq. everrbound), NaN outside its domain */
  double r_norm;      /* ||r||, r = trunc(H_gamma psi - lambda psi), ||psi|| = 1 */
  double s_norm;      /* ||S r|| = residual of the preconditioned problem */
  double eta_res;     /* accepted residual tolerance */
  double lambda_star; /* lower Ritz value of the 2x2 step (Rem. omegamin) */
  double eta_psi;     /* truncation tolerance of the update */
  double seconds;     /* wall time of the iteration */
  int retries;        /* tolerance reductions (x 4/5) taken */
  int cap_bound;      /* 1 if any truncation of the iteration was limited by rank_cap, the
                       * intermediate rank m_zip dropped a singular value, or a simultaneous
                       * truncation could not certify its tolerance (see pv_set_truncation) */
  int max_rank;       /* maximal bond rank of the new iterate */
  int stopped;        /* 1 on the iteration where the tolerance test succeeded */
  int zip_bound;      /* 1 if m_zip dropped a singular value above the numerical-zero level in
                       * the H application of the accepted residual: r is then not within
                       * eta_res of H_gamma psi - lambda psi, rho and bound are estimates, and
                       * the run does not stop on them */
  double zip_discard; /* sqrt of the sum of the squared singular values that m_zip dropped
                       * there, in the panels' own metric (the discarded part of H psi is
                       * that weight times at most the norm of the operator's right parts) */
} pv_iter;

typedef struct {
  double energy, lambda, rho, bound;
  double eta_res, s_last, s_prev;  /* state for resuming (see pv_params) */
  int iterations;     /* number of history rows written */
  int converged;
} pv_result;

/* One step m of the outer iteration (Algorithm 3). */
typedef struct {
  double eta;         /* eta^m (eta^0 = 1/(2 theta)) */
  double tau;         /* eigenvector tolerance of the inner run, eta^m/(2(1+(1+alpha)kappa)) */
  double lambda;      /* Rayleigh quotient at the end of the inner run */
  double energy;      /* lambda - gamma */
  double rho;         /* residual bound rho of the inner run's last iteration */
  double rel_bound;   /* relative eigenvalue bound of eq. releigerr (NaN outside its domain) */
  double trunc_eps;   /* psi-space tolerance s_min theta eta^m of the outer truncation (0 on the last step) */
  int inner_iterations;
  int cap_bound;      /* 1 if the outer truncation was limited by rank_cap */
  int max_rank;       /* maximal bond rank after the step */
  int stopped;        /* 1 on the step whose eigenvalue bound met tol */
} pv_outer_iter;

/* Largest number of columns of the subspace iteration. */
#define PV_SUBSPACE_MAX_D 8

/* One row of the subspace iteration history (Algorithm 4); entries i >= D are unused. */
typedef struct {
  double lambda[PV_SUBSPACE_MAX_D];      /* Rayleigh quotients of the E-orthonormal Ritz basis, ascending */
  double energy[PV_SUBSPACE_MAX_D];      /* lambda - gamma */
  double rho[PV_SUBSPACE_MAX_D];         /* residual bound of each column (eq. rhobound) */
  double s_norm[PV_SUBSPACE_MAX_D];      /* ||S r_i|| */
  double lambda_star[PV_SUBSPACE_MAX_D]; /* lowest D Ritz values of the 2D-dimensional step */
  double bound;       /* eigenvector error bound of column 1 (eq. everrbound), NaN outside its domain */
  double eta_res;     /* accepted residual tolerance (per column) */
  double eta_psi;     /* truncation tolerance of each new column */
  double seconds;     /* wall time of the iteration */
  int retries;        /* tolerance reductions (x 4/5) taken */
  int cap_bound;      /* 1 if any truncation of the iteration was limited by rank_cap */
  int max_rank;       /* maximal bond rank over the new columns */
  int stopped;        /* 1 on the iteration where the tolerance test succeeded */
} pv_subspace_iter;

const char* pv_last_error(void);

/* Context on HIP device `device`.  stream: a hipStream_t of the caller on that device
 * that every launch of the context goes to (the caller keeps ownership and must keep it
 * alive until pv_destroy), or NULL for a stream the context creates and destroys.  The
 * simultaneous truncation also forks work to a side stream of its own, ordered by events
 * before and after.  Fails with PV_EDEVICE when there is no GPU. */
pv_status pv_create(pv_ctx** out, int device, void* stream);
void pv_destroy(pv_ctx* ctx);

/* Copies h, v; builds the MPO of H_gamma (Thm. opranks, host) and uploads it; computes
 * theta_i (Section 7.1.1), t_min, t_max and the exponential-sum terms (Section 4.3). */
pv_status pv_set_hamiltonian(pv_ctx* ctx, int L, int N, const double* h, const double* v,
                             double gamma);

/* Preconditioner scalars: out[0..6] = t_min, t_max, T, h, alpha_0 (C_lower=C_upper=1
 * unless set by pv_run), s_min, s_max; m_range[0..1] = M^-, M^+. */
pv_status pv_precond_info(pv_ctx* ctx, double* out, int* m_range);

/* MPS management.  pv_mps_create copies `n` doubles in the export layout with the
 * given block table; pv_mps_determinant builds the rank-one determinant with the
 * listed N occupied orbitals (Section 7.1.4). */
pv_status pv_mps_create(pv_ctx* ctx, const int32_t* rho, const double* data, size_t n, int* handle);
pv_status pv_mps_determinant(pv_ctx* ctx, const int32_t* occupied, int* handle);
pv_status pv_mps_layout(pv_ctx* ctx, int handle, int32_t* rho, size_t* n);
pv_status pv_mps_download(pv_ctx* ctx, int handle, double* data, size_t n);
pv_status pv_mps_free(pv_ctx* ctx, int handle);

/* Truncation used by pv_round, pv_apply_h and pv_apply_s on this context.
 * mode 0: sequential TT-SVD: right-orthogonalisation, then bond by bond from the left the
 *   kept left singular vectors of the current tensor (Section 2.2); each bond discards at
 *   most (eps/sqrt(L-1))^2.  Singular values from a two-pass Gram eigendecomposition.
 * mode 1: simultaneous truncation P_1 ... P_{L-1} x, P_k the projector onto the kept left
 *   singular vectors of the k-th matricisation of x itself, every bond decided from the
 *   left and right Gram matrices in one batched step with tolerance eps/sqrt(L-1); since
 *   x - P_1 Y = (I - P_1) x + P_1 (x - Y) is an orthogonal sum, ||x - trunc(x)||^2 is at
 *   most the sum of the bonds' discarded tails (eq. ttsvdquasiopt).  Singular values are
 *   accurate to about 1e-8 of the largest; those at or below 1e-6 of it are numerical
 *   zeros, and when their weight exceeds a bond's share of eps^2 the tolerance is not
 *   certified and cap_bound is reported.  The intermediate-rank H application uses
 *   single-pass factorisations. */
pv_status pv_set_truncation(pv_ctx* ctx, int mode);

/* Tuning of the symmetric eigensolver behind every truncation (the Householder reduction
 * to tridiagonal form, Section 2.2's SVDs taken through Gram matrices): a batch of at most
 * max_problems matrices is reduced one Householder step per launch with several
 * workgroups per matrix; a larger batch by panels of 32 steps with one workgroup per
 * matrix and GEMM trailing updates.  Both give the same decomposition up to rounding.
 * Default PV_TRIDIAG_STEPS_DEFAULT.  PV_EINVAL for max_problems < 0. */
#define PV_TRIDIAG_STEPS_DEFAULT 1073741824
pv_status pv_set_tridiag_steps(pv_ctx* ctx, int max_problems);

/* Tile shape of the float64 grouped GEMM (the operator contractions, environments, Gram
 * matrices and trailing updates; no passage of the paper: a tuning of this library).
 * Two shapes exist, 64 x 64 and 32 x 32 tiles; both form every element of C by the same
 * chain of MFMA products in the same order, so the shape never changes a result bit,
 * only the time.  Modes:
 *   PV_GEMM_TILES_RULE  (default) 32 x 32 for launches of at most 256 64 x 64 tiles;
 *   PV_GEMM_TILES_TUNE  online autotuner: a launch is keyed by (device, kernel, log2 of
 *                       its 64 x 64 tile count, log2 of its longest K); the first eight
 *                       launches of a key alternate the shapes, each timed by its own
 *                       start and stop events (read at the context's next
 *                       synchronisation), then the key keeps the shape with the smaller
 *                       time per flop; the rule decides meanwhile;
 *   PV_GEMM_TILES_TABLE the tuner's decided keys without further exploration, the rule
 *                       for the others;
 *   PV_GEMM_TILES_SMALL, PV_GEMM_TILES_LARGE  one shape forced (measurement, tests).
 * The table is one per process, shared by every context and host thread.  The
 * float32 and bfloat16 kernels have the 64 x 64 shape only.  The context's stream is
 * synchronised first.  PV_EINVAL for other modes. */
#define PV_GEMM_TILES_RULE 0
#define PV_GEMM_TILES_TUNE 1
#define PV_GEMM_TILES_TABLE 2
#define PV_GEMM_TILES_SMALL 3
#define PV_GEMM_TILES_LARGE 4
pv_status pv_set_gemm_tiles(pv_ctx* ctx, int mode);

/* The autotuner's table: *n_rows receives the number of keys; the first
 * min(n_rows, max_rows) rows of 9 doubles go to rows (host, row-major): device, kernel
 * precision (0 float64, 2 float64 trailing updates), log2 bucket of the 64 x 64 tile
 * count, log2 bucket of the longest K, choice (-1 undecided, 0: 64 x 64, 1: 32 x 32),
 * samples of the 64 x 64 and of the 32 x 32 shape, and their measured rates in TFLOP/s.
 * rows may be NULL when max_rows is 0.  PV_EINVAL for a null n_rows or a negative
 * max_rows.  pv_gemm_tune_clear empties the table (no context may be running). */
pv_status pv_gemm_tune_table(double* rows, int max_rows, int* n_rows);
pv_status pv_gemm_tune_clear(void);
/* Load n_rows rows (host, row-major, the layout pv_gemm_tune_table writes) into the table,
 * replacing the entries of their keys: a table measured once (on this device model and
 * workload) serves later processes in PV_GEMM_TILES_TABLE mode without exploring.  The
 * stored rates are kept (pv_gemm_tune_table returns them unchanged).  Every row is checked
 * before any is loaded: PV_EINVAL for non-finite values, a kernel precision other than 0
 * or 2, a choice outside -1..1, negative counts, rates or buckets, or NULL rows with
 * n_rows > 0. */
pv_status pv_gemm_tune_load(const double* rows, int n_rows);

/* <a|b> (Euclidean inner product) by a transfer sweep. */
pv_status pv_dot(pv_ctx* ctx, int a, int b, double* out);
/* <bra|H_gamma|ket> by an environment sweep with the MPO (eq. exactrq, one term). */
pv_status pv_expect_h(pv_ctx* ctx, int bra, int ket, double* out);
/* a*x + b*y as block concatenation (Section 2.3: addition = concatenation). */
pv_status pv_lincomb(pv_ctx* ctx, double a, int x, double b, int y, int* out);
/* trunc(x; eps, cap): sequential TT-SVD truncation (eq. ttsvdquasiopt), eps/sqrt(L-1)
 * per bond, at most `cap` total rank per bond.  Result left-orthogonal, norm in the last
 * core.  *cap_bound (may be NULL) is set to 1 when the cap limited a bond. */
pv_status pv_round(pv_ctx* ctx, int x, double eps, int cap, int* out, int* cap_bound);
/* trunc(H_gamma x; eps, cap), H applied site by site (Section 2.4, applied one site at a
 * time) with intermediate rank m_zip (m_zip <= 0: exact product up to numerical zeros):
 * x is made right-orthogonal, then at site k the carry is contracted with x_k and the MPO
 * core and the panel of every new sector is factorised; across the sectors the m_zip
 * largest singular values are kept.  The intermediate result is Q Q^T H x for the
 * orthonormal left basis Q it builds.  *cap_bound (may be NULL) is set when the cap or
 * m_zip limited a rank; *zip_discard (may be NULL) receives the square root of the sum
 * of the squared singular values that m_zip dropped, in the panels' own metric. */
pv_status pv_apply_h(pv_ctx* ctx, int x, double eps, int cap, int m_zip, int* out, int* cap_bound,
                     double* zip_discard);
/* S x by the sorted sequential truncated sum of Lemma truncr with total tolerance eta. */
pv_status pv_apply_s(pv_ctx* ctx, int x, double eta, int cap, int* out, int* cap_bound);

/* Algorithm 2 from the determinant of the N smallest h_ii (ties: lower index), or from
 * the MPS `start` when start >= 0.  Writes up to hist_cap history rows; *psi (may be
 * NULL) receives a handle of the final iterate.  The run stops (converged) when the
 * eigenvector bound meets tau, or when the search direction S^2 r vanishes under the
 * truncation tolerances (the iterate is then an eigenvector to those tolerances, as on a
 * sector of dimension 2). */
pv_status pv_run(pv_ctx* ctx, const pv_params* prm, int start, pv_result* res,
                 pv_iter* hist, int hist_cap, int* psi);

/* Outer iteration (Algorithm 3, Section 5.6, Thm. quasioptr) from the determinant:
 * kappa = sqrt((1+c)/(1-c)) sqrt(L-1) (eq. kappadef), theta = (1+alpha) kappa /
 * (2 (1 + (1+alpha) kappa)), eta^0 = 1/(2 theta).  Step m runs Algorithm 2 (pv_run with
 * prm, tau replaced by eta^m/(2(1+(1+alpha)kappa)), at most prm->max_iter iterations) from
 * the current iterate; it stops when the relative eigenvalue bound of eq. releigerr of
 * the last residual bound is below tol; otherwise the normalised iterate is truncated with
 * tolerance s_min theta eta^m (rank cap prm->rank_cap) and eta is halved.  Writes up to
 * hist_cap rows; res->iterations = outer steps taken, res->converged = 1 when tol was met;
 * *psi (may be NULL) receives the final iterate.  PV_EINVAL for alpha <= 0, tol <= 0 or
 * max_outer < 1; errors of an inner run are returned with the step named. */
pv_status pv_run_outer(pv_ctx* ctx, const pv_params* prm, double alpha, double tol, int max_outer,
                       pv_result* res, pv_outer_iter* hist, int hist_cap, int* psi);

/* Algorithm 2 on the paper's own variable x (the "z-form"), for checking the psi-form of
 * pv_run on small problems.  The products with A = S H_gamma S and E = S^2 are summed term
 * by term over the pairs of rank-one terms S_k of S (eq. exactrq); the residual is the sorted
 * sequential truncated sum of its (M^+ - M^- + 1)^2 terms S_k (H_gamma - lambda) S_k' x,
 * each formed exactly (Lemma truncr and the recipe after it), and eta_res starts from their
 * norms (eq. startetar); x is normalised in the A-norm; the Ritz step uses {x, r/||r||};
 * the update x <- trunc_{eta_in}(x_*) truncates x itself.  Each H application is exact up to
 * m_zip (<= 0: exact) and numerically zero singular values, so the sizes are limited by the
 * eigensolver (n <= 1024 per sector Gram): L up to about 10 at small ranks.  hist rows use
 * pv_iter with s_norm = r_norm = ||res_eta(x)|| and eta_psi = eta_in; x (NULL or one int)
 * receives a handle of the final iterate (in the variable x).  Errors as pv_run. */
pv_status pv_run_zform(pv_ctx* ctx, const pv_params* prm, int start, pv_result* res, pv_iter* hist,
                       int hist_cap, int* x);

/* Algorithm 4 (perturbed inverse subspace iteration, Section 6) on D columns, 1 <= D <=
 * PV_SUBSPACE_MAX_D, in the physical variable psi = S x like pv_run.  The columns are kept
 * as D block-sparse MPS rather than one joint MPS with an index core (Section 6.2): the
 * normalisation Psi <- Psi V of each iteration is carried as a D x D coefficient matrix
 * and applied exactly (MPS concatenation) where a column is needed, and every truncation
 * of the iterate acts on each column with the whole tolerance.  Per iteration: D x D
 * Rayleigh-Ritz on the current columns (E-orthonormal Ritz basis, Rayleigh quotients
 * ascending); per column the residual and its preconditioned forms as in pv_run (one
 * tolerance eta_res for all columns, reduced while the smallest ||S r_i|| is below
 * (1 + 1/zeta) eta_res); termination on the eigenvector bound of column 1; a 2D x 2D
 * Rayleigh-Ritz step on the columns and their normalised directions S^2 r_i; the new
 * columns truncated with s_min eta_in, eta_in the smallest of the per-column tolerances
 * of Algorithm 4.  The small generalised eigenproblems are solved on the host.
 * starts: D MPS handles of the starting columns (not consumed), or NULL for the
 * determinant of the N smallest h_ii and its D-1 single excitations i -> a of smallest
 * h_aa - h_ii (ties: lower i, then lower a).  res describes column 1 (energy, lambda,
 * rho, bound); hist receives up to hist_cap rows; psi (NULL or D ints) receives handles of
 * the final columns (the Ritz basis of the last iteration when it stopped, else the last
 * truncated update).  The run also stops (converged) when every direction vanishes under
 * the truncation tolerances (the columns then span an invariant subspace to those
 * tolerances); PV_ENOCONV when only some vanish.  PV_EINVAL for a D out of range, a
 * sector of dimension below 2D (the 2D Ritz vectors would be dependent) or invalid
 * parameters, PV_ESTATE without a Hamiltonian, PV_ENOTSPD when a Gram or Ritz pencil is
 * not positive definite. */
pv_status pv_run_subspace(pv_ctx* ctx, const pv_params* prm, int D, const int* starts, pv_result* res,
                          pv_subspace_iter* hist, int hist_cap, int* psi);

/* Algorithm 4 with the D columns held jointly (Section 6.2, joint tensor parameterisation):
 * one block-sparse MPS whose right boundary rho[L][N] = D is the column index (the
 * paper's additional core at position K+1).  The steps are those of pv_run_subspace, but
 * every product with H, residual (R = H Psi - Psi Lambda), sorted S sum and truncation acts
 * on all columns at once: one tolerance for the joint tensor (Frobenius norm) and ranks
 * shared by the columns, which need a rank cap of up to the sum of the columns' ranks.
 * The normalisation Psi <- Phi V and the Ritz combinations [Psi | P] W are applied to the
 * column index (the last core).  start: a handle of a joint MPS with D columns
 * (pv_mps_create with rho[L][N] = D, columns in the last core's column index), or -1 for
 * the D start determinants of pv_run_subspace; *psi (may be NULL) receives the handle of
 * the final joint MPS.  res, hist and the errors as pv_run_subspace. */
pv_status pv_run_subspace_joint(pv_ctx* ctx, const pv_params* prm, int D, int start, pv_result* res,
                                pv_subspace_iter* hist, int hist_cap, int* psi);

/* Learned correction of the preconditioner diagonal (an extension, not in the paper).
 * The correction Delta (L x (N+1), row-major, entry [i][n]) changes theta_i to
 * theta_i + Delta_{i,n} on the occupied state of site i when n particles sit on the sites
 * before it, so each term alpha_m exp(-beta_m d) of S stays a product of site factors;
 * t_min and t_max become the extremes of the corrected diagonal d over the N-particle
 * determinants, and alpha_m, beta_m, s_min, s_max follow from them as for the plain S.
 *
 * pv_set_correction: delta (host, L (N+1) doubles, copied) is used by pv_run,
 * pv_run_outer, pv_run_subspace and pv_apply_s until cleared by NULL or a new
 * Hamiltonian; pv_run_zform then fails with PV_ESTATE.  Like pv_set_hamiltonian it sets
 * up S with c0 = 0.1 for pv_apply_s and pv_precond_info (the runs set it up from their
 * own parameters).  PV_EINVAL for non-finite entries,
 * PV_ENOTSPD when some theta_i + Delta_{i,n} (n < N) is not positive.
 *
 * The network: per row (i, n) the six features theta_i/tbar, h_ii/tbar, n/N, i/L, <n_i>
 * of the iterate and lambda/(N tbar) (tbar = mean |theta_i|, lambda the Rayleigh quotient
 * of the iterate), two hidden layers of PV_MLP_WIDTH units with tanh and a linear output
 * z; Delta = (min_i theta_i / 2) tanh(z) (zero when min theta_i <= 0).  params holds
 * PV_MLP_PARAMS float32 values: W1 (width x 6, row-major), b1, W2 (width x width,
 * row-major), b2, W3, b3.  The passes use the parameters rounded to bfloat16 and float32
 * MFMA products.  psi: the iterate whose densities and Rayleigh quotient enter the
 * features, or -1 for the start determinant of pv_run.
 *
 * pv_learned_correction: writes Delta (L (N+1) doubles) to delta.
 * pv_learned_train: `steps` Adam steps (beta1 0.9, beta2 0.999, epsilon 1e-8, learning
 * rate lr, zero initial moments) on loss = mean_b (d(m_b) - <m_b|H + gamma|m_b>)^2 / tbar^2
 * over the nmask determinants m_b (bit i = orbital i; each must hold N particles within
 * the L <= 64 orbitals).  params is updated in place; loss (NULL or steps + 1 doubles)
 * receives the loss before each step and after the last; grad (NULL or PV_MLP_PARAMS
 * doubles) the gradient at the final parameters.  PV_EINVAL for nmask < 1, steps < 0,
 * lr < 0, L > 64 or a mask with the wrong particle number; the Adam moments start at
 * zero on every call. */
#define PV_MLP_WIDTH 256
#define PV_MLP_PARAMS (PV_MLP_WIDTH * 6 + PV_MLP_WIDTH + PV_MLP_WIDTH * PV_MLP_WIDTH + PV_MLP_WIDTH + PV_MLP_WIDTH + 1)
pv_status pv_set_correction(pv_ctx* ctx, const double* delta);
pv_status pv_learned_correction(pv_ctx* ctx, const float* params, int psi, double* delta);
pv_status pv_learned_train(pv_ctx* ctx, float* params, int psi, const uint64_t* masks, int nmask, int steps,
                           float lr, double* loss, double* grad);

/* The solve form of the training (an extension): the misfit
 *     loss = sum_b (r_b / d(m_b) - t_b)^2 / sum_b t_b^2
 * between the corrected diagonal preconditioner's action on a residual r of the method
 * (r_b = <m_b|r>) and the exact solve t = (H + gamma)^{-1} r on the N-particle sector
 * (t_b = <m_b|t>), d(m) the corrected diagonal of the determinant m; S^2 is close to
 * 1/d, so the network learns to make S^2 act on the method's residuals like the exact
 * inverse.  rvals, tvals: nmask doubles each (host).  Otherwise as pv_learned_train
 * (features from psi, Adam, params updated in place, loss and grad outputs). */
pv_status pv_learned_train_solves(pv_ctx* ctx, float* params, int psi, const uint64_t* masks, int nmask,
                                  const double* rvals, const double* tvals, int steps, float lr, double* loss,
                                  double* grad);
/* Attach a network (PV_MLP_PARAMS float32 values, copied) to the runs of this context:
 * pv_run recomputes the correction from the current iterate's features (densities and
 * Rayleigh quotient) on its first iteration and every `refresh` iterations after, and
 * sets up S with it as pv_set_correction does.  NULL detaches it (a new Hamiltonian
 * does too).  PV_EINVAL for refresh < 1 or non-finite parameters. */
pv_status pv_set_learned_network(pv_ctx* ctx, const float* params, int refresh);

/* Per-step judge of a corrected S (the learned correction, an extension without a paper
 * passage; the plain S of Section 4.3 is the fallback).  With on = 1 and a correction in
 * force (pv_set_correction or an attached network), every iteration of pv_run forms the
 * search direction twice from the same residual r and tolerance eta: with the corrected
 * S, and with the plain S (its own s_max and s_min).  The direction whose 2 x 2 Ritz
 * value (eq. reducedevp) is lower makes the step; the corrected one on ties.  The update's
 * truncation tolerance takes the chosen S's s_min; the iteration's rho and bound are
 * those of the corrected S.  A judged iteration costs two more S applications, two
 * sandwiches and an inner product.  Default off.  pv_learned_judge_counts returns how
 * many steps of the last pv_run each S won.  PV_EINVAL for on outside {0, 1} or null
 * arguments. */
pv_status pv_set_learned_judge(pv_ctx* ctx, int on);
pv_status pv_learned_judge_counts(pv_ctx* ctx, int* plain, int* corrected);
/* x = (H + gamma)^{-1} b on the N-particle sector by preconditioned conjugate gradients in
 * block-sparse form: the products with H by the exact H application, the preconditioner
 * S^2 (every term of both S applications kept), and every sum truncated only at its
 * numerical zeros (no rank cap), until ||b - H x|| <= rel_tol ||b|| (recursive residual)
 * or max_iter steps.  *out receives the handle of x; iters and rel_res (may be NULL) the
 * steps taken and the final relative residual.  The ranks are those of the exact
 * solution, so this is for the small sizes that generate training targets. */
pv_status pv_solve_h(pv_ctx* ctx, int b, double rel_tol, int max_iter, int* out, int* iters, double* rel_res);
/* out[i] = <m_i|x> for the determinants masks[i] (bit j = orbital j occupied; each must
 * hold N particles, L <= 64), by transfer sweeps with their rank-one MPS. */
pv_status pv_mps_amplitudes(pv_ctx* ctx, int handle, const uint64_t* masks, int n, double* out);

/* Batched independent problems (many Hamiltonians of uneven size at once): runs pv_run from
 * the determinant on each of the `count` distinct contexts ctxs[i] (each with its
 * Hamiltonian already set) with parameters prm[i], writing res[i] and, when status is not
 * NULL, status[i].  Each context keeps its own HIP stream and memory pool; up to 16 host
 * threads drive them at once, so the device overlaps the kernels of different problems.
 * The results are those of pv_run on each context alone (the kernels are deterministic).
 * Returns PV_OK when every problem succeeded, else the status of the first failed problem,
 * whose message pv_last_error gives; PV_EINVAL for null pointers or a repeated context.
 * A context must not be used by another thread during the call. */
pv_status pv_run_batch(pv_ctx* const* ctxs, int count, const pv_params* prm, pv_result* res, pv_status* status);

/* Kernel timing of the last pv_run / op, accumulated with HIP events per kernel class:
 * out[i] = milliseconds, flops[i] = algorithmic flops (GEMM: sum 2mnk; eigenproblems:
 * Jacobi 10/3 n^3 each; tridiagonal solver: panel kernels 2/3 n^3 flops and 4/3 n^3
 * bytes (the symmetric products), trailing updates as GEMMs, step launches 6 m^2 flops
 * and 16 m^2 bytes for a trailing block of order m (the block read and written), the
 * LDS tail 4/3 m^3 flops and 8 m^2 bytes, back-transformation 2 n^2 k for k wanted
 * vectors; Cholesky panels: n^3/3 over all panels), bytes[i] = algorithmic bytes, for
 * i < n classes (fourteen classes: grouped GEMM float64, Jacobi eigensolver, MPO W-step,
 * copy/scale, split-K reduction, tridiagonal reduction (panels or step launches),
 * Cholesky panels, grouped GEMM float32, eigenvectors of the tridiagonal matrix,
 * back-transformation, eigenvalues of the tridiagonal matrix, trailing updates of the
 * tridiagonal reduction, grouped GEMM with bfloat16 operands, the tail of the step
 * reduction (last 192 steps in one workgroup)); the step launches are timed one in eight, each standing for the launches
 * up to the next timed one;
 * names via pv_timer_name. */
pv_status pv_timers(pv_ctx* ctx, int n, double* ms, double* flops, double* bytes, int* calls);
const char* pv_timer_name(int i);
pv_status pv_timers_reset(pv_ctx* ctx);
/* Which kernel classes are timed: bit i of mask enables class i (pv_timer_name(i)); the
 * default is every class.  Each timed launch records two HIP events, which costs the host
 * a few microseconds per launch; classes left out accumulate nothing.  Takes effect for
 * the launches after the call (the context's stream is synchronised first). */
pv_status pv_set_timer_mask(pv_ctx* ctx, uint32_t mask);

/* Sampled timing for classes with many short launches: a class in mask (and in the timer
 * mask) records events on a pseudo-random one-in-every subset of its launches (chosen by
 * a hash of the launch's index, so no regular launch pattern biases it), and each timed
 * launch counts for `every` launches in pv_timers (milliseconds, flops, bytes and calls).
 * The averages per launch are those of the sample.  every = 1: every launch.  PV_EINVAL
 * for every < 1.  The step launches of the tridiagonal reduction are always timed one in
 * eight. */
pv_status pv_set_timer_sampling(pv_ctx* ctx, uint32_t mask, int every);

/* Symmetric eigenproblem on the device (the eigensolvers behind the Gram
 * factorisations): A is n x n column-major (upper triangle read), w receives the
 * eigenvalues descending, V (n x n) the eigenvectors.  method 0: cyclic Jacobi with
 * relative accuracy on nearly diagonal input; 1: Householder tridiagonalisation,
 * bisection and inverse iteration (eigenvectors of eigenvalues <= 1e-12 max|lambda|
 * are returned as zero).  For tests. */
pv_status pv_sym_eig(pv_ctx* ctx, int n, const double* A, double* w, double* V, int method);

/* Attainable float64 MFMA rate of the context's device in TFLOP/s, measured: eight
 * workgroups of four wavefronts per compute unit, each wavefront a chain of 20,000 steps
 * of four independent 16x16x4 float64 MFMA products on register operands (no memory
 * traffic), timed with HIP events on the context's stream (about 20 ms).  The ceiling
 * against which the grouped GEMM's rate can be read beside the published peak.
 * PV_EINVAL for null arguments. */
pv_status pv_mfma_f64_rate(pv_ctx* ctx, double* tflops);

/* C = alpha op(A) op(B) + beta C on the device through the grouped block GEMM of the
 * operator contractions (the tile shape and split-K choice are the library's own):
 * column-major host arrays, op(A) = A (M x K, ld lda) for ta = 0 or A^T (A is K x M) for
 * ta = 1, likewise op(B) (K x N) with tb; C is M x N with ld ldc.  precision 0: float64
 * MFMA; 1: operands rounded to float32, float32 accumulation; 2: operands rounded to
 * bfloat16, float32 accumulation.  PV_EINVAL for bad sizes,
 * leading dimensions or flags.  For tests. */
pv_status pv_gemm(pv_ctx* ctx, int M, int N, int K, const double* A, int lda, int ta, const double* B, int ldb,
                  int tb, double* C, int ldc, double alpha, double beta, int precision);

/* As pv_sym_eig with method 1, but eigenvectors only for the nvec largest eigenvalues
 * (0 <= nvec <= n; columns nvec.. of V are zero; all n eigenvalues are returned).  The
 * truncations use this form: they select ranks from the eigenvalues first and compute
 * the kept vectors only.  PV_EINVAL for nvec outside [0, n].  For tests. */
pv_status pv_sym_eig_top(pv_ctx* ctx, int n, const double* A, double* w, double* V, int nvec);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the eigensolver of pv_sym_eig with
 * method 1, on device buffers, allocating nothing.  A (n x n, column-major, upper triangle
 * read), w (n, eigenvalues descending) and V (n x n, eigenvectors; those of eigenvalues
 * <= 1e-12 max|lambda| are zero) are device pointers owned by the caller; the call runs on
 * the context's stream and has finished when it returns (make the inputs ready first).
 * The work area (7 n^2 + 5 n + 2 doubles) and the launch descriptor live in a file-scope
 * device array sized for n <= PV_NOALLOC_MAX_N (about 14.7 MB, held on every device the
 * library runs on until the process ends); PV_EINVAL for larger n.  Every call on one
 * device shares that array, so calls that overlap on one device (several contexts or
 * threads at once) race; no kernel timing is recorded.  The call always takes the
 * step reduction to tridiagonal form, whatever pv_set_tridiag_steps says for the context.
 * No hipMalloc, hipFree or HIP event creation happens inside the call. */
#define PV_NOALLOC_MAX_N 512
pv_status pv_sym_eig_noalloc(pv_ctx* ctx, int n, const double* A, double* w, double* V);

/* Cholesky factor of a symmetric positive semidefinite matrix on the device (the factor
 * of the left Gram matrices in the simultaneous truncation): A is n x n column-major
 * (lower triangle read), W (n x n) receives a lower triangular W with W W^T = A up to
 * the columns whose pivot falls to 1e-12 of their diagonal entry, which are zero.  For
 * tests. */
pv_status pv_cholesky(pv_ctx* ctx, int n, const double* A, double* W);

/* Host-only diagnostics (no GPU needed). */
/* Bond dimensions of the MPO of H: dims[0..L] and per-charge counts q=-2..2 in
 * qdims[(L+1)*5]. */
pv_status pv_mpo_bond_dims(int L, const double* h, const double* v, int32_t* dims, int32_t* qdims);
/* Dense 2^L x 2^L matrix of H + gamma/N * sum_i n_i from the MPO, row-major,
 * index bit i = occupation of orbital i (L <= 8). */
pv_status pv_mpo_dense(int L, const double* h, const double* v, double diag_shift, double* out);

#ifdef __cplusplus
}
#endif
#endif /* PINVIT_H */
