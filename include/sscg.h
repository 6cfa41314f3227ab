/*
 * sscg.h - Sakurai-Sugiura eigensolver for the Hermitian Wilson fermion matrix,
 * with one shifted-CG run solving every quadrature shift (gfx950 / MI355X).
 *
 * Paper: H. Ohno, Y. Kuramashi, T. Sakurai, H. Tadano, "A quadrature-based
 * eigensolver with a Krylov subspace method for shifted linear systems for
 * Hermitian eigenproblems in lattice QCD" (arXiv:1004.0292).
 *
 * Conventions shared by every call
 * --------------------------------
 *  Lattice   dims = {Lx, Ly, Lz, Lt}, V = Lx Ly Lz Lt sites, periodic in all four
 *            directions; site s = x + Lx (y + Ly (z + Lz t)).
 *  Spinors   complex128 (interleaved re, im doubles), canonical layout
 *            [nsrc][V][4 spin][3 colour]; a vector has n = 12 V complex entries,
 *            entry 12 s + 3 spin + colour.
 *  Gauge     complex128 [4 mu][V][3][3], row-major colour matrices; mu = 0..3 is
 *            x, y, z, t and U_mu(x) multiplies psi(x + mu) in the forward hop.
 *  Matrix    A = gamma5 (I - kappa D) (Sec. 4), Hermitian, with the Wilson hopping
 *            matrix (r = 1)
 *              (D psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                   + (1 + gamma_mu) U_mu(x-mu)^H psi(x-mu)]
 *            and Dirac matrices in the chiral basis, gamma5 = diag(1, 1, -1, -1).
 *  Memory    "device" pointers are HIP device allocations on the context's device
 *            (e.g. torch tensors); "host" pointers are ordinary host memory. The
 *            caller owns every buffer it passes; the context owns the packed gauge
 *            field and all workspaces (allocated on first use of a given shape,
 *            reused, freed by sscg_destroy). Nothing is allocated inside the
 *            iteration loop.
 *  Streams   all device work runs on the stream given to sscg_create (NULL = the
 *            default stream). Calls marked "stream-ordered" return before the work
 *            is done; the others synchronise that stream before returning.
 *  Errors    every int-returning call returns SSCG_OK or a negative status; no
 *            exception or abort crosses the ABI. On error the outputs are
 *            undefined and sscg_last_error() holds a message. One context must not
 *            be used from two host threads at once.
 *  Launch    kernel launch shapes (dslash kernel, sources per thread, block or tile
 *  shapes    size, t-slices per block, XCD order; shift batch width, load unroll,
 *            streaming stores) are chosen by timing on first use of each problem
 *            shape. Timing noise can make two processes pick different shapes, so
 *            results agree to rounding, not bit for bit, across processes. The
 *            environment variable SSCG_AUTOTUNE=0, or any of SSCG_NR, SSCG_BS,
 *            SSCG_XCD, SSCG_CT, SSCG_TBS, SSCG_WBATCH, SSCG_UNROLL, SSCG_NT set,
 *            fixes the shapes (read at sscg_create); with fixed shapes a solve is
 *            bitwise reproducible (the reductions do not depend on the schedule).
 *            SSCG_BLOCK (0, 4, 8, 16, 24 or 32; default 24) sets the block length B
 *            of the in-loop moment update (see moments_in_loop; 0 selects the
 *            per-iteration form); SSCG_MOMUB (1, 2 or 4; default 1) sets how many
 *            shifts' loads the per-iteration form issues together, and SSCG_MOMPF
 *            (default 1) whether it issues the next group's loads before the
 *            current group's stores (all read at the start of each solve; the
 *            results agree to rounding across them).
 */
#ifndef SSCG_H
#define SSCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sscg_ctx sscg_ctx;

enum {
  SSCG_OK = 0,
  SSCG_EINVAL = -1,      /* bad argument (size, pointer, parameter range)        */
  SSCG_ENOMEM = -2,      /* device or pinned host allocation failed              */
  SSCG_EDEVICE = -3,     /* a HIP call failed                                    */
  SSCG_ENOTCONV = -4,    /* maxiter reached before every shift converged         */
  SSCG_EBREAKDOWN = -5,  /* <p, (sigma I - A) p> = 0 or a non-finite CG scalar   */
  SSCG_ESTATE = -6,      /* call out of order (e.g. no gauge field set)          */
  SSCG_EINACCURATE = -7  /* a mixed-precision solve converged, but some shift's
                            FP64 true residual exceeds true_factor * tol          */
};

enum { SSCG_FP64 = 0,    /* every vector, product and scalar in FP64                 */
       SSCG_MIXED = 1,   /* FP64 until the largest active shifted residual falls
                            below switch_tol, then FP32 dslash, FP32 seed and shift
                            vectors, with FP64 reliable updates of the seed residual
                            every ru_interval iterations; scalar recurrences and dot
                            products stay FP64. The FP32 seed can lose the FP64
                            convergence of an indefinite seed (many more seed
                            iterations on large random fields); the FP64 check after
                            the solve reports the accuracy reached                  */
       SSCG_MIXED_SHIFTS = 2 }; /* FP64 seed CG throughout; after the switch the
                            shift vectors x_j, p_j are kept in FP32 and folded into
                            the FP64 solutions every ru_interval iterations        */

enum { SSCG_PATH_LINES = 0, SSCG_PATH_CIRCLE = 1 };
enum { SSCG_RR = 0, SSCG_HANKEL = 1 };

/* Create a context for one lattice on HIP device `device`, using `hip_stream`
 * (a hipStream_t, or NULL for the default stream). dims: host int32[4].
 * kappa: hopping parameter (Sec. 4); r: Wilson parameter, must be 1.
 * Returns SSCG_EINVAL for non-positive dims or r != 1. */
int sscg_create(sscg_ctx **out, const int32_t dims[4], double kappa, double r,
                int32_t device, void *hip_stream);
void sscg_destroy(sscg_ctx *ctx);
const char *sscg_last_error(const sscg_ctx *ctx);
/* Library-wide message for failures before a context exists (sscg_create). */
const char *sscg_global_error(void);

/* Set the gauge links: U host complex128 [4][V][3][3] (copied). link_reals = 18
 * stores full 3x3 links; 12 stores the first two rows and rebuilds the third as
 * the conjugated cross product of the first two on load (valid for SU(3) only;
 * applies to the FP32 arithmetic of SSCG_MIXED; FP64 always keeps 18). */
int sscg_set_gauge(sscg_ctx *ctx, const double *U, int32_t link_reals);

/* y = A x for nsrc spinors (Sec. 4; the matrix whose eigenpairs are sought, Sec. 2.1).
 * x, y: device complex128 canonical [nsrc][V][4][3]; must not overlap.
 * prec SSCG_FP64 computes in FP64; SSCG_MIXED rounds x and the links to FP32,
 * applies A in FP32 and widens the result. Stream-ordered. */
int sscg_apply_A(sscg_ctx *ctx, const void *x, void *y, int32_t nsrc, int32_t prec);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): sscg_apply_A with the same
 * arguments, layout and result, but no device allocation and no launch-shape timing.
 * The planar staging of x and y lives in one library-wide device array of 32 MiB per
 * device (held until the process ends): nsrc * 12 V may be at most 1048576 (FP64) or
 * 2097152 (FP32), else SSCG_EINVAL. It uses the launch shape sscg_apply_A tuned for
 * (prec, nsrc) on this context if there is one, else the default shape (results then
 * agree with sscg_apply_A to rounding). Every call on a device shares that device's
 * array: calls that overlap in time on one device (other streams, other contexts,
 * other host threads) race and must be ordered by the caller. Stream-ordered. */
int sscg_apply_A_noalloc(sscg_ctx *ctx, const void *x, void *y, int32_t nsrc, int32_t prec);

typedef struct {
  double tol;            /* per-shift stop: ||r_j|| <= tol ||v|| (Sec. 4 criterion)   */
  int32_t maxiter;       /* seed iterations at most                                    */
  int32_t prec;          /* SSCG_FP64 | SSCG_MIXED | SSCG_MIXED_SHIFTS                 */
  int32_t ru_interval;   /* MIXED: reliable update every this many FP32 iterations    */
  int32_t poll_every;    /* host checks the device "all converged" word this often    */
  double switch_tol;     /* MIXED: FP64 -> FP32 switch when max active ||r_j||/||v||
                            is below this                                              */
  int32_t use_graph;     /* 1: replay the iterations between polls as a HIP graph;
                            the graphs stay in the context, and a later solve whose
                            launches are the same (shapes, buffers, options) replays
                            them without capturing again                            */
  int32_t pad;
  double true_factor;    /* MIXED and MIXED_SHIFTS: after the solve every shift's
                            FP64 true residual ||v - (z_j I - A) y_j|| / ||v|| is
                            recomputed (FP32 updates can leave it above the implicit
                            residual that froze the shift); if one exceeds
                            true_factor * tol (times the shift's own tolerance
                            multiplier, see weighted_tol) the solve returns
                            SSCG_EINACCURATE with every output written. 0: the
                            residuals are still computed and reported, no status   */
} sscg_solve_opts;

/* Default options: tol 1e-12, maxiter 100000, FP64, ru 50, poll 50, switch 1e-6, graph 1,
 * true_factor 100. */
void sscg_default_opts(sscg_solve_opts *o);

/* Shifted CG (Sec. 2.2, eqs. 4-5): solves (z_j I - A) y_{l,j} = v_l for every
 * shift j < nshift and source l < nsrc from the single Hermitian seed system
 * (sigma_seed I - A) x = v_l with a real seed shift (one product with A per
 * iteration and source serves all shifts). Converged shifts are frozen. The shifted
 * iterates do not depend on sigma_seed in exact arithmetic; a seed outside the
 * spectrum (sigma_seed > 1 + 8 kappa) never grows its residual and leaves smaller
 * FP64 rounding gaps than a seed at the centre, in the same iterations.
 *   v          device complex128 [nsrc][n] canonical
 *   z          host complex128 [nshift] (interleaved re, im)
 *   y          device complex128 [nsrc][nshift][n] canonical (output; also used as
 *              the solver's accumulator storage during the call)
 *   conv_iter  host int32 [nsrc][nshift] (output, may be NULL): iteration after
 *              which the shift met the tolerance, -1 if it never did
 *   true_res   host double [nsrc][nshift] (output, may be NULL):
 *              ||v_l - (z_j I - A) y_{l,j}|| / ||v_l|| recomputed in FP64
 *   iters      host int32 [nsrc] (output, may be NULL): seed iterations per source
 * Returns SSCG_ENOTCONV if some shift did not converge within maxiter (outputs are
 * still written), SSCG_EINACCURATE if a mixed-precision solve left some true
 * residual above true_factor * tol (outputs written; true_res, when given, names the
 * shifts), SSCG_EBREAKDOWN on a CG breakdown, SSCG_EINVAL for a zero or non-finite
 * source. Blocking. */
int sscg_shifted_cg_solve(sscg_ctx *ctx, const void *v, int32_t nsrc,
                          const double *z, int32_t nshift, double sigma_seed,
                          const sscg_solve_opts *opts, void *y, int32_t *conv_iter,
                          double *true_res, int32_t *iters);

/* Moment sums eq. (2): s_{l,k} = sum_j c[k][j] y_{l,j} for k < nmom, with
 * c[k][j] = w_j zeta_j^k supplied by the caller (host complex128 [nmom][nshift]).
 * y device complex128 [nsrc][nshift][n]; s device complex128 [nsrc][nmom][n].
 * Any layout of the n entries works as long as y and s agree. Stream-ordered. */
int sscg_ss_moments(sscg_ctx *ctx, const void *y, int32_t nsrc, int32_t nshift,
                    const double *c, int32_t nmom, void *s);

typedef struct {
  double gamma, rho, beta;  /* interval centre and half-width, line offset (Sec. 3) */
  int32_t N;                /* quadrature points                                    */
  int32_t M;                /* moments per source                                   */
  int32_t Nprime;           /* acceptance rectangle: the Nprime nodes nearest gamma
                               (Sec. 3); 0 = N                                       */
  int32_t path;             /* SSCG_PATH_LINES | SSCG_PATH_CIRCLE                   */
  int32_t method;           /* SSCG_RR (Rayleigh-Ritz) | SSCG_HANKEL (Sec. 2.1)      */
  double rank_tol;          /* numerical rank: keep singular values > rank_tol*max  */
  double spur_tol;          /* report pairs with ||A x - lambda x|| <= spur_tol      */
  sscg_solve_opts solve;
  int32_t npairs;           /* lines path: number of adjacent line pairs (Sec. 3, end):
                               pair p+1 is pair p moved by the N'-2 nodes of its
                               acceptance rectangle, the pairs are centred on gamma
                               as a group and share nodes, all distinct nodes are
                               solved by one shifted CG; 1 = a single pair         */
  int32_t moments_in_loop;  /* 1: accumulate the moments of eq. (2) inside the solve:
                               each shift's step alpha_j p_j is added to every
                               s_k = sum_j w_j zeta_j^k y_j as it is made, so the
                               solutions y_j are never stored (one fewer vector
                               read and write per shift and iteration; the shift
                               scalars and coefficients of an iteration are formed
                               once into a small device table). Rayleigh-
                               Ritz sums M moments per pair, Hankel 2M (its block
                               moments V^H s_k run to k = 2M - 1); needs npairs
                               times that <= 32, a solve precision of SSCG_FP64
                               or SSCG_MIXED_SHIFTS and 12 V < 2^27 (vectors under
                               2 GiB), else SSCG_EINVAL. The shift directions are
                               stored in 64-entry chunks per (source, shift).
                               Block form (the default, block length B = 24): the
                               recurrences of B iterations are composed into one
                               linear map per shift, p_j(B) = C_j p_j(0) +
                               sum_m D_jm r(m) with the seed residuals r(m) of the
                               block (kept in a ring of B vectors per source), and
                               the moments gain sum_j G_kj p_j(0) + sum_m H_km r(m),
                               so the directions are read and written once per B
                               iterations; a block cut short by the iteration limit
                               is applied after the loop. The poll interval is
                               rounded up to a multiple of B. 0: solutions stored,
                               moments after the solve.                             */
  int32_t weighted_tol;     /* 1: shift j stops at tol * m / m_j, where m_j is the
                               largest |w_j zeta_j^k| over the moments (and pairs)
                               it enters and m the largest m_j: every shift's
                               contribution to the moments then carries at most the
                               error of the largest-weight shift at tol. 0: one tol */
  int32_t seed_mode;        /* seed shift sigma of the shifted CG: 0 or 1 = gamma, the
                               interval centre (Sec. 4 uses the centre); 2 = outside
                               the spectrum, sigma = 1 + 8 kappa + 0.25 (|A| <= 1 + 8
                               kappa), so sigma I - A is positive definite. The shifted
                               iterates do not depend on sigma in exact arithmetic (the
                               Krylov space is the same) and the shifts converge in the
                               same iterations; with the seed at the centre CG passes
                               near-breakdowns where ||r|| grows by orders of magnitude,
                               which leaves an FP64 rounding gap of about 1e-11 in the
                               true residuals, while a definite seed keeps ||r|| <= ||v||
                               and the true residuals at the tolerance. (SSCG_MIXED
                               does not converge with a definite seed.)               */
} sscg_ss_params;

typedef struct {
  int32_t rank;             /* dimension of the extraction subspace                 */
  int32_t n_candidates;     /* Ritz / Hankel values before acceptance               */
  int32_t iters;            /* max seed iterations over sources                     */
  int32_t solve_status;     /* status of the shifted-CG stage                       */
  double t_solve, t_moments, t_extract;  /* seconds                                 */
  int64_t shift_updates;    /* (source, shift) vector updates summed over iterations */
  int64_t matvecs;          /* applications of A to one vector (solve + extraction)  */
  int64_t shift_updates_fp32; /* of shift_updates, those made in the FP32 phase       */
  int64_t seed_iters;       /* seed iterations summed over sources                   */
  int64_t seed_iters_fp32;  /* of seed_iters, those made in the FP32 phase           */
  int32_t switch_iter;      /* iteration at which the FP32 phase began, -1 if never  */
  int32_t pad;
  double max_true_res;      /* largest FP64 true residual ||v - (z_j I - A) y_j||/||v||
                               over every node and source, recomputed after a
                               mixed-precision solve with stored solutions; -1 when
                               not computed (FP64 solves, moments in the loop)       */
  int64_t extract_bytes;    /* device memory the extraction stage works in beyond the
                               solve's: moment vectors, bases, products and vectors  */
} sscg_ss_info;

void sscg_default_ss_params(sscg_ss_params *p);

/* Eigenpairs of A in [gamma - rho, gamma + rho] (Sec. 2-3): line (or circle)
 * quadrature, shifted CG for all nodes, moments eq. (2), Rayleigh-Ritz or block
 * Hankel extraction (Sec. 2.1, block form with nsrc sources), then the acceptance
 * rectangle of Sec. 3 and the residual filter res <= spur_tol. With npairs > 1 the
 * interval is covered by adjacent line pairs that reuse nodes (Sec. 3): one shifted
 * CG over the N + (npairs - 1)(N' - 2) distinct nodes, then moments, extraction and
 * acceptance per pair (each pair's rectangle is half-open on the right except the
 * last, so an eigenvalue on a shared edge is reported once).
 *   v       device complex128 [nsrc][n] canonical sources
 *   lambda  host double [max_eigs] (output, ascending)
 *   X       device complex128 [max_eigs][n] canonical unit eigenvectors, or NULL
 *   res     host double [max_eigs]: ||A x - lambda x||_2 (output)
 *   n_found host int32 (output): pairs accepted; if more than max_eigs qualify,
 *           the max_eigs nearest gamma are returned and n_found is the full count
 *   info    host (output, may be NULL)
 * Returns SSCG_OK, or SSCG_ENOTCONV / SSCG_EINACCURATE from the solve stage with the
 * extraction still done and every output written. Blocking. */
int sscg_ss_eigs(sscg_ctx *ctx, const sscg_ss_params *p, const void *v, int32_t nsrc,
                 int32_t max_eigs, double *lambda, void *X, double *res,
                 int32_t *n_found, sscg_ss_info *info);

/* Quadrature on the two horizontal lines z = gamma + rho (x +- i beta), -1 <= x <= 1
 * (Sec. 3): N/2 equally spaced points per line with both ends included, even j on
 * the upper line; weights solve sum_j w_j zeta_j^(k-1) = delta_k0, k < N.
 * Outputs host complex128 [N] each (z, zeta = (z - gamma)/rho, w). N even, >= 4. */
int sscg_quad_lines(int32_t N, double gamma, double rho, double beta,
                    double *z, double *zeta, double *w);
/* Circle of centre gamma, radius rho (Sec. 2.1): z_j = gamma + rho e^{2 pi i (j+1/2)/N},
 * dimensionless weights w_j = zeta_j / N. */
int sscg_quad_circle(int32_t N, double gamma, double rho, double *z, double *zeta, double *w);

/* Several independent problems (own lattice, gauge, sources, shifts, seed) solved
 * together: every stage of every iteration is one grouped kernel launch covering
 * all problems, and the iterations between polls replay as one HIP graph.
 * Arrays of length nprob; entry i has the meaning of the same argument of
 * sscg_shifted_cg_solve for context ctxs[i] (all contexts on one device and
 * stream; opts shared, prec applies to all). Each problem's result equals its
 * own sscg_shifted_cg_solve run with the same options. Blocking. */
int sscg_batch_solve(sscg_ctx *const *ctxs, int32_t nprob, const void *const *v,
                     const int32_t *nsrc, const double *const *z, const int32_t *nshift,
                     const double *sigma_seed, const sscg_solve_opts *opts,
                     void *const *y, int32_t *const *conv_iter, double *const *true_res,
                     int32_t *const *iters);

/* Eigen-decomposition of a small Hermitian matrix (host, FP64: Householder reduction
 * to a real symmetric tridiagonal matrix, then implicit symmetric QR steps with
 * Wilkinson shifts), the dense step of the Rayleigh-Ritz and Hankel extraction
 * (Sec. 2.1).
 *   A      host complex128 n x n, column-major (element (i, j) at 2 (i + n j)); read only
 *   evals  host double [n] (output, ascending)
 *   evecs  host complex128 n x n column-major (output, column k = unit eigenvector k),
 *          or NULL
 * Only the Hermitian part of A is used. Needs no device. Returns SSCG_ENOTCONV if the
 * QR iteration does not converge within 30 n + 30 steps (outputs undefined); the
 * extraction in sscg_ss_eigs returns the same status in that case. */
int sscg_herm_eig(int32_t n, const double *A, double *evals, double *evecs);

/* Per-stage timing of the last solve on this context, from HIP events on the
 * context's stream, in milliseconds summed over the solve; counts in calls.
 * stage: 0 dslash, 1 seed alpha scalars, 2 seed residual update, 3 (not used: the
 * shift scalars are formed inside the shift update), 4 fused shift update (block form:
 * the table of the iteration and the seed direction update), 5 reliable update, 6
 * whole iteration loop (wall clock; its count is the iterations launched), 7 block
 * sweep of the block form (composition, moment and direction kernels).
 * Timing is recorded only when enabled with sscg_set_profiling(ctx, level):
 *   level 0  off (the default);
 *   level 1  every launch of the solve loop is bracketed by events, and the loop runs
 *            its launches directly (no graph replay);
 *   level k > 1  graph replay stays on, and every stage of the iterations i of each
 *            poll interval with i % k == k / 2 is bracketed by event-record nodes in the
 *            graph, as is every reliable update (stage 5, on the last iteration of an
 *            FP32 chunk); in the block form (length B) the sampled iterations are the
 *            last of every q-th block, q = max(1, k / B) (so the sweep is timed too). Stage averages are then over that sample, at a small cost
 *            to the loop; sscg_stage_launches gives the launches to scale them by.
 * A level below 0 is SSCG_EINVAL. When timing is on, sscg_apply_A also adds its dslash
 * time to stage 0 (and blocks until it ends). */
int sscg_set_profiling(sscg_ctx *ctx, int32_t level);
int sscg_stage_times(const sscg_ctx *ctx, double ms[8], int64_t calls[8]);
/* Launches of each stage (indices as above) in the last solve on this context that did
 * work, counted whether or not they were timed: those of the iterations in which a
 * source still iterated (stage 7: the sweeps of blocks holding such iterations); the
 * launches after the last source finished (up to the next poll) exit at once, and
 * timing samples taken there are not counted in sscg_stage_times either. Stage 6 holds
 * the iterations launched. A stage's time in the solve is ms[k] / calls[k] *
 * launched[k]. */
int sscg_stage_launches(const sscg_ctx *ctx, int64_t launched[8]);
/* Algorithmic HBM bytes moved by the block sweeps (stage 7: the moment and direction
 * kernels of the block form of the in-loop moment update) in the last solve on this
 * context: per (source, block) the moment kernel reads the directions of the shifts
 * updated in the block, the block's B residuals and the M moment sums and writes the
 * sums; the direction kernel (run if a shift is still active) reads the same
 * directions and the residuals and writes the active directions; 16 bytes per FP64
 * entry, 8 per FP32 direction entry. 0 for the per-iteration form and stored
 * solutions. Stage 7 of sscg_stage_times / sscg_stage_launches times the sweeps. */
int sscg_sweep_bytes(const sscg_ctx *ctx, int64_t *bytes);

#ifdef __cplusplus
}
#endif
#endif /* SSCG_H */
