/*
 * rp.h -- C ABI of librpfit, the MI355X (gfx950) library for the data-parallel
 * hot path of the rational-program technique for choosing program launch
 * parameters:
 *
 *   1. rational-function estimation (Section 3.3, step 2; Section 4.2): fit
 *      f = N/Q to sampled low-level metrics by linearised least squares,
 *      minimising sum_i (N(u_i) - y_i Q(u_i))^2 with Q's constant term fixed
 *      at 1, so that the problem is linear in the coefficients (Ax = b);
 *   2. rational-program evaluation and selection (Section 3.3, steps 4-5;
 *      Section 4.3): evaluate the program at a data size for every candidate
 *      launch configuration of the finite set F and keep the minimiser.
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Pointers: arguments documented "device" are device pointers on the device of
 *   the rp_ctx, owned by the caller; the library never frees them.  "host"
 *   arrays are read during the call only (plans and programs copy what they
 *   keep).
 * Streams: device work is enqueued on `stream` (a hipStream_t; NULL = the
 *   default stream) and the call returns without waiting for it.  Entry points
 *   taking a plan or a program allocate nothing: the plan/program owns the
 *   device workspace it needs, sized when it was created.  Calls that share a
 *   plan or program must not overlap on different streams.
 * Errors: every entry point returns RP_OK (0) or a negative RP_E* code; the
 *   message of the calling thread's last failure is rp_last_error().  An
 *   argument error is detected before anything is enqueued.  Numerical trouble
 *   in a fit is not an API error: it is reported per fit in `status`.
 * Monomial order: the exponents of total degree <= d in v variables, graded
 *   (total degree ascending), and within one degree the exponent of x1
 *   descending, then of x2 descending, and so on; the constant is index 0.
 * Coefficients of one model: [alpha_0 .. alpha_{a-1} | beta_1 .. beta_b] with
 *   a = C(v+dn, dn) numerator terms and b = C(v+dq, dq) - 1 denominator terms;
 *   beta_0 = 1 is implicit (the normalisation of the linearised problem).
 */
#ifndef RP_H
#define RP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* rp_stream_t;   /* the same type as hipStream_t */

/* return codes */
#define RP_OK            0
#define RP_EINVAL       -1   /* bad argument value or NULL pointer            */
#define RP_ESHAPE       -2   /* inconsistent sizes or offsets                 */
#define RP_EHIP         -3   /* a HIP runtime call failed                     */
#define RP_ENOMEM       -4   /* device or host allocation failed              */
#define RP_EUNSUPPORTED -5   /* model shape or option not compiled in         */

/* per-fit status */
#define RP_FIT_OK               0
#define RP_FIT_RANK_DEFICIENT   1   /* a design column is dependent (see
                                       rp_fit_rational: numerical rank)     */
#define RP_FIT_UNDERDETERMINED  2   /* fewer samples than unknowns              */
#define RP_FIT_NONFINITE_INPUT  3   /* a sample was NaN or infinite             */
#define RP_FIT_Q_NONPOSITIVE    4   /* fitted Q(u_i) <= 0 at some sample         */
#define RP_FIT_NOT_CONVERGED    5   /* refinement stopped at its iteration cap  */

/* arithmetic forms of the fit */
#define RP_FP64        0   /* FP64 design and Gram, FP64 solve, FP64 refinement  */
#define RP_MIXED_FP32  1   /* FP32 design, FP32 MFMA Gram, FP64 solve + PCG      */
#define RP_MIXED_BF16  2   /* BF16 design, BF16 MFMA Gram (FP32 accumulate),
                              FP64 solve + PCG                                   */
#define RP_AUTO        3   /* per shape bucket, the form rp_plan_tune measured
                              fastest (RP_FP64 with the moment Gram before any
                              tuning); rp_fit_rational and rp_fit_graph_create */

/* how the FP64 Gram is formed */
#define RP_GRAM_AUTO     0   /* the library's choice per shape (weighted moments)   */
#define RP_GRAM_MFMA     1   /* design tiles in LDS contracted on FP64 MFMA          */
#define RP_GRAM_MOMENTS  2   /* weighted moments of degree <= 2d on FP64 VALU: each
                                Gram entry of a monomial design is such a moment    */

/* program templates */
#define RP_TEMPLATE_SINGLE  0   /* E = one rational g_1                            */
#define RP_TEMPLATE_MWPCWP  1   /* E = MWP-CWP-style cycles from 16 metric rationals */
#define RP_TEMPLATE_OCCUPANCY 2 /* E = hardware occupancy from 2 metric rationals    */

/* selection sense */
#define RP_SELECT_MIN   1      /* the smallest E wins (a time, a cycle count)      */
#define RP_SELECT_MAX  (-1)    /* the largest E wins (an occupancy)                */

#define RP_NUM_METRICS 16      /* metric slots of RP_TEMPLATE_MWPCWP              */
#define RP_HW_COUNT    17      /* entries of the hardware vector                  */

/* Message of the calling thread's last failing call ("" if none). */
const char* rp_last_error(void);

/* ------------------------------------------------------------------------ */
/* Host tables (Section 4.2 model display; Section 3.3 finite set F)          */
/* ------------------------------------------------------------------------ */

/* Exponents of the monomials of total degree <= degree in nvars variables, in
 * the monomial order above, as count rows of nvars bytes.  exps may be NULL to
 * query *count.  1 <= nvars <= 8, 0 <= degree <= 15; else RP_EINVAL. */
int rp_monomials(int nvars, int degree, uint8_t* exps, int* count);

/* The per-variable degree box of the Section 4.2 model display (each
 * variable's degree bounded on its own): every exponent e with
 * 0 <= e_k <= maxdeg[k] (host, nvars entries), in the monomial order above,
 * as count rows of nvars bytes; exps may be NULL to query *count (the
 * product of maxdeg[k] + 1).  1 <= nvars <= 8, 0 <= maxdeg[k] <= 15; else
 * RP_EINVAL.  A host table: the fit kernels take total-degree models. */
int rp_monomials_box(int nvars, const int32_t* maxdeg, uint8_t* exps, int* count);

/* Number of unknowns a + b of a model (see "Coefficients" above). */
int rp_num_coefs(int nvars, int deg_num, int deg_den, int* count);

/* The candidate set of 2-D block formats: every integer pair (bx, by) >= 1 with
 * bx*by <= max_prod and bx*by a multiple of `multiple`, ordered by bx then by
 * (Section 3.3: F is finite and program parameters may depend on each other;
 * Section 4: threads per block are bounded).  bxby (host, count*2 int32) may
 * be NULL to query *count. */
int rp_candidates_2d(int max_prod, int multiple, int32_t* bxby, int* count);

/* ------------------------------------------------------------------------ */
/* Context and fit plans                                                     */
/* ------------------------------------------------------------------------ */

typedef struct rp_ctx_s* rp_ctx;
typedef struct rp_plan_s* rp_plan;

/* Bind a context to HIP device `device`.  Fails with RP_EHIP if it is absent. */
int rp_create(rp_ctx* out, int device);
int rp_destroy(rp_ctx ctx);

/* A plan for an uneven batch of num_fits fits.  Host arrays (copied):
 *   sample_off[num_fits+1]  prefix sums; fit f owns global samples
 *                           [sample_off[f], sample_off[f+1])
 *   nvars, deg_num, deg_den [num_fits]
 * Compiled shapes: 1 <= nvars <= 4 and deg_num == deg_den in 1..4; any other
 * shape gives RP_EUNSUPPORTED.  A fit holds fewer than 2^28 samples (else
 * RP_ESHAPE).  The plan uploads its metadata, buckets fits by
 * shape, orders each bucket by decreasing cost and allocates its workspace. */
int rp_plan_create(rp_ctx ctx, int num_fits, const int64_t* sample_off,
                   const int32_t* nvars, const int32_t* deg_num,
                   const int32_t* deg_den, rp_plan* out);
int rp_plan_destroy(rp_plan plan);

/* Host copies of the plan's offsets, each [num_fits+1]: coef_off (fit f owns
 * coef[coef_off[f] .. coef_off[f+1])), a_off (fit f's design rows start at
 * element a_off[f] in rp_assemble_design) and gram_off (fit f's packed Gram
 * starts at element gram_off[f] in rp_gram).  Any pointer may be NULL. */
int rp_plan_offsets(rp_plan plan, int64_t* coef_off, int64_t* a_off, int64_t* gram_off);

typedef struct {
    int32_t precision;    /* RP_FP64, RP_MIXED_FP32, RP_MIXED_BF16 or RP_AUTO    */
    int32_t max_refine;   /* FP64: iterative-refinement steps (default 1);
                             mixed: preconditioned CG iterations (default 12
                             for RP_MIXED_FP32, 40 for RP_MIXED_BF16; a fit
                             whose observed rate cannot reach the bar by the
                             cap stops early); a fit left at the cap is
                             re-solved in FP64 (see rp_fit_rational)          */
    double  tol;          /* stop refining once the correction's max-norm is
                             <= tol * max|coef| (default 1e-13 for RP_FP64,
                             1e-12 for the mixed forms, whose CG corrections
                             can understate the error of an ill-conditioned
                             fit by a few orders)                              */
    int32_t check_q;      /* nonzero: flag RP_FIT_Q_NONPOSITIVE and compute the
                             final residual norm (FP64 form with refinement:
                             from the last refinement pass; otherwise one more
                             pass over the samples)                             */
    int32_t gram_algo;    /* RP_GRAM_AUTO, RP_GRAM_MFMA or RP_GRAM_MOMENTS (FP64
                             form and the refinement's Jacobian Gram)            */
} rp_fit_opts;

/* Materialise the linearised design (Section 4.2, Ax = b): for fit f and its
 * i-th sample, row i of A_f is [m_j(u_i)]_{j<a} ++ [-y_i m'_j(u_i)]_{1<=j<=b}
 * and b_f[i] = y_i.  Device inputs: x[k*ld_x + s] is variable k of global
 * sample s (k < nvars of its fit), y[s].  Outputs (device): A, row-major per
 * fit starting at element a_off[f]; rhs[s] at the global sample index.
 * precision selects the element type of A and rhs: RP_FP64 double, RP_MIXED_FP32
 * float, RP_MIXED_BF16 bfloat16 (round to nearest even). */
int rp_assemble_design(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                       int precision, void* A, void* rhs, rp_stream_t stream);

/* Batched augmented Gram of the linearised problems (Section 4.2: the normal
 * equations of A x = b): for fit f, the packed lower triangle of
 * [A_f b_f]^T [A_f b_f] in FP64, (nc+1)(nc+2)/2 entries starting at element
 * gram_off[f] of `gram` (device).  Entry (i, j), j <= i, sits at
 * i(i+1)/2 + j; index nc is the rhs column, so row nc holds A^T b and entry
 * (nc, nc) is b^T b.  precision selects the products: RP_FP64 (formed as
 * gram_algo says), RP_MIXED_FP32 on FP32 MFMA, RP_MIXED_BF16 on BF16 MFMA
 * (FP32 accumulation); the design rows are assembled on chip and never
 * stored.  Non-finite samples propagate into the fit's entries. */
int rp_gram(rp_plan plan, const double* x, int64_t ld_x, const double* y, int precision,
            int gram_algo, double* gram, rp_stream_t stream);

/* Batched Jacobian Gram of the true loss sum_i (N/Q - y)^2 at given
 * coefficients: the Gauss-Newton normal equations of a refinement of the
 * fitted rationals on their true loss.  This refinement is this library's
 * addition, not a step of the paper (whose fit stops at the linearised least
 * squares of Section 4.2).  For fit f with coefficients
 * coef[coef_off[f] ..] (device, FP64, read only), the packed lower triangle of
 * [J r]^T [J r] with row i of J equal to (1/Q(u_i)) [m(u_i), -f(u_i) m'(u_i)],
 * f = N/Q, and r_i = y_i - f(u_i); layout as for rp_gram (entry (nc, nc) is
 * the loss).  FP64; gram_algo as for rp_gram.  Non-finite samples or a
 * vanishing Q propagate into the fit's entries. */
int rp_gram_jacobian(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                     const double* coef, int gram_algo, double* gram, rp_stream_t stream);

/* Fit every model of the plan by linearised least squares (Section 3.3 step 2,
 * Section 4.2).  Inputs as for rp_assemble_design.  opts may be NULL for the
 * defaults.  Outputs (device): coef[coef_off[num_fits]] FP64; status[num_fits];
 * resid[num_fits] = ||b - A c|| (NaN when opts->check_q == 0); iters[num_fits]
 * = refinement steps taken.  A fit flagged RP_FIT_RANK_DEFICIENT or
 * RP_FIT_UNDERDETERMINED gets the least-squares minimiser of smallest norm
 * (the SVD's answer, Section 4.2), computed in FP64 after the fit: from the
 * m x m sample Gram A A^T when m < unknowns, else by projecting the basic
 * solution onto the row space of A.  A fit whose refinement reached its step
 * cap (any form) is re-solved the same way in FP64 with up to 10 refinement
 * steps before its status is final.  resid and iters then describe that
 * solve.  The mixed forms flag underdetermined fits only among the
 * rank-related statuses (their shifted factorisation keeps every pivot).
 * Numerical rank (the paper's SVD solve needs a tolerance and names none):
 * taking the unknowns in coefficient order, a design column whose distance
 * from the span of the columns kept before it is at most 1e-5 of its own norm
 * is dependent (the sweep compares each pivot of the equilibrated Gram with
 * 1e-10 times its diagonal); dependent columns are replaced by their
 * projections onto the kept ones for the minimum-norm solve.  With fewer
 * samples than unknowns, the unique minimum-norm interpolant is returned
 * unless a sample's design row lies within sqrt(1e-13) of its norm from the
 * span of the rows before it, in which case the column rule decides. */
int rp_fit_rational(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                    const rp_fit_opts* opts, double* coef, int32_t* status,
                    double* resid, int32_t* iters, rp_stream_t stream);

/* Autotuning of a plan (this library's addition; the paper fits one metric
 * at a time on the host, Section 4.2).  For every shape bucket, time the
 * bucket's whole fit (rp_fit_rational with default options on these inputs)
 * in each candidate form -- RP_FP64 with the Gram by weighted moments, RP_FP64
 * with the Gram on MFMA tiles, RP_MIXED_FP32, RP_MIXED_BF16 -- with HIP events
 * (one warm-up and two timed launches each), and keep the fastest: RP_AUTO
 * then fits the bucket in that form, and RP_GRAM_AUTO uses the faster FP64
 * Gram (before tuning: RP_FP64 with moments).  Allocates scratch outputs for
 * the timing runs and synchronises `stream`.
 * The table has RP_TUNE_COLS int32 columns per bucket: nvars, deg_num,
 * deg_den, the chosen precision, the chosen FP64 gram_algo, then the measured
 * microseconds of the four candidates in the order above (-1: not measured);
 * count = buckets.  rp_plan_set_tuning restores the choices (columns 0-4) of
 * a persisted table; rows whose shape is not in the plan are ignored. */
#define RP_TUNE_COLS 9
int rp_plan_tune(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                 rp_stream_t stream);
int rp_plan_tuning(rp_plan plan, int32_t* table /* [count*RP_TUNE_COLS] or NULL */, int* count);
int rp_plan_set_tuning(rp_plan plan, const int32_t* table, int count);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * fit of rp_fit_rational with default options for a uniform batch -- num_fits
 * fits of one shape (nvars, degree/degree), fit f owning the global samples
 * [f*num_samples, (f+1)*num_samples) and the coefficients
 * [f*nc, (f+1)*nc), nc = rp_num_coefs(nvars, degree, degree) -- with no plan
 * and no allocation.  The scratch the fit needs (per-fit offsets, the packed
 * Gram workspace, flags, the re-solve list, the moment map) lives in one
 * device array of 32 MiB per GPU, set up by rp_create: a batch needing more
 * (about 5000 fits of degree 3/3 in three variables, 420 of degree 4/4 in
 * four) fails with RP_ESHAPE before anything is enqueued.  Inputs as for
 * rp_fit_rational (x[k*ld_x + s], ld_x >= num_fits*num_samples); outputs
 * (device) coef, status, resid and iters (iters may be NULL), identical to
 * rp_fit_rational's on a plan of the same batch.  Every call on one GPU
 * shares that GPU's scratch and re-initialises what it reads: calls that
 * overlap on one GPU (different streams or threads) race and must not be
 * issued. */
int rp_fit_uniform_static(rp_ctx ctx, int num_fits, int num_samples, int nvars, int degree,
                          const double* x, int64_t ld_x, const double* y, double* coef,
                          int32_t* status, double* resid, int32_t* iters, rp_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Decision nodes fitted from the samples (Section 3.2, third consequence)    */
/* ------------------------------------------------------------------------ */

typedef struct rp_split_s* rp_split;

/* A rational program's decision nodes are rational functions too, so they can
 * be fitted like its process nodes (Section 3.2, third consequence).  This
 * fits the simplest such node: a threshold on one variable with a rational of
 * degree `degree`/`degree` on each side, y = f_L(u) where u_s <= theta and
 * f_R(u) elsewhere (s = split_var), for num_nodes independent nodes of
 * num_samples samples each (node f owns the global samples
 * [f*num_samples, (f+1)*num_samples); 0 <= num_samples <= 4096).  Exhaustive
 * search: in the order of ascending u_s (equal values by sample index),
 * every split after the k-th sample with n_min <= k <= num_samples - n_min
 * that does not separate equal values of u_s is a candidate; both sides are
 * fitted by the linearised least squares of rp_fit_rational (FP64, default
 * options); the candidate with the smallest sum of the two sides' squared
 * residual norms wins, the smallest k on exact ties; theta = (u_s of sorted
 * sample k-1 + u_s of sorted sample k) / 2.  n_min >= the model's unknowns
 * keeps both sides determined.  rp_split_create allocates the workspace:
 * the sorted samples once per candidate, (nvars + 1) * 8 * num_nodes *
 * candidates * num_samples bytes, plus an internal fit plan of two fits per
 * candidate. */
int rp_split_create(rp_ctx ctx, int num_nodes, int num_samples, int nvars, int degree,
                    int split_var, int n_min, rp_split* out);
int rp_split_destroy(rp_split split);

/* Fit every node.  Inputs (device) x[k*ld_x + s], y[s] as for
 * rp_fit_rational (ld_x >= num_nodes*num_samples).  Outputs (device, per node
 * f): k[f] = the winning split (samples on the left; -1 when no candidate is
 * admissible or a sample is not finite), theta[f], coef_l and coef_r
 * (unknowns per node each, the layout of rp_fit_rational; NaN when k = -1),
 * status_l / status_r (the two fits' statuses; RP_FIT_NONFINITE_INPUT for a
 * non-finite sample, RP_FIT_UNDERDETERMINED when there is no candidate) and
 * obj[f] (the winning summed squared residual; +inf when k = -1). */
int rp_split_fit(rp_split split, const double* x, int64_t ld_x, const double* y, int64_t* k,
                 double* theta, double* coef_l, double* coef_r, int32_t* status_l,
                 int32_t* status_r, double* obj, rp_stream_t stream);

typedef struct rp_graph_s* rp_graph;

/* The whole fit of a plan (rp_fit_rational with these buffers and options),
 * every shape bucket's kernels as an independent branch, captured once into a
 * HIP graph and replayed by rp_graph_launch as one launch on `stream`.  The
 * buffers must stay valid while the graph is used; the graph owns its capture
 * streams.  The replay allocates nothing. */
int rp_fit_graph_create(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                        const rp_fit_opts* opts, double* coef, int32_t* status,
                        double* resid, int32_t* iters, rp_graph* out);
int rp_graph_launch(rp_graph graph, rp_stream_t stream);
int rp_graph_destroy(rp_graph graph);

typedef struct {
    int32_t max_iter;     /* Gauss-Newton / Levenberg-Marquardt steps (default 20) */
    double  rtol;         /* stop when a step lowers the loss by <= rtol * loss
                             (default 1e-14)                                      */
    int32_t gram_algo;    /* RP_GRAM_AUTO, RP_GRAM_MFMA or RP_GRAM_MOMENTS          */
} rp_refine_opts;

/* Refine coef (device, in/out, FP64) on the true loss sum_i (N_i/Q_i - y_i)^2
 * by Levenberg-Marquardt steps in FP64 (this library's addition; the paper
 * stops at the linearised fit): the Jacobian row of sample i is
 * (1/Q_i)[m(u_i), -f_i m'(u_i)]; its Gram and right-hand side are formed as
 * opts->gram_algo says (RP_GRAM_AUTO: weighted moments on the FP64 vector
 * units, see rp_gram_jacobian); the damped normal equations
 * (J^T J + lambda diag(J^T J)) d = J^T r are solved by the sweep operator on
 * the equilibrated matrix in FP64; lambda starts at 0, is multiplied by 10
 * (from 1e-6) on a rejected step and divided by 10 on an accepted one.
 * Outputs: loss[num_fits] (device) = final loss; status as for
 * rp_fit_rational (RP_FIT_NOT_CONVERGED when max_iter ran out). */
int rp_refine_rational(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                       const rp_refine_opts* opts, double* coef, int32_t* status,
                       double* loss, rp_stream_t stream);

#define RP_LOSS_FWD 0
#define RP_LOSS_BWD 1

/* True loss and its adjoint in FP32, for gradient-based refinement.
 * FWD: loss[f] = sum_i (N_i/Q_i - y_i)^2 over fit f's samples.
 * BWD: dcoef = dloss[f] * dloss[f]/dcoef, i.e. for numerator terms
 *   2 dloss[f] sum_i r_i m_j(u_i)/Q_i and for denominator terms
 *   -2 dloss[f] sum_i r_i N_i/Q_i^2 m'_j(u_i), r_i = N_i/Q_i - y_i
 *   (loss is also written).  coef, dcoef follow the plan's coef_off; all
 * pointers device.  dloss/dcoef are ignored in FWD mode. */
int rp_loss_grad(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                 const float* coef, float* loss, const float* dloss, float* dcoef,
                 int mode, rp_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Rational programs (Section 2, Definition 1; Examples 1-2; Section 3.3)     */
/* ------------------------------------------------------------------------ */

typedef struct rp_prog_s* rp_prog;

/* A batch of num_programs programs, each combining num_metrics metric
 * rationals over nvars = 1 + cand_dim variables u = (n / scale[0],
 * c_0 / scale[1], ..., c_{cand_dim-1} / scale[cand_dim]): the data size n
 * first, then the candidate's program parameters.
 *   template_id  RP_TEMPLATE_SINGLE: E = g_1 (num_metrics == 1), a candidate
 *                whose Q <= 0 is infeasible;
 *                RP_TEMPLATE_MWPCWP: E = the MWP-CWP-style estimate of cycles
 *                from RP_NUM_METRICS metric rationals, the hardware vector and
 *                the block format (bx, by) = candidate (cand_dim == 2).
 *   deg_num, deg_den  host [num_programs * num_metrics]
 *   coef_off          host [num_programs * num_metrics + 1]
 *   coef              device, FP64, per metric in the layout above
 *   hw                device [num_programs * RP_HW_COUNT] or NULL (SINGLE)
 *   scale             host [nvars]
 * Metric slots (in order): comp_insts, coal_mem_insts, uncoal_mem_insts,
 * synch_insts, coal_per_mw, uncoal_per_mw, load_bytes_per_warp,
 * regs_per_thread, lds_bytes_per_block, total_blocks, sfu_insts, lds_insts,
 * lds_conflict_rate, branch_insts, l2_hit_rate, divergence_rate.
 * Hardware entries (in order): wave_size, num_cu, simd_per_cu,
 * max_threads_per_block, max_blocks_per_cu, max_waves_per_cu, regs_per_cu,
 * lds_bytes_per_cu, mem_latency, l2_latency, departure_del_coal,
 * departure_del_uncoal, issue_cycles, sfu_issue_cycles, lds_issue_cycles,
 * clock_ghz, mem_bandwidth_gbs.
 * The template (Section 2, Examples 1-2): T = bx*by; resident blocks
 * B = min(max_blocks, floor(max_waves/ceil(T/W)), floor(regs_cu/(R W ceil(T/W))),
 * floor(lds_cu/Z)); active waves N = min(floor(B T / W), max_waves) (equation
 * (occupancy)); memory and computation warp parallelism MWP, CWP from the
 * latencies, departure delays and bandwidth; cycles by the three MWP-CWP
 * cases times ceil(blocks/(B active_cu)), plus the synchronisation term.
 * E = +inf when T > max_threads_per_block or B = 0.
 *                RP_TEMPLATE_OCCUPANCY (Section 2, Example 1): E = hardware
 *                occupancy N / max_waves of the block format (bx, by) =
 *                candidate (cand_dim == 2), with B and N as above from metric
 *                0 = registers per thread and metric 1 = LDS bytes per block
 *                (num_metrics == 2) and the hardware vector; E = -inf when
 *                T > max_threads_per_block or B = 0. */
typedef struct {
    int32_t template_id;
    int32_t num_programs;
    int32_t num_metrics;
    int32_t nvars;
    const int32_t* deg_num;
    const int32_t* deg_den;
    const int64_t* coef_off;
    const double* coef;
    const double* hw;
    const double* scale;
} rp_program_desc;

int rp_program_create(rp_ctx ctx, const rp_program_desc* desc, rp_prog* out);
int rp_program_destroy(rp_prog prog);

/* Exhaustive evaluation and selection (Section 3.3, steps 4-5).  For program p
 * and data size n_grid[j]: argmin[p*num_n + j] = the candidate index with the
 * smallest finite E (lowest index on exact ties; -1 if no candidate is
 * finite), best[...] its E and second[...] the smallest E among the other
 * candidates (+inf if none).  n_grid (device, FP64 [num_n]) and cand (device,
 * int32 [num_cand * cand_dim], candidate-major) are inputs.  precision:
 * RP_FP64 evaluates in FP64; RP_MIXED_FP32 scans in FP32 and re-scores its four
 * best candidates per (p, j) in FP64 (the selection and values returned are
 * the FP64 re-scores).  values (device, FP64 [num_programs*num_n*num_cand]) may
 * be non-NULL to also receive every E (FP64 form only). */
int rp_eval_program_argmin(rp_prog prog, const double* n_grid, int num_n,
                           const int32_t* cand, int num_cand, int cand_dim,
                           int precision, int32_t* argmin, double* best,
                           double* second, double* values, rp_stream_t stream);

/* Selection with a sense and a second performance metric (Section 3.3 step 5:
 * when several configurations optimise E, a second metric refines the
 * choice).  As rp_eval_program_argmin with the order given by sense
 * (RP_SELECT_MIN or RP_SELECT_MAX; an occupancy program is maximised): choice
 * = the winning candidate (-1 if no E is finite), best = its E, second = the
 * winning-most E among the other candidates (+inf for MIN, -inf for MAX if
 * none).  tie_prog (NULL for none; RP_FP64 only) is a single-rational or
 * occupancy program with the same num_programs and nvars, evaluated at the
 * same (n, candidate): among candidates whose E equals the winner's exactly,
 * the one whose tie value wins by tie_sense is chosen (a non-finite tie value
 * ranks last), then the lowest index.  rp_eval_program_argmin is this call
 * with RP_SELECT_MIN and no tie program. */
int rp_eval_program_select(rp_prog prog, int sense, rp_prog tie_prog, int tie_sense,
                           const double* n_grid, int num_n, const int32_t* cand,
                           int num_cand, int cand_dim, int precision, int32_t* choice,
                           double* best, double* second, double* values,
                           rp_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Specialised evaluators (Section 3.3 step 3, Section 4.3: code generation)  */
/* ------------------------------------------------------------------------ */

typedef struct rp_spec_s* rp_spec;

/* The HIP source of the evaluator specialised to the programs of d (1..256
 * programs), with the coefficients, scales and hardware vectors (HOST
 * pointers in d here) written in as literals and the template code appended.
 * buf may be NULL to query *len (bytes including the terminating NUL);
 * RP_ESHAPE, with *len set, when *len is too small.  Host only. */
int rp_program_source(const rp_program_desc* d, char* buf, size_t* len);

/* Generate, compile (hipRTC, for the device of prog) and load the specialised
 * evaluator of prog's programs.  Reads prog's coefficients and hardware
 * vectors from the device once (synchronously): later changes to those arrays
 * are not seen by the evaluator.  1..256 programs.  Compile errors come back
 * as RP_EHIP with the compiler log in rp_last_error(). */
int rp_program_specialize(rp_prog prog, rp_spec* out);

/* The source an evaluator was compiled from (buf / len as above). */
int rp_spec_source(rp_spec spec, char* buf, size_t* len);

/* rp_eval_program_select with the specialised evaluator, FP64, no tie
 * program: same arguments and outputs (values optional). */
int rp_eval_spec_select(rp_spec spec, int sense, const double* n_grid, int num_n,
                        const int32_t* cand, int num_cand, int cand_dim, int32_t* choice,
                        double* best, double* second, double* values, rp_stream_t stream);

int rp_spec_destroy(rp_spec spec);

#ifdef __cplusplus
}
#endif
#endif /* RP_H */
