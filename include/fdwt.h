/*
 * fdwt.h -- C ABI of libfdwt: fast discrete Walsh transforms on digital nets
 * over Z_p, native on AMD MI355X (gfx950).
 *
 * Method: K.-I. Liu, J. Dick, F. J. Hickernell, "A Multivariate Fast Discrete
 * Walsh Transform with an Application to Function Interpolation".
 *
 * Conventions used by every call
 *   - p in {2, 3, 5, 7}; m >= 1; N = p^m <= 2^26 points; 1 <= s <= 64.
 *   - Point index n = n_0 + n_1 p + ... + n_{m-1} p^{m-1} (digit vector
 *     n_vec least significant first).  Coefficient index h = h_0 + h_1 p + ...
 *     where h_vec = C . k is the label of the coset of wavenumber k
 *     (Section 2.1); the transform leaves coefficient k at position h, as in
 *     Algorithm 1 (no digit reversal).
 *   - Buffers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *     tensors on the current device), owned by the caller; *_host pointers
 *     are host memory owned by the caller.  Coordinate-major layouts are
 *     [s][N] (all N values of coordinate 1, then coordinate 2, ...).
 *   - stream is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *     on it and return without waiting, except those that return host
 *     results (fdwt_eff_dim, fdwt_split_cost, fdwt_kernel_tune,
 *     fdwt_batch_check, fdwt_batch_autotune), which synchronise the stream.
 *   - Calls made with one net handle must be ordered on one stream (or
 *     synchronised by the caller): the handle owns a workspace they share.
 *   - Errors: every int-returning call returns FDWT_OK (0) or a negative
 *     code; fdwt_last_error() gives a message for the calling thread.  No
 *     exception crosses the ABI.  Invalid arguments are rejected before any
 *     work is enqueued.
 *   - Tuning knobs from the environment (the first two read once per
 *     process, the last two at each call): FDWT_EFFDIM_CHUNK_MB, the
 *     workspace budget of fdwt_eff_dim's kernel-data columns in MiB
 *     (default 12288; smaller budgets process the columns in chunks, with
 *     bit-identical results); FDWT_LDS_KB_WIDE, the
 *     LDS budget in KiB of the float64 pass tiles (default 160: 2^14-element
 *     tiles; other budgets change the pass plan and so the rounding);
 *     FDWT_EFFDIM_BLOCKED = 0 keeps fdwt_eff_dim's p = 2 intermediate
 *     columns in natural order instead of the blocked layout (the variances
 *     are bit-identical; var_qmc is summed in another order);
 *     FDWT_REDUCE_WKEEP = 0 makes each round of the p = 2 grouped-sum pass
 *     reload its tile's weights instead of a workgroup keeping one tile's
 *     weights for all its columns (bit-identical variances).
 */
#ifndef FDWT_H
#define FDWT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDWT_OK            0
#define FDWT_EINVAL       -1   /* bad argument (p, m, s, sizes, types, NULL)  */
#define FDWT_ENOMEM       -2   /* device or host allocation failed            */
#define FDWT_EDEVICE      -3   /* a HIP runtime call failed                   */
#define FDWT_EBUDGET      -4   /* request exceeds a configured memory budget  */
#define FDWT_EUNSUPPORTED -5   /* valid math, not supported here (e.g. p = 11)*/
#define FDWT_ETIMEOUT     -6   /* a bounded device-side wait gave up          */

/* Element types of transform inputs and outputs. */
#define FDWT_F32  1   /* float                                               */
#define FDWT_I32  2   /* int32, arithmetic modulo 2^32 (p = 2 only)          */
#define FDWT_CF32 3   /* complex float, interleaved (re, im)                 */
#define FDWT_F64  4   /* double                                              */
#define FDWT_CF64 5   /* complex double, interleaved (re, im)                */

typedef struct fdwt_net fdwt_net;

/* ------------------------------------------------------------------ nets */

/* Build the digital (t,m,s)-net P(C) of Section 1 (Definition of a digital
 * net, Eq. (defy)): x_{j,n} = sum_r y_{j,n,r} p^-r with y_vec = C_j n_vec over
 * Z_p.  C_host is uint8 [s][m][m]: C_host[(j*m + r)*m + c] is the entry of
 * C_{j+1} in row r+1 (output digit y_{r+1}, weight p^-(r+1)) and column c
 * (input digit n_c).  Entries must be < p; singular matrices are allowed.
 * The handle copies what it needs from C_host (caller keeps ownership) and
 * owns device tables and a workspace; free it with fdwt_net_free.  The
 * current HIP device at this call is the device of every later call.
 * Errors: FDWT_EINVAL (p not prime, m < 1, p^m > 2^26, s outside 1..64,
 * entry >= p, NULL), FDWT_EUNSUPPORTED (prime p other than 2, 3, 5, 7),
 * FDWT_ENOMEM, FDWT_EDEVICE. */
int fdwt_net_generate(int p, int m, int s, const uint8_t* C_host, fdwt_net** out);

/* p, m, s and N = p^m of a net (any pointer may be NULL). */
int fdwt_net_info(const fdwt_net* net, int* p, int* m, int* s, int64_t* n_points);

/* Integer coordinates X_{j,n} = sum_r y_{j,n,r} p^{m-r} (so x = X p^-m) into
 * X_dev uint32 [s][N].  Bit-exact. */
int fdwt_net_digits(const fdwt_net* net, uint32_t* X_dev, void* stream);

/* Points x_{j,n} = X_{j,n} p^-m as float into x_dev [s][N], correctly
 * rounded to nearest (exact for p = 2 and m <= 24). */
int fdwt_net_points(const fdwt_net* net, float* x_dev, void* stream);

void fdwt_net_free(fdwt_net* net);

/* The handle caches the kernel spectrum K~ (float64, N values, complex for
 * p odd) of the last kernel (alpha, gamma) used by fdwt_spline_coef,
 * fdwt_walsh_interp or fdwt_eff_dim: the spectrum depends on the net and the
 * kernel only, so calls with the same kernel reuse it (a call on another
 * stream waits for it on the device).  fdwt_net_drop_spectrum forgets it
 * (the next call recomputes it into the same memory, which the handle keeps
 * until fdwt_net_free).  Calls on one handle must not overlap in time (they
 * share its workspace and cache). */
int fdwt_net_drop_spectrum(fdwt_net* net);

/* ------------------------------------------------------------ sampling */

#define FDWT_FAMILY_PRODUCT  1   /* f = prod_j (1 + a_j (x_j - 1/2))              */
#define FDWT_FAMILY_EXP      2   /* f = exp(-sum_j a_j x_j^2)                     */
#define FDWT_FAMILY_WANGFANG 3   /* f = prod_j (|4 x_j - 2| + a_j)/(1 + a_j),
                                    the test function of Section 5.2              */
#define FDWT_FAMILY_ASIAN    4   /* discounted payoff of the arithmetic-average
                                    Asian call of Section 5.3: coordinate j drives
                                    step j of the standard construction,
                                    S_j = S_{j-1} exp((r - sigma^2/2) T/s
                                          + sigma sqrt(T/s) Phi^-1(x_j)),
                                    f = exp(-rT) max(A - K, 0), A the mean
                                    of S_0..S_s (the prices at t_j = jT/s,
                                    j = 0..s; Table 4's variances are those of
                                    this mean);
                                    a_host = {S0, K, sigma, r, T} (5 values,
                                    whatever s), evaluated in double            */

/* Sample a test function at the net: f_dev[n] = f(x_n), float [N], computed
 * on the device from the net (the points are not materialised).  a_host is
 * double [s] (read during the call; 5 model values for FDWT_FAMILY_ASIAN).
 * Values are evaluated in float (the Asian payoff in double). */
int fdwt_sample(const fdwt_net* net, int family, const double* a_host, float* f_dev, void* stream);

/* ----------------------------------------------------------- transforms */

/* Forward discrete Walsh transform, Algorithm 1 (Section 2.2), i.e. the
 * coefficients of Eq. (eq_dwalshcoeff):
 *     out[h] = p^-m sum_n in[n] omega_p^(-n_vec . h_vec).
 * Allowed (in_type -> out_type):
 *     p = 2:  F32 -> F32 (normalised as above);
 *             I32 -> I32 (NOT normalised: out = p^m times the coefficient,
 *                         exact modulo 2^32);
 *             F64 -> F64 (normalised; a double-precision reference path);
 *     p odd:  F32 -> CF32, CF32 -> CF32 (normalised);
 *             F64 -> CF64, CF64 -> CF64 (normalised, double precision).
 * in_dev and out_dev may be the same buffer when both types have the same
 * size.  Sizes: N elements each. */
int fdwt_dwt_forward(const fdwt_net* net, int in_type, const void* in_dev,
                     int out_type, void* out_dev, void* stream);

/* Forward transform of a test function sampled at the net on the device:
 * fdwt_sample(family, a_host) followed by fdwt_dwt_forward (two launches;
 * the samples never leave the device).  out_type is F32 (p = 2) or CF32
 * (p odd); out_dev holds N elements of it.  p odd uses the net's workspace
 * for the samples. */
int fdwt_dwt_forward_family(const fdwt_net* net, int family, const double* a_host, int out_type,
                            void* out_dev, void* stream);

/* Inverse transform, Algorithm 2 (Section 3.3), the Lemma's sum:
 *     out[n] = sum_h in[h] omega_p^(+n_vec . h_vec)   (no normalisation).
 * Allowed: p = 2: F32 -> F32, I32 -> I32 (mod 2^32), F64 -> F64; p odd:
 * CF32 -> CF32, and CF32 -> F32, which returns the real part (exact result
 * when the input is the transform of real data); likewise CF64 -> CF64 and
 * CF64 -> F64.  In place allowed for equal sizes. */
int fdwt_dwt_inverse(const fdwt_net* net, int in_type, const void* in_dev,
                     int out_type, void* out_dev, void* stream);

/* fdwt_dwt_inverse for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, types and results, bit for bit, but no call to
 * hipMalloc, hipFree or any allocating routine.  The one case in which the
 * inverse needs scratch memory -- a real output from complex coefficients
 * (p odd, CF32 -> F32 or CF64 -> F64) over more than one pass -- keeps its
 * intermediate passes (N elements of the complex type: 8 N or 16 N bytes) in
 * a fixed 64 MiB device array of the library, one per GPU, held until the
 * process ends; larger transforms fail with FDWT_EBUDGET before any work is
 * enqueued (CF32 -> F32 fits up to N = 2^23 points, CF64 -> F64 up to 2^22).
 * Every call on a GPU shares that GPU's array: calls that overlap in time on
 * one GPU (on different streams, or from different threads) race and must be
 * ordered by the caller.  Nothing in the array needs to start at zero; each
 * call overwrites what it reads. */
int fdwt_dwt_inverse_noalloc(const fdwt_net* net, int in_type, const void* in_dev,
                             int out_type, void* out_dev, void* stream);

/* ------------------------------------------------------- spline kernel */

/* Weighted Walsh kernel of Section 4: K(x,y) = prod_j [1 + gamma_j K'(x_j (-) y_j, 0)]
 * with K'(z,0) = 1 - p^(i(1-alpha)) (p^alpha - 1)/(p - 1), i the index of the
 * first non-zero base-p digit of z (K'(0,0) = 1).  alpha > 1, gamma_j > 0,
 * s must equal the net's s; gamma is host memory read during the call. */
typedef struct {
  double alpha;
  const double* gamma;
  int s;
} fdwt_kernel;

/* Query depth D: queries are D-digit base-p integers Q, q = Q p^-D, with
 * D = 32 (p = 2), 20 (p = 3), 13 (p = 5), 11 (p = 7). */
int fdwt_query_depth(int p);

/* Spline coefficients (Section 3.2, Eq. (splinecoef), then Algorithm 2):
 *     c~(h) = ft(h) / (p^m K~(h)),  c = inverse DWT of c~,
 * where ft is the forward transform of the data (dwt_forward output: F32 for
 * p = 2, CF32 for p odd) and K~ the DWT of the kernel data (K(x_n, 0))_n,
 * computed on the device in float64 (its dynamic range is beyond float).  c_dev is
 * float [N]: the c_n with Sf = sum_n c_n K(., x_n) interpolating the data. */
int fdwt_spline_coef(const fdwt_net* net, const fdwt_kernel* kern, int ft_type,
                     const void* ft_dev, float* c_dev, void* stream);

/* Evaluate Sf(q) = sum_n c_n K(q, x_n) (Section 3.2) at nq queries.  q_dev
 * is uint32 [s][nq] of D-digit integers (see fdwt_query_depth); sf_dev is
 * float [nq].  Partial sums over point blocks are combined in a fixed order
 * (deterministic). */
int fdwt_spline_eval(const fdwt_net* net, const fdwt_kernel* kern, const float* c_dev,
                     int64_t nq, const uint32_t* q_dev, float* sf_dev, void* stream);

/* Whole interpolation: forward DWT of f_dev (float [N] at the net points),
 * spline coefficients (into c_dev if non-NULL, float [N]) and, when nq > 0,
 * Sf at the queries into sf_dev. */
int fdwt_walsh_interp(const fdwt_net* net, const fdwt_kernel* kern, const float* f_dev,
                      float* c_dev, int64_t nq, const uint32_t* q_dev, float* sf_dev,
                      void* stream);

/* As fdwt_walsh_interp, with the queries given as q_depth-digit integers
 * (q = Q p^-q_depth, 1 <= q_depth <= D, every entry below p^q_depth; larger
 * entries are outside [0, 1) and give undefined results); they are lifted
 * on the device to D digits (Q p^(D - q_depth)), the same points.
 * q_depth == D is fdwt_walsh_interp itself.  FDWT_EINVAL for a q_depth out
 * of range. */
int fdwt_walsh_interp_depth(const fdwt_net* net, const fdwt_kernel* kern, const float* f_dev,
                            float* c_dev, int64_t nq, const uint32_t* q_dev, int q_depth,
                            float* sf_dev, void* stream);

/* ------------------------------------------------- effective dimension */

/* ANOVA variances of the spline and effective dimensions (Section 4):
 *   var_trc[d] = sigma^2_trc(Sf; d) = p^2m sum_h |c~(h)|^2 (R_d - 1)~(h),
 *                R_d = prod_{j<=d} (1 + gamma_j^2 R'(x_j, 0)),
 *   var_sup[d] = sigma^2_sup(Sf; d) = sum_{j<=d} p^2m sum_h |c~(h)|^2 Q~_j(h),
 *                Q_j = j-th elementary symmetric polynomial of the
 *                gamma_l^2 R'(x_l, 0),
 * for d = 0..s (index 0 holds 0; var_sup[s] = var_trc[s], the two being
 * sigma^2(Sf) by definition, so Q_s is never transformed), var_total = var_trc[s] = sigma^2(Sf)
 * (Eq. (varSf), with the h = 0 bin included), var_total_h0 = the h = 0
 * bin's share of it, var_qmc = sum_{h != 0} |ft(h)|^2 (the sample variance
 * of the data), d_trc / d_sup = smallest d with var_*[d] >= 0.99 var_total.
 * The kernel data and spectra are computed in float64 and the grouped sums
 * over h accumulated in float64 in a fixed order (deterministic).  var_trc and var_sup are
 * caller-owned host arrays of s+1 doubles. */
typedef struct {
  double* var_trc;
  double* var_sup;
  double var_total;
  double var_total_h0;
  double var_qmc;
  int d_trc;
  int d_sup;
} fdwt_effdim;

/* ft_dev: the forward transform of the data (F32 for p = 2, CF32 for p odd).
 * Synchronises stream before returning. */
int fdwt_eff_dim(const fdwt_net* net, const fdwt_kernel* kern, int ft_type,
                 const void* ft_dev, fdwt_effdim* out, void* stream);

/* The same from the data themselves, eff_dim(net, kernel, f) as Section 4
 * states it: f_dev is float [N], f(x_n) at the net's points; the forward
 * transform (Algorithm 1) runs first, into a stream-ordered allocation of
 * this call.  Results equal fdwt_dwt_forward then fdwt_eff_dim bit for bit.
 * Synchronises stream before returning. */
int fdwt_eff_dim_data(const fdwt_net* net, const fdwt_kernel* kern, const float* f_dev,
                      fdwt_effdim* out, void* stream);

/* ------------------------------------------- kernel-parameter selection */

/* Section 5.1, p = 2.  `net` has m + 1 digits (2N points) and its first N
 * points must form an m-digit net (true when every C_j is upper
 * triangular; otherwise FDWT_EINVAL); f2_dev holds f at all 2N points
 * (float [2N], index order).  The spline with kernel (alpha, gamma_j =
 * beta j^q) is fitted to the first half and the cost is
 *     sum over n = N..2N-1 of (f(x_n) - Sf(x_n))^2
 * (every point of the second half), computed with Walsh transforms: the
 * second half is the first half shifted by x_N, so Sf there is a group
 * convolution of the spline coefficients with K(. (+) x_N, 0).
 * fdwt_split_cost returns the cost (and, if sf_dev is not NULL, Sf at the
 * second half, float [N]); fdwt_kernel_tune minimises it by the Nelder-Mead
 * simplex method in (log(alpha - 1), log beta, q) from start = {alpha, beta,
 * q} with at most max_evals cost evaluations.  Both synchronise `stream`;
 * p odd gives FDWT_EUNSUPPORTED.  Errors: FDWT_EINVAL for alpha <= 1,
 * beta <= 0, a non-finite q or NULL pointers. */
typedef struct {
  double alpha, beta, q;   /* the selected parameters          */
  double cost;             /* their cost                        */
  int evaluations;         /* cost evaluations used             */
} fdwt_kernel_fit;

int fdwt_split_cost(const fdwt_net* net, const float* f2_dev, double alpha, double beta, double q, float* sf_dev,
                    double* cost, void* stream);
int fdwt_kernel_tune(const fdwt_net* net, const float* f2_dev, const double* start, int max_evals,
                     fdwt_kernel_fit* out, void* stream);

/* ------------------------------------------------------------- batches */

/* A ragged batch of independent p = 2 forward transforms (float data, job j
 * of N_j = 2^{m_j} points, 1 <= m_j <= 26, normalised as fdwt_dwt_forward;
 * in_dev == out_dev allowed; different jobs' buffers must not overlap).  The
 * transforms are Algorithm 1 applied to raw data: no net is needed, the
 * output index is the coset label as usual.  Precision / kernel family:
 *   FDWT_PREC_F32          float32; jobs of equal m (>= 7) form a group and
 *                          each pass of a group is one launch of the static
 *                          pass kernels over all its jobs (pointer tables);
 *                          the per-group plan comes from fdwt_batch_autotune
 *                          (or an earlier tuning of that m in the process);
 *   FDWT_PREC_F32_GENERIC  float32 through one persistent launch per pass
 *                          level over all jobs' tiles (at most three);
 *   FDWT_PREC_BF16X2       as FDWT_PREC_F32_GENERIC, but in each job's first
 *                          pass the stages of index digits 0..3 (16-point
 *                          Walsh-Hadamard blocks) run on the matrix cores as
 *                          H16 (hi + lo), x split into two bfloat16 terms,
 *                          float32 accumulation (relative error about 2^-18
 *                          per element from the split);
 *   FDWT_PREC_F32_ONE_LAUNCH  float32, every pass of every job in one
 *                          persistent launch: workgroups take the work items
 *                          (job, pass, tile) in the order fdwt_batch_schedule
 *                          reports from a ticket counter, and an item of pass
 *                          k > 0 waits (device-scope acquire) until its job's
 *                          pass k-1 is complete (device-scope release by each
 *                          finished tile).  Every wait is on items with earlier
 *                          tickets, which running workgroups hold, so the
 *                          launch completes whatever the number of resident
 *                          workgroups.  Waits give up after 2 s of device
 *                          time (the environment variable FDWT_BATCH_WAIT_MS,
 *                          read at creation, sets another limit; 0 makes
 *                          every wait give up, for tests of this path);
 *                          fdwt_batch_check then returns FDWT_ETIMEOUT
 *                          (outputs incomplete).
 * Jobs with m < 7 always take the generic path (with FDWT_PREC_F32).
 * Except in FDWT_PREC_F32_ONE_LAUNCH no workgroup waits on another (the
 * kernel boundaries order the passes).  fdwt_batch_create copies the job list
 * to the device (buffers are fixed at creation); fdwt_batch_run enqueues the
 * launches (nothing else; it can be captured in a HIP graph);
 * fdwt_batch_check waits for the stream and reports any HIP error and, for
 * FDWT_PREC_F32_ONE_LAUNCH, a wait that gave up.
 * fdwt_batch_autotune times every distinct plan of every group (first pass
 * of 2^10 .. 2^14 elements) `reps` times on `stream` and keeps the fastest
 * (median); it overwrites the outputs and skips groups with a job in place.
 * fdwt_batch_describe reports the groups (m, plan's first-pass bound emax,
 * jobs), up to `cap` of them.  The batch owns its device lists; free it with
 * fdwt_batch_free (which synchronises the device first). */
typedef struct {
  int m;
  const float* in_dev;
  float* out_dev;
} fdwt_batch_job;

#define FDWT_PREC_F32         0
#define FDWT_PREC_BF16X2      1
#define FDWT_PREC_F32_GENERIC 2
#define FDWT_PREC_F32_ONE_LAUNCH 3

typedef struct fdwt_batch fdwt_batch;

int fdwt_batch_create(int n_jobs, const fdwt_batch_job* jobs_host, int precision, fdwt_batch** out);
int fdwt_batch_run(fdwt_batch* batch, void* stream);
int fdwt_batch_check(fdwt_batch* batch, void* stream);
int fdwt_batch_autotune(fdwt_batch* batch, int reps, void* stream);
int fdwt_batch_describe(const fdwt_batch* batch, int cap, int* m, int* emax, int* njobs, int* n_groups);
void fdwt_batch_free(fdwt_batch* batch);

/* The work items of FDWT_PREC_F32_ONE_LAUNCH for jobs of sizes m[0..n_jobs)
 * in ticket order, computed on the host (no device is used): item i is tile
 * tile[i] of pass pass[i] of job job[i] (index into m), and need[i] is the
 * number of tiles of that job's pass pass[i] - 1 that must be done first (0
 * for pass 0).  Jobs with m >= 13 have tiles of 2^13 points in every pass
 * (2^(m-13) per pass); smaller jobs one pass of one tile.
 * Writes the first min(cap, total) items into each non-NULL array, the total
 * into *n_items and the items per ticket into *chunk (if non-NULL). */
int fdwt_batch_schedule(int n_jobs, const int* m, int cap, int* job, int* pass, int* tile, int* need, int* n_items,
                        int* chunk);

/* ------------------------------------------------------------- serving */

/* A request loop for interpolation and effective-dimension jobs of any
 * (p, m, s) on one device.  Each request carries its net (p, m, s, C and a
 * caller-chosen net_key), a test-function family with its parameters
 * (sampled on the device as fdwt_sample), the kernel (alpha, gamma) of
 * Section 4 and, for interpolation, nq query points (digits as
 * fdwt_spline_eval).  An interpolation job computes the coefficients of
 * Eq. (eq_dwalshcoeff), the spline coefficients of Eq. (splinecoef) and
 * Sf at the queries (Section 3.3); an effective-dimension job computes the
 * variances and dimensions of fdwt_eff_dim (Section 5).
 *
 * The server holds one device allocation of hbm_budget bytes.  Nets, kernel
 * spectra (per net_key and kernel) and the packed point coordinates used by
 * the evaluation (per net_key) stay resident in it between requests and are
 * evicted least recently used when an arriving job needs room and no running
 * job holds them.  A job is admitted when one of `lanes` HIP streams is idle
 * and its buffers fit; admitted jobs run concurrently.  Admission follows
 * arrival order, except that a job that does not fit may be overtaken by
 * later ones at most max_bypass times.  A job's results are bit-identical
 * whether it runs alone or among others.  effdim_chunk_bytes bounds the
 * kernel-data columns an effective-dimension job holds at once (0: 1 GiB).
 *
 * fdwt_server_submit copies the request (the caller may free its arrays on
 * return) and returns at once with an id; it fails with FDWT_EBUDGET when
 * the request alone exceeds the budget and with FDWT_EINVAL when net_key
 * already names different (p, m, s, C).  fdwt_server_wait blocks until job
 * `id` has finished, fills `info` and the results (sf_host: nq floats for an
 * interpolation; eff: arrays of s + 1 doubles for an effective-dimension
 * job; either may be NULL) and forgets the job; it returns the job's status.
 * Times are seconds on the server's clock (from creation).  Any thread may
 * submit and wait.  fdwt_server_free finishes every submitted job, then
 * releases everything.
 *
 * A job that fails (on the device, or while its work is enqueued) completes
 * with its error status; its memory returns to the arena once its lane is
 * idle, cache entries it was computing are discarded (later jobs recompute
 * them), and no other job is affected.  For testing that isolation,
 * FDWT_SERVER_INJECT_ENOMEM (read by fdwt_server_create) lists job ids,
 * comma-separated, whose work fails with FDWT_ENOMEM right after their
 * kernel-spectrum step, as an allocation failure in mid-job would. */
#define FDWT_JOB_INTERP 1
#define FDWT_JOB_EFFDIM 2

typedef struct {
  size_t hbm_budget;
  int lanes;
  int max_bypass;
  size_t effdim_chunk_bytes;
} fdwt_server_config;

typedef struct {
  int kind;                  /* FDWT_JOB_INTERP or FDWT_JOB_EFFDIM          */
  int p, m, s;
  uint64_t net_key;          /* equal keys must mean equal (p, m, s, C)     */
  const uint8_t* C_host;     /* [s][m][m], as fdwt_net_generate             */
  int family;                /* FDWT_FAMILY_*                               */
  const double* a_host;      /* family parameters: [s], or 5 for ASIAN      */
  double alpha;              /* kernel smoothness, > 1                      */
  const double* gamma_host;  /* [s] kernel weights, > 0                     */
  int64_t nq;                /* interpolation: 1..2^24 queries              */
  const uint32_t* q_host;    /* interpolation: [s][nq] query digits         */
} fdwt_request;

typedef struct {
  int status;
  double t_submit, t_admit, t_done;
  size_t bytes;              /* job buffers held while running (no caches)  */
  int spectrum_hit;          /* the kernel spectrum was resident            */
  int packed_hit;            /* the packed coordinates were resident        */
} fdwt_job_info;

typedef struct {
  int64_t submitted, completed, failed, rejected, pending, in_flight;
  size_t arena_bytes, arena_used, arena_peak;
  int64_t spectrum_hits, spectrum_misses, packed_hits, packed_misses, evictions, nets_built;
} fdwt_server_counters;

typedef struct fdwt_server fdwt_server;

/* Device bytes a request needs: its own buffers (job_bytes) and the cache
 * entries it creates on a miss (cache_bytes).  Host-only. */
int fdwt_server_request_bytes(const fdwt_request* req, size_t effdim_chunk_bytes, size_t* job_bytes,
                              size_t* cache_bytes);
int fdwt_server_create(const fdwt_server_config* cfg, fdwt_server** out);
int fdwt_server_submit(fdwt_server* server, const fdwt_request* req, int64_t* id);
int fdwt_server_wait(fdwt_server* server, int64_t id, fdwt_job_info* info, float* sf_host, fdwt_effdim* eff);
int fdwt_server_stats(fdwt_server* server, fdwt_server_counters* stats);
void fdwt_server_free(fdwt_server* server);

/* ------------------------------------------------------------ timing */

/* Per-launch timing of the library's kernels, for benchmarks and tracing.
 * While enabled, every kernel launch of the classes below is bracketed by a
 * pair of HIP events recorded on the stream it is launched on, together with
 * its algorithmic work (bytes that must cross HBM for the transform passes:
 * every element read once and written once, or read once and reduced; bytes
 * written for the generators; coordinate evaluations for FDWT_TC_EVAL).
 * Enabling (or disabling) discards earlier records.  fdwt_timing_query
 * waits for the recorded events of a class and returns the summed duration
 * in milliseconds, the number of launches and the summed work.  Recording
 * costs two event records per launch; it is off by default. */
#define FDWT_TC_PASS_F32   0   /* transform passes, float / int32 elements     */
#define FDWT_TC_PASS_CF32  1   /* transform passes, complex float              */
#define FDWT_TC_PASS_F64   2   /* kernel-spectrum passes, double / complex double */
#define FDWT_TC_SAMPLE     3   /* net generation + test-function sampling      */
#define FDWT_TC_KCOLS      4   /* kernel-data columns (K, R_d - 1, Q_j)        */
#define FDWT_TC_EVAL       5   /* interpolant evaluation at queries            */
#define FDWT_TC_BATCH      6   /* one batch run (all its level launches)       */
#define FDWT_TC_COUNT      7

int fdwt_timing_enable(int on);
int fdwt_timing_query(int cls, double* total_ms, int64_t* launches, double* work);

/* ------------------------------------------------------------ errors */

/* Message of the last failed call on this thread ("" if none).  The pointer
 * stays valid until the next fdwt_* call on the thread. */
const char* fdwt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDWT_H */
