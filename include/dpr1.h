/*
 * dpr1.h -- C ABI of libdpr1.so: forward-stable eigendecomposition of
 * diagonal-plus-rank-one (DPR1) matrices  A = D + rho * z * z^T  on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Jakovcevic Stor, Slapnicar, Barlow, "Forward stable eigenvalue
 * decomposition of rank-one modifications of diagonal matrices", Algorithm 1.
 * Every eigenpair is computed independently in O(n): shift to the nearest pole
 * d_i (Alg. 1, shift test), form the arrowhead inverse of A - d_i I
 * (eq. invAi) with its tip b (eq. b_ob) in double-double arithmetic, find the
 * extreme eigenvalue nu of that inverse (eq. secAi), set mu = 1/nu,
 * lambda = d_i + mu (eq. 8) and x = (D - d_i I - mu I)^{-1} z
 * (eq. eigenvecAi), v = x/||x||_2.
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers unless the name ends in _host.
 *    The caller owns every buffer.  The library allocates no device memory:
 *    it uses the caller's workspace, whose size the *_workspace_size queries
 *    return (dpr1_eig_noalloc: a static device array of the library).
 *    Workspace contents need not be initialised.
 *  - All work is enqueued asynchronously on `stream` (a hipStream_t passed as
 *    void*; NULL = the default stream); dpr1_eig with eigenvectors and
 *    opts.vwrite >= 2 forks part of its work to a second stream of the
 *    library and joins it back into `stream` through events before it
 *    returns.  No call
 *    synchronises the host, so the launches may be captured into a hipGraph,
 *    except dpr1_batched_plan (it copies from host memory), the autotuners
 *    and dpr1_eig_general.
 *  - Inputs (Sec. 1 of the paper): n >= 1, d strictly decreasing, every
 *    z_j != 0, rho != 0 and finite.  rho < 0 is reduced to rho > 0 as in
 *    Sec. 1 by solving with (-d reversed, z reversed, -rho) and mapping back.
 *    dpr1_eig and the batched path report reducible problems (info) rather
 *    than solve them; dpr1_eig_general sorts and deflates first.
 *  - Outputs: lambda[k] decreasing (strict interlacing, eq. interlace);
 *    V column-major, column k (k = 0..n-1) = v_k at V + k*ldv, with the sign
 *    of eq. (Aeigenvec): v_k has the direction of (D - lambda_k I)^{-1} z.
 *  - Synchronous return codes: 0 success; -p argument p (1-based) invalid
 *    (null pointer, n < 1, ldv < n, non-finite or zero rho, workspace too
 *    small); DPR1_EHIP a HIP launch failed.
 *  - Asynchronous per-problem device `info` (int32, set by the library on the
 *    stream): 0 ok; DPR1_INFO_UNSORTED d not strictly decreasing;
 *    DPR1_INFO_ZERO_Z some z_j == 0 (reducible, Sec. 1); DPR1_INFO_NONFINITE
 *    a non-finite input; DPR1_INFO_BAD_RHO zero or non-finite rho (batched);
 *    DPR1_INFO_RANGE the problem leaves the binary64 range of the method:
 *    some 0 < |z_j| < 2^-511 (its square is not a normal number), two poles
 *    closer than 2^-1000, or the shifted representation (d_i, mu) of some
 *    eigenpair not representable (mu not a normal number, |mu| ||x|| not
 *    finite: an eigenvalue within ~1e-300 of a pole whose zeta_i is ~1e-150
 *    while the poles spread over many decades).  Deflating such z_j avoids
 *    it; dpr1_eig_general does so for |z_j| < 2^-511.
 *    When info != 0 the outputs of that problem are unspecified.
 */
#ifndef DPR1_H
#define DPR1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPR1_OK 0
#define DPR1_EHIP (-1000)
#define DPR1_ETOOBIG (-1001) /* n above DPR1_NOALLOC_MAX_N (dpr1_eig_noalloc) */

#define DPR1_INFO_OK 0
#define DPR1_INFO_UNSORTED 1
#define DPR1_INFO_ZERO_Z 2
#define DPR1_INFO_NONFINITE 3
#define DPR1_INFO_BAD_RHO 4
#define DPR1_INFO_RANGE 5

/* Counters written to the optional device `stats` array (int32, length
 * DPR1_NSTATS; the library zeroes it before counting).                      */
#define DPR1_STAT_KB_GT_100 0 /* eigenvalues with K_b > 100 (eq. knu2): the
                                 paper's test for double-precision b        */
#define DPR1_STAT_POLISHED 1  /* roots polished by double-double Newton     */
#define DPR1_STAT_NEARZERO 2  /* lambda recomputed from A^{-1} (eq. gamma)  */
#define DPR1_STAT_SINGULAR 3  /* f(0) rounded to 0: lambda set to 0         */
#define DPR1_STAT_ITERS_MAX 4 /* most root-finder passes for one eigenvalue */
#define DPR1_STAT_ITERS_SUM 5 /* root-finder passes summed over eigenvalues */
#define DPR1_STAT_CONTINUED 6 /* root searches finished by the cooperative
                                 kernel after the pass budget               */
#define DPR1_STAT_POLISH_STEPS_MAX 7 /* most double-double steps one polish
                                 took (including the one that confirmed the
                                 root)                                      */
#define DPR1_STAT_KNU_GT 8    /* eigenpairs with K_nu > knu_thr (eq. K0)     */
#define DPR1_STAT_REMEDY_R1 9 /* eigenpairs recomputed by remedy (R1)        */
#define DPR1_STAT_REMEDY_R2 10 /* eigenpairs recomputed by remedy (R2)       */
#define DPR1_STAT_EXT_B 11    /* eigenvalues whose tip b (eq. b_ob) was formed
                                 in double-double                          */
#define DPR1_NSTATS 12

/* Options.  dpr1_default_opts fills the defaults noted below.               */
typedef struct dpr1_opts {
  int32_t mode_b;      /* tip b of A_i^{-1}: 0 double-double always (default);
                          1 double-double only when K_b > 100; 2 never (the
                          paper's dpr1eig_nd); 3 Algorithm 1's gate:
                          double-double when the bound of eq. (knu2),
                          min((n+4) sqrt(n) K_b, 3 sqrt(n) + (n+4)(1 + 2 K_z))
                          from the standard-precision K_b, exceeds
                          100 (n+4) sqrt(n)                                  */
  int32_t root;        /* 0 bisection (Alg. 1); 1 (default) safeguarded
                          model iteration: the nearest pole exact plus one
                          pole fitted to the value, slope and curvature of
                          the rest of the secular sum (Sec. 2.2 leaves the
                          root finder open)                                 */
  int32_t polish;      /* 1 (default): double-double Newton polish of roots
                          whose rounding amplification is large; 0 off     */
  int32_t split;       /* waves that share one block of 64 eigenvalues by
                          splitting the inner sum; 0 = chosen from n        */
  double kappa_polish; /* polish threshold on kappa_g*max(1,|mu/lambda|);
                          default 16                                        */
  double nearzero;     /* near-zero rule factor: recompute lambda from
                          A^{-1} when factor*|lambda| < distance to the
                          neighbouring poles; default 10, 0 disables        */
  int32_t main_passes; /* model solver: passes the eigenvalue kernel runs
                          (the last one with compensated summation) before
                          it hands an unconverged eigenpair to the
                          cooperative kernel; 0 = default (2 for dpr1_eig,
                          3 for dpr1_eig_batched)                          */
  int32_t waves_per_simd; /* register budget of the eigenvalue kernel: 4
                          (default, 0) waves per SIMD with up to 128 VGPRs,
                          6 (80) or 8 (64); more waves hide more latency,
                          fewer registers spill more of the outer state;
                          other values are rejected                        */
  void* events;        /* profiling hook, NULL (default) = off: a host array
                          of 4 hipEvent_t that the solve records on `stream`
                          right before and after the eigenvalue kernel
                          ([0], [1]) and around the second phase ([2], [3]):
                          the flagged eigenpairs overlapped with the
                          eigenvector write                                 */
  int32_t vwrite;      /* eigenvectors of a single problem of order n >= 8192:
                          0 (default) or 1: every column after the
                          eigenvalue kernel, on `stream` only; K = 2 .. 8: the eigenvalue
                          kernel runs in K launches over consecutive chunks
                          of the eigenvalues, and each chunk's columns but
                          the last are written on a second stream (a library
                          stream per device, created on first use, default
                          priority) while the next chunk is solved.
                          Results are the same bit for bit.  Other values
                          are rejected.  dpr1_eig_noalloc always writes
                          after the eigenvalue kernel.                     */
  int32_t remedy;      /* Sec. 2, Algorithm 1's last branch: 1 = where K_nu
                          of eq. (K0) exceeds knu_thr, recompute the
                          eigenpair by remedy (R1) -- the other neighbouring
                          pole, when its K_nu is smaller and below the
                          threshold -- else by remedy (R2) -- A - sigma I with
                          sigma between the nearest pole and lambda, its
                          inverse in double-double; 0 (default) = K_nu only
                          counted (and written to knu); the double-double
                          polish (polish) acts either way                   */
  double knu_thr;      /* threshold on K_nu; default 32                     */
  double* knu;         /* optional device output [n] (a batch: [sum n_p],
                          packed like lambda): K_nu of every eigenpair,
                          ||A_i^{-1}||_2/|nu| at its shift pole             */
} dpr1_opts;

void dpr1_default_opts(dpr1_opts* opts);

/* Bytes of device workspace dpr1_eig needs for a problem of order n.       */
size_t dpr1_workspace_size(int64_t n);

/* All eigenpairs of one DPR1 matrix (Alg. 1 for k = 1..n).
 *   d, z          [n]  input (device, float64)
 *   rho           scalar (host)
 *   lambda        [n]  output eigenvalues, decreasing
 *   V             [ldv*n] output eigenvectors (column-major) or NULL for
 *                 eigenvalues only
 *   ldv           leading dimension of V (>= n; ignored when V == NULL)
 *   shift_idx     [n] optional output: index i of the pole d_i used as shift
 *   mu            [n] optional output: mu_k = lambda_k - d_{i_k}; the pair
 *                 (d_i, mu) represents lambda to about twice the working
 *                 precision (Example 2)
 *   xnorm         [n] optional output: ||x_k||_2 of eq. (eigenvecAi)
 *   info          [1] device int32 (see above)
 *   stats         [DPR1_NSTATS] optional device int32 counters
 *   opts          NULL = defaults
 *   work, work_bytes  device workspace (>= dpr1_workspace_size(n))          */
int dpr1_eig(const double* d, const double* z, double rho, int64_t n, double* lambda,
             double* V, int64_t ldv, int32_t* shift_idx, double* mu, double* xnorm,
             int32_t* info, int32_t* stats, const dpr1_opts* opts, void* work,
             size_t work_bytes, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dpr1_eig
 * without the workspace argument.  Its workspace is a static device array of
 * the library, dpr1_noalloc_scratch_bytes() bytes (about 6.2 MB, sized for
 * n = DPR1_NOALLOC_MAX_N), of which every GPU the library runs on holds its
 * own copy until the process ends.  The call allocates nothing (no hipMalloc,
 * no allocating library routine); on its first use on a device it looks up
 * that device's copy of the array (hipGetSymbolAddress) and keeps the
 * address.  Arguments, outputs, info codes and results are those of
 * dpr1_eig with the same options (the same kernels run on the same data).
 * Returns DPR1_ETOOBIG when n > DPR1_NOALLOC_MAX_N, the other codes as
 * dpr1_eig (-4 for n < 1, -13 for an invalid waves_per_simd), DPR1_EHIP when
 * the array cannot be reached.  All calls on one GPU share its array and the
 * array keeps the last call's contents (the solve clears its own counters):
 * calls that overlap on one GPU (different streams, or host threads, without
 * ordering between them) race and give undefined results; calls ordered on
 * one stream are safe.                                                      */
#define DPR1_NOALLOC_MAX_N 32768
size_t dpr1_noalloc_scratch_bytes(void);
int dpr1_eig_noalloc(const double* d, const double* z, double rho, int64_t n, double* lambda,
                     double* V, int64_t ldv, int32_t* shift_idx, double* mu, double* xnorm,
                     int32_t* info, int32_t* stats, const dpr1_opts* opts, void* stream);

/* Batched: nprob independent problems of sizes n_p packed back to back
 * (problem p occupies [offs[p], offs[p+1]) of d, z, lambda, shift_idx, mu,
 * xnorm; its V block starts at voffs[p] with leading dimension n_p).  As in
 * divide-and-conquer merges the sizes are ragged; all problems are solved by
 * one persistent launch whose blocks take (problem, 64 eigenvalues) items
 * from a device work queue, larger problems first.
 *
 * dpr1_batched_workspace_size(nprob, offs_host): bytes of workspace for the
 *   batch with these host offsets (0 if the offsets are invalid).
 * dpr1_batched_plan: reads the host offsets (offs_host[0] = 0, sizes >= 1),
 *   builds the work queue and the launch shape, copies the queue into the
 *   workspace and synchronises `stream` (the only host->device copy and the
 *   only synchronisation of the batched path).  The plan struct (host memory,
 *   caller-owned) is then passed to every solve of that batch shape; the
 *   solve can be repeated or captured in a hipGraph with the same workspace.
 * dpr1_eig_batched: the solve, kernel launches only.  offs [nprob+1] and
 *   voffs [nprob] are device arrays (the same offsets as planned; voffs may be
 *   NULL when V is NULL); rho is a device array [nprob]; info is [nprob].   */
typedef struct dpr1_plan {
  int64_t nprob, ntotal, nitems, nmax, ngroups;
  int32_t split, grid;
  dpr1_opts opts;
} dpr1_plan;

size_t dpr1_batched_workspace_size(int64_t nprob, const int64_t* offs_host);
int dpr1_batched_plan(int64_t nprob, const int64_t* offs_host, const dpr1_opts* opts,
                      dpr1_plan* plan, void* work, size_t work_bytes, void* stream);
int dpr1_eig_batched(const dpr1_plan* plan, const int64_t* offs, const double* d,
                     const double* z, const double* rho, double* lambda, double* V,
                     const int64_t* voffs, int32_t* shift_idx, double* mu, double* xnorm,
                     int32_t* info, int32_t* stats, void* work, size_t work_bytes,
                     void* stream);

/* Autotuning (not in the paper): the launch shape is chosen by measurement.
 * The candidates are the split W in {1, 2, 4, 8, 12, 16} (waves sharing one
 * block of 64 eigenvalues, i.e. W threads per eigenvalue; every wave's slice
 * of the inner sum keeps at least 64 terms), the register budget
 * waves_per_simd in {4, 6, 8}, for the model iteration (root = 1) the pass
 * budget main_passes ({2, 3} single, {2, 3, 4} batched) and, for one problem
 * with eigenvectors at n >= 8192, the write vwrite in {0 (after the
 * eigenvalue kernel), 2 (overlapped in two chunks)}.  Each
 * candidate is solved once untimed and then `reps` times (0 = 3) between two
 * events on `stream`; the fastest mean wins, ties keep the earlier candidate
 * (smaller W, then fewer waves, then the smaller budget), and a 6- or 8-wave
 * register budget (which spills part of the eigenvalue kernel's state) must
 * be 4 % faster than the best so far to be chosen.  Both calls run on
 * the caller's data and buffers, leave a
 * valid solution in the outputs (that of the last candidate, equal to the
 * tuned one's within the parity bounds) and synchronise `stream`.
 * dpr1_autotune: arguments as dpr1_eig; opts (in/out, required) supplies the
 *   other options and receives the chosen split, waves_per_simd,
 *   main_passes and vwrite; best_ms
 *   (optional) the fastest mean time.
 * dpr1_batched_autotune: arguments as dpr1_eig_batched; plan (in/out, from
 *   dpr1_batched_plan for these offsets) receives the chosen split, grid,
 *   waves_per_simd and main_passes.  Return codes as the solves they time;
 *   -13 reps < 0.                                                            */
int dpr1_autotune(const double* d, const double* z, double rho, int64_t n, double* lambda, double* V,
                  int64_t ldv, int32_t* shift_idx, double* mu, double* xnorm, int32_t* info,
                  dpr1_opts* opts, int32_t reps, double* best_ms, void* work, size_t work_bytes,
                  void* stream);
int dpr1_batched_autotune(dpr1_plan* plan, const int64_t* offs, const double* d, const double* z,
                          const double* rho, double* lambda, double* V, const int64_t* voffs,
                          int32_t* shift_idx, double* mu, double* xnorm, int32_t* info, int32_t reps,
                          double* best_ms, void* work, size_t work_bytes, void* stream);

/* Reverse mode (not in the paper; standard eigenvalue perturbation theory).
 * For L(Lambda, V) with lambda_bar = dL/dlambda, V_bar = dL/dV:
 *   Abar = V X V^T,  X = diag(lambda_bar) + F o (V^T V_bar),
 *   F_lk = 1/(lambda_k - lambda_l) (l != k) with the gaps taken from the
 *   shifted representation (d_{i_k} + mu_k) - (d_{i_l} + mu_l);
 *   d_bar_j = Abar_jj, rho_bar = z^T Abar z, z_bar = rho (Abar + Abar^T) z,
 * evaluated as d_bar_j = sum_k (V X)_jk V_jk, y_k = v_k^T z = -1/(rho ||x_k||),
 * rho_bar = y^T X y, z_bar = rho V (X + X^T) y.  The two n^3 products use
 * FP64 matrix cores.  Without V_bar only the eigenvalue part remains and is
 * evaluated in closed form in O(n^2): d_bar_j = sum_k lambda_bar_k V_jk^2,
 * z_bar_j = -2 sum_k lambda_bar_k V_jk / ||x_k||,
 * rho_bar = sum_k lambda_bar_k / (rho ||x_k||)^2.  Problems of one batch have equal size n and are stored
 * with strides n (vectors) and n*n (matrices, column-major, ld = n).
 *   shift_idx, mu, xnorm: as returned by the forward call.
 *   V: the forward's eigenvectors, or NULL: then every element the two
 *     products need is recomputed from z and the shifted representation,
 *     v_k[j] = z_j / (((d_j - d_{i_k}) - mu_k) ||x_k||) (eq. eigenvecAi),
 *     inside the GEMM tile loads, so that V need not be kept (or even
 *     written: a forward without eigenvectors suffices).  z may be NULL only
 *     when V is given (-4 otherwise).
 *   lambda_bar, V_bar: either may be NULL (treated as zero).
 *   d_bar, z_bar [nbatch*n], rho_bar [nbatch]: outputs.                    */
size_t dpr1_backward_workspace_size(int64_t n, int64_t nbatch);
int dpr1_eig_backward_batched(int64_t nbatch, int64_t n, const double* d, const double* z,
                              const double* rho, const int32_t* shift_idx, const double* mu,
                              const double* xnorm, const double* V, const double* lambda_bar,
                              const double* V_bar, double* d_bar, double* z_bar,
                              double* rho_bar, void* work, size_t work_bytes, void* stream);
/* One problem, the same reverse mode with rho a host scalar (!= 0, finite) and
 * V, V_bar column-major with leading dimensions ldv, ldvb >= n (ignored when
 * the matrix is NULL); workspace dpr1_backward_workspace_size(n, 1) bytes;
 * rho_bar [1] device.  Argument errors -p as the parameter list orders them
 * (z may be NULL only when V is given: -2; ldv: -9, ldvb: -12, work_bytes:
 * -17).  Kernel launches only.                                              */
int dpr1_eig_backward(const double* d, const double* z, double rho, int64_t n,
                      const int32_t* shift_idx, const double* mu, const double* xnorm,
                      const double* V, int64_t ldv, const double* lambda_bar,
                      const double* V_bar, int64_t ldvb, double* d_bar, double* z_bar,
                      double* rho_bar, void* work, size_t work_bytes, void* stream);

/* Reducible inputs (Sec. 1): any finite d (any order, repeated values) and
 * any finite z (zeros allowed).  The poles are sorted decreasingly; a pole
 * with z_j == 0 is deflated (eigenpair (d_j, e_j)); a group of equal poles
 * d_j with part w of z is merged by a Householder reflection H of its block
 * with H w = -sign(w_first) ||w|| e_first: the pole enters the reduced problem
 * once, with z = ||w||, and the other columns of H are eigenvectors for the
 * eigenvalue d_j (orthogonal to w).  The reduced problem, strictly decreasing
 * with no zero z, is solved by dpr1_eig on the device (eigenvalues and the
 * shifted representation only); its eigenvectors are then written directly
 * in the caller's row order from eq. (eigenvecAi) evaluated on the original
 * d and z.
 *   d, z         [n] input (device, float64), rows in the caller's order
 *   rho          scalar (host), != 0 and finite
 *   lambda       [n] output, decreasing
 *   V            [ldv*n] output or NULL; column k = v_k with rows in the
 *                caller's order (V^T A V = diag(lambda) for the unsorted A);
 *                columns of equal eigenvalues form an orthonormal basis of
 *                the eigenspace, in no particular order
 *   info         [1] device int32: 0, DPR1_INFO_NONFINITE, or a code of the
 *                reduced solve
 *   opts         options of the reduced solve (NULL = defaults; an invalid
 *                waves_per_simd is argument -9)
 *   work, work_bytes  device workspace (>= dpr1_general_workspace_size(n),
 *                O(n) bytes)
 * Unlike every other entry point this one SYNCHRONISES the host with
 * `stream`: the reduction (a sort and a scan of n numbers) runs on the host
 * from a device-to-host copy of d and z, and the reduced eigenvalues are
 * merged with the deflated poles on the host.  It cannot be captured in a
 * hipGraph.  Returns 0, -p for an invalid argument p, or DPR1_EHIP.         */
size_t dpr1_general_workspace_size(int64_t n);   /* also for dpr1_eig_hermitian */
int dpr1_eig_general(const double* d, const double* z, double rho, int64_t n, double* lambda,
                     double* V, int64_t ldv, int32_t* info, const dpr1_opts* opts, void* work,
                     size_t work_bytes, void* stream);

/* Hermitian DPR1 (the remark after Algorithm 1 says the method extends to it):
 * A = D + rho z z^H with real d, complex z.  With Phi = diag(z_j / |z_j|)
 * (1 where z_j = 0), Phi is unitary, Phi D Phi^H = D and z = Phi |z|, so
 * A = Phi (D + rho |z| |z|^T) Phi^H: the eigenvalues are those of the real
 * problem with |z| (solved as by dpr1_eig_general: any order, repeated poles,
 * zero z_j) and v_k = Phi v_k^real.
 *   z    [2n] device, interleaved (re, im) -- complex128
 *   V    [2*ldv*n] device complex128 or NULL: element (i, k) at V[2 (i + k ldv)]
 *        (re) and V[2 (i + k ldv) + 1] (im); column k = v_k, V^H A V = diag(lambda)
 * Everything else (lambda, info, opts, workspace, errors, host
 * synchronisation) as for dpr1_eig_general.                                 */
int dpr1_eig_hermitian(const double* d, const double* z, double rho, int64_t n, double* lambda,
                       double* V, int64_t ldv, int32_t* info, const dpr1_opts* opts, void* work,
                       size_t work_bytes, void* stream);

/* Symmetric tridiagonal eigensolver by divide and conquer whose merges are
 * DPR1 problems (the application named in Sec. 1).  T has diagonal a [n] and
 * off-diagonal b [n-1] (device).  A block is split at m = size/2 with
 * beta = b there: T = diag(T1 - beta e_m e_m^T, T2 - beta e_1 e_1^T)
 * + beta u u^T, u = e_m + e_{m+1}; the halves are solved recursively down to
 * 1 x 1, and each merge is the DPR1 problem D = diag(Lambda1, Lambda2),
 * z = [last row of Q1, first row of Q2], rho = beta, reduced as by
 * dpr1_eig_general (beta = 0 decouples the halves), solved for all merges
 * of one depth in one batched launch, and followed by Q = diag(Q1, Q2) V.
 *   lambda  [n] output, decreasing
 *   Q       [ldq*n] output (required: the merges need it), column k = q_k
 *   info    [1] device int32: 0, DPR1_INFO_NONFINITE, or a code of a merge
 *   opts    options of the merges' DPR1 solves (NULL = defaults; an invalid
 *           waves_per_simd is argument -8)
 *   work, work_bytes  >= dpr1_tridiag_workspace_size(n): about 16 n^2 bytes
 *           (a second Q buffer and the merges' V) plus O(n)
 * 1 <= n <= 65536.  Synchronises the host with `stream` a few times per
 * depth of the split tree (the merges are reduced on the host); the merges'
 * DPR1 solves run on a second stream of the library (created once per
 * device, default priority) beside the products on `stream`, and the call
 * returns when the work on both has finished.  Returns 0,
 * -p for an invalid argument p (-10 also when the workspace is too small),
 * or DPR1_EHIP.                                                             */
size_t dpr1_tridiag_workspace_size(int64_t n);
int dpr1_tridiag_eig(const double* a, const double* b, int64_t n, double* lambda, double* Q,
                     int64_t ldq, int32_t* info, const dpr1_opts* opts, void* work,
                     size_t work_bytes, void* stream);

/* Text for a return code or an info code.                                   */
const char* dpr1_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* DPR1_H */
