/*
 * dpr1_oracle.c -- CPU oracle for the forward-stable eigensolver of
 * diagonal-plus-rank-one (DPR1) matrices A = D + rho*z*z^T
 * (Jakovcevic Stor, Slapnicar, Barlow, "Forward stable eigenvalue
 * decomposition of rank-one modifications of diagonal matrices", Alg. 1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  It is loaded only by the test suite, by
 * the package's smoke check and by the benchmark's CPU-baseline leg; the
 * library itself never links, loads or calls it.  It shares no source with
 * the GPU path.
 *
 * Arithmetic: IEEE binary64 everywhere the paper works in the working
 * precision; IEEE binary128 (__float128) wherever the paper asks for "double
 * the working precision" (Sec. 2.3: the third of its implementations, a
 * 128-bit REAL(16) evaluation, is exactly this).  Built with
 * -ffp-contract=off and without fast-math, so every binary64 operation below
 * is one correctly rounded IEEE operation in source order.
 *
 * Notation follows the paper: d_j poles (strictly decreasing), zeta_j the
 * entries of z, sigma = d_i the shift, delta_j = d_j - sigma (the diagonals of
 * D_1, D_2), xi_j = 1/delta_j (diagonal of the arrowhead inverse), w_j the
 * arrow, b the tip, nu the extreme eigenvalue of the inverse, mu = 1/nu.
 * Indices are 0-based here; the paper's k is (k+1).
 *
 * Readings of the paper (every one is also listed in the design notes):
 *  - b in extended precision: mode 0 always (default), mode 1 only when
 *    K_b > 100 (the threshold that reproduces the counts of Example 4),
 *    mode 2 never (the paper's dpr1eig_nd).
 *  - Bisection (Sec. 2.1/2.2) walks the binary64 numbers in order: the
 *    midpoint of two same-signed endpoints is the midpoint of their bit
 *    patterns, so it ends with two adjacent numbers after at most 63 halvings
 *    whatever the bracket's dynamic range.
 *  - After bisection one Newton step with the secular sum accumulated by
 *    compensated (Neumaier) summation makes nu independent of summation order
 *    to about 4*kappa_g*eps_M, where kappa_g is the rounding-amplification of
 *    g at the root.  When kappa_g * max(1,|mu/lambda|) exceeds a threshold
 *    (16), the result is polished by safeguarded Newton steps with g
 *    evaluated in binary128: the paper's remedy (R2) in its last form, which
 *    falls back to twice the working precision.  This also covers k = 1,
 *    where (R1) is impossible (there is no pole on the other side).
 *  - The near-zero rule (Alg. 1, last test) fires when
 *    10*|lambda| < min |lambda - neighbouring pole|.
 *  - Range of the arrowhead inverse (eq. invAi, secAi): with a tiny zeta_i
 *    beside a close pole the arrow w_j = -zeta_j/(zeta_i delta_j) can exceed
 *    2^511 (zeta_i near 1e-150 beside a pole 1e-13 away gives 1e162), so its
 *    square, and the terms of g, leave binary64 although the eigenpair does
 *    not.  For such an eigenpair the whole secular function -- its bracket,
 *    every evaluation of g for the bisection and the Newton step -- is carried
 *    in binary128 (exponent range 1e+-4932) from the exact shifted
 *    differences, with the binary128 tip (there is no binary64 b to gate).
 *    Every other eigenpair is computed in binary64 exactly as above.
 */
#include <float.h>
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 quad;

typedef struct {
  int32_t mode_b;        /* 0 quad always, 1 quad iff K_b > 100, 2 never,
                            3 quad iff the bound of eq. (knu2) exceeds
                            100 (n+4) sqrt(n)                              */
  int32_t polish;        /* 1: extended-precision polish when flagged        */
  double kappa_polish;   /* threshold on kappa_g*max(1,|mu/lambda|)          */
  double nearzero;       /* factor of the near-zero test                     */
  int32_t remedy;        /* 1: remedies (R1)/(R2) where K_nu > knu_thr       */
  int32_t pad;
  double knu_thr;        /* threshold on K_nu of eq. (K0)                    */
} oracle_opts;

typedef struct {
  int32_t i;             /* shift index, sigma = d[i]                        */
  int32_t side;          /* +1: sigma = d_k, rightmost nu; -1: leftmost      */
  int32_t used_ext_b;    /* b evaluated in binary128                         */
  int32_t polished;      /* extended-precision Newton polish applied         */
  int32_t nearzero;      /* lambda recomputed from A^{-1} (eq. gamma)        */
  int32_t singular;      /* f(0) rounded to zero: lambda set to 0            */
  int32_t bisect_iters;
  int32_t polish_iters;
  double sigma, mu, nu, lambda, b;
  double Kb, Kz, kappa_nu_bound, kappa_g;
  double xnorm;          /* ||x||_2 of the unnormalised eigenvector          */
  double Knu;            /* K_nu of eq. (K0) at the shift pole (all-pairs
                            driver only; 0 where not computed)              */
  int32_t remedied;      /* 0 none, 1 remedy (R1), 2 remedy (R2)             */
  int32_t pad2;
} oracle_eigdiag;

#define ORC_OK 0
#define ORC_EARG (-1)
#define ORC_UNSORTED 1
#define ORC_ZERO_Z 2
#define ORC_NONFINITE 3


void oracle_default_opts(oracle_opts* o) {
  o->mode_b = 0;
  o->polish = 1;
  o->kappa_polish = 16.0;
  o->nearzero = 10.0;
  o->remedy = 0;
  o->pad = 0;
  o->knu_thr = 32.0;
}

/* ---------------------------------------------------------------- helpers */

static uint64_t dbits(double x) { uint64_t u; memcpy(&u, &x, 8); return u; }
static double bitsd(uint64_t u) { double x; memcpy(&x, &u, 8); return x; }

/* Midpoint in the ordering of binary64 numbers, for 0 < lo < hi or
 * lo < hi < 0.  Returns lo or hi only when they are adjacent. */
static double fmid(double lo, double hi) {
  if (lo > 0) {
    uint64_t a = dbits(lo), b = dbits(hi);
    return bitsd(a + (b - a) / 2);
  } else {
    uint64_t a = dbits(-hi), b = dbits(-lo);
    return -bitsd(a + (b - a) / 2);
  }
}

static int adjacent(double lo, double hi) {
  if (lo > 0) return dbits(hi) - dbits(lo) <= 1;
  return dbits(-lo) - dbits(-hi) <= 1;
}

int oracle_check(const double* d, const double* z, double rho, int64_t n) {
  if (n < 1 || !d || !z) return ORC_EARG;
  if (!isfinite(rho) || rho == 0.0) return ORC_EARG;
  for (int64_t j = 0; j < n; ++j)
    if (!isfinite(d[j]) || !isfinite(z[j])) return ORC_NONFINITE;
  for (int64_t j = 0; j + 1 < n; ++j)
    if (!(d[j] > d[j + 1])) return ORC_UNSORTED;
  for (int64_t j = 0; j < n; ++j)
    if (z[j] == 0.0) return ORC_ZERO_Z;
  return ORC_OK;
}

/* ------------------------------------------------ the arrowhead inverse */
/* Per eigenpair the oracle materialises the entries of A_i^{-1} (eq. invAi,
 * b_ob): xi_j = 1/delta_j and w_j = -zeta_j/(zeta_i*delta_j) for j != i, in
 * binary64, and the tip b.  It also keeps the binary128 versions used by the
 * extended-precision polish. */
typedef struct {
  int64_t n, i;
  double sigma, rho;
  double* delta; /* [n] binary64 d_j - sigma, delta_i = 0 */
  double* xi;    /* [n] 1/delta_j (xi_i unused)           */
  double* w;     /* [n] arrow (w_i unused)                */
  double b;
  quad bq;       /* b in binary128 (when evaluated)       */
} arrow_t;

/* Secular function of the arrowhead (eq. secAi), with the diagonal of the
 * arrowhead being D_1^{-1}, D_2^{-1}:  g(nu) = b - nu - sum w_j^2/(xi_j - nu).
 * Plain binary64 evaluation in ascending j. */
static double g_plain(const arrow_t* A, double nu) {
  double s = 0.0;
  for (int64_t j = 0; j < A->n; ++j) {
    if (j == A->i) continue;
    s += A->w[j] * A->w[j] / (A->xi[j] - nu);
  }
  return (A->b - nu) - s;
}

/* The same function, its sum accumulated by Neumaier's compensated
 * summation, plus the derivative g' and the amplification estimate
 * kappa_g = (|b| + |nu| + |sum|)/(|nu| |g'|). */
static void g_comp(const arrow_t* A, double nu, double* g, double* gp, double* kap) {
  double s = 0.0, c = 0.0, sp = 0.0, sabs = 0.0;
  for (int64_t j = 0; j < A->n; ++j) {
    if (j == A->i) continue;
    double den = A->xi[j] - nu;
    double t = A->w[j] * A->w[j] / den;
    double u = s + t;
    if (fabs(s) >= fabs(t)) c += (s - u) + t; else c += (t - u) + s;
    s = u;
    sp += A->w[j] * A->w[j] / (den * den);
    sabs += fabs(t);
  }
  double S = s + c;
  *g = (A->b - nu) - S;
  *gp = -1.0 - sp;
  /* in two divisions: |nu| |g'| alone can overflow when nu nears 1e304 */
  *kap = ((fabs(A->b) + fabs(nu) + sabs) / fabs(nu)) / fabs(*gp);
}

/* g evaluated entirely in binary128 at a binary64 point nu, with the entries
 * of A_i^{-1} formed in binary128 from the binary64 data (double the
 * working precision, Sec. 2.3). */
static void g_quad(const double* d, const double* z, const arrow_t* A, double nu,
                   quad* g, quad* gp, quad* sabs) {
  quad zi = (quad)z[A->i];
  quad s = 0, sp = 0, sa = 0, nq = (quad)nu;
  for (int64_t j = 0; j < A->n; ++j) {
    if (j == A->i) continue;
    quad dl = (quad)d[j] - (quad)A->sigma;
    quad xi = 1 / dl;
    quad w = -(quad)z[j] / (zi * dl);
    quad den = xi - nq;
    quad t = w * w / den;
    s += t;
    sa += t < 0 ? -t : t;
    sp += w * w / (den * den);
  }
  *g = (A->bq - nq) - s;
  *gp = -1 - sp;
  if (sabs) *sabs = sa;
}

/* b from eq. (b_ob) in binary128: (1/zeta_i^2)(1/rho + sum_{j!=i} zeta_j^2/(d_j - sigma)). */
static quad b_quad(const double* d, const double* z, int64_t n, int64_t i, double sigma, double rho) {
  quad acc = 1 / (quad)rho;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    quad zj = (quad)z[j];
    acc += zj * zj / ((quad)d[j] - (quad)sigma);
  }
  quad zi = (quad)z[i];
  return acc / (zi * zi);
}

/* ----------------------------------------------------- one eigenpair */

/* One eigenpair; force_i >= 0 takes the shift pole d_{force_i} (k or k-1)
 * instead of Algorithm 1's test (remedy (R1)); nuq_out (nullable) receives
 * nu after one more Newton step with g in binary128, carried in binary128. */
static int dpr1eig_at(const double* d, const double* z, double rho, int64_t n, int64_t k,
                      const oracle_opts* opts_in, double* lambda_out, double* v_out,
                      oracle_eigdiag* dg_out, int64_t force_i, quad* nuq_out) {
  oracle_opts opts;
  if (opts_in) opts = *opts_in; else oracle_default_opts(&opts);
  oracle_eigdiag dg;
  memset(&dg, 0, sizeof dg);
  if (n < 1 || k < 0 || k >= n || !(rho > 0)) return ORC_EARG;

  if (n == 1) {
    /* The 1x1 case: A = d_1 + rho*zeta_1^2, v = x/|x| with x = zeta_1/(d_1 - lambda). */
    double mu = rho * z[0] * z[0];
    dg.i = 0; dg.side = 1; dg.sigma = d[0]; dg.mu = mu; dg.nu = 1.0 / mu;
    dg.lambda = d[0] + mu; dg.b = 1.0 / mu; dg.Kb = 1; dg.Kz = 0; dg.kappa_g = 1;
    dg.xnorm = fabs(z[0] / mu);
    if (lambda_out) *lambda_out = dg.lambda;
    if (v_out) v_out[0] = (z[0] > 0) ? -1.0 : 1.0;
    if (dg_out) *dg_out = dg;
    return ORC_OK;
  }

  /* Shift (Alg. 1): k=1 -> sigma = d_1; otherwise evaluate f at the midpoint
   * tau above d_k; F > 0 means the root lies below the midpoint, so d_k is
   * the nearest pole; otherwise (including F == 0) d_{k-1}. */
  int64_t i;
  int side;
  if (force_i >= 0) {
    i = force_i; side = (i == k) ? 1 : -1;
  } else if (k == 0) {
    i = 0; side = 1;
  } else {
    double tau = (d[k - 1] - d[k]) / 2;
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += z[j] * z[j] / ((d[j] - d[k]) - tau);
    double F = 1.0 + rho * s;
    if (F > 0) { i = k; side = 1; } else { i = k - 1; side = -1; }
  }
  double sigma = d[i];
  double zi = z[i];

  arrow_t A;
  A.n = n; A.i = i; A.sigma = sigma; A.rho = rho;
  A.delta = (double*)malloc(sizeof(double) * 3 * n);
  A.xi = A.delta + n;
  A.w = A.xi + n;
  for (int64_t j = 0; j < n; ++j) {
    A.delta[j] = d[j] - sigma;
    if (j == i) { A.xi[j] = 0; A.w[j] = 0; continue; }
    A.xi[j] = 1.0 / A.delta[j];
    A.w[j] = -z[j] / (zi * A.delta[j]);
  }

  /* b in binary64, summed as (1/rho + z_1^T D_1^{-1} z_1) + z_2^T D_2^{-1} z_2
   * with each partial sum in ascending j; the diagnostics of eq. (knu2). */
  double s1 = 0.0, s2 = 0.0, sz = 0.0;
  for (int64_t j = 0; j < i; ++j) s1 += z[j] * z[j] / A.delta[j];
  for (int64_t j = i + 1; j < n; ++j) s2 += z[j] * z[j] / A.delta[j];
  for (int64_t j = 0; j < n; ++j) if (j != i) sz += fabs(z[j]);
  double rzi = 1.0 / zi;                        /* eq. (b_ob): (1/zeta_i)^2 (...) */
  double b64 = ((1.0 / rho + s1) + s2) * (rzi * rzi);
  double P = rho * s1, N = rho * s2;           /* P > 0, N < 0 */
  double Kb64 = (1.0 + P - N) / fabs(1.0 + P + N);
  dg.Kz = sz / fabs(zi);

  A.bq = b_quad(d, z, n, i, sigma, rho);
  double Kb_acc = (1.0 + P - N) / fabs((double)(A.bq * (quad)rho * (quad)zi * (quad)zi));
  int use_ext;
  if (opts.mode_b == 0) use_ext = 1;
  else if (opts.mode_b == 1) use_ext = (Kb64 > 100.0);
  else if (opts.mode_b == 3) {
    /* Algorithm 1's gate: the bound of eq. (knu2) from the standard-precision
     * K_b, "much larger than O(n)" read as above 100 (n+4) sqrt(n), i.e.
     * K_b > 100 unless K_z shows that b cannot influence ||A_i^{-1}|| */
    double sn = sqrt((double)n);
    double k1 = (n + 4) * sn * Kb64, k2 = 3 * sn + (n + 4) * (1 + 2 * dg.Kz);
    use_ext = (k1 < k2 ? k1 : k2) > 100.0 * (n + 4) * sn;
  } else use_ext = 0;
  A.b = use_ext ? (double)A.bq : b64;
  if (!use_ext) A.bq = (quad)b64;   /* the polish then sees the b in use */
  /* An arrow entry whose square leaves binary64 (|w_j| >= 2^511), or a tip
   * beyond binary64: the secular function is carried in binary128. */
  int wide = !(fabs(A.b) < INFINITY);
  for (int64_t j = 0; j < n && !wide; ++j)
    if (j != i && !(fabs(A.w[j]) < 0x1p+511)) wide = 1;
  if (wide) {
    A.bq = b_quad(d, z, n, i, sigma, rho);
    A.b = (double)A.bq;
    use_ext = 1;
  }
  dg.used_ext_b = use_ext;
  dg.Kb = use_ext ? Kb_acc : Kb64;
  {
    double sn = sqrt((double)n);
    double k1 = (n + 4) * sn * dg.Kb;
    double k2 = 3 * sn + (n + 4) * (1 + 2 * dg.Kz);
    dg.kappa_nu_bound = k1 < k2 ? k1 : k2;
  }

  /* Bracket of the extreme eigenvalue nu of A_i^{-1}.  Rightmost (side +1):
   * nu > max xi_j; leftmost: nu < min xi_j.  The far end uses the 2x2
   * Loewner bound from Xi <= xi_max*I (resp. >= xi_min*I): the extreme
   * eigenvalue of [[x, ||w||], [||w||, b]], i.e. (b+x)/2 +- sqrt(h^2 + ||w||^2)
   * with h = (b-x)/2, written as max(b,x) + ||w||^2/(|h| + sqrt(h^2 + ||w||^2))
   * (resp. min(b,x) - ...) so that b never cancels against the square root:
   * with a tiny zeta_i, |b| can exceed nu by fifteen orders of magnitude.
   * The final sum can still cancel (for k = 1 when nu << |x|), so a bound on
   * its rounding error, 8 eps (|max(b,x)| + the quotient), is added.
   * Neither h^2 nor ||w||^2 is formed: with a tiny zeta_i, |b| and ||w|| can
   * exceed 1e154 (a squared 1e184 overflows and would collapse the bound
   * onto the pole), so the quotient is ||w|| (||w|| / (|h| + hypot(h, ||w||)))
   * with ||w|| summed scaled by its largest entry. */
  double wmax = 0.0, xmax = -INFINITY, xmin = INFINITY;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    if (fabs(A.w[j]) > wmax) wmax = fabs(A.w[j]);
    if (A.xi[j] > xmax) xmax = A.xi[j];
    if (A.xi[j] < xmin) xmin = A.xi[j];
  }
  double wn = 0.0;
  if (wmax > 0.0) {
    double acc = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double q = A.w[j] / wmax;
      acc += q * q;
    }
    wn = wmax * sqrt(acc);
  }
  const double grow = 1.0 + 0x1p-40;
  /* Far end of the bracket: the same 2x2 bound.  On the binary128 path it is
   * formed in binary128 from the exact shifted differences (||w|| can exceed
   * binary64 there) and rounded outwards; beyond binary64 it is the largest
   * finite number. */
  double far = 0.0;
  if (wide) {
    quad zq = (quad)zi, w2 = 0, xe = (side > 0) ? -(quad)INFINITY : (quad)INFINITY;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      quad dl = (quad)d[j] - (quad)sigma;
      quad wq = (quad)z[j] / (zq * dl);
      w2 += wq * wq;
      quad xq = 1 / dl;
      if (side > 0 ? xq > xe : xq < xe) xe = xq;
    }
    quad wnq = sqrtq(w2);
    quad hq = fabsq(A.bq - xe) / 2;
    quad mq = (side > 0) ? (A.bq > xe ? A.bq : xe) : (A.bq < xe ? A.bq : xe);
    quad tq = wnq > 0 ? wnq * (wnq / (hq + sqrtq(hq * hq + wnq * wnq))) : 0;
    quad fq = (side > 0) ? (mq + tq) * (1 + (quad)0x1p-100) : (mq - tq) * (1 + (quad)0x1p-100);
    if (fq > (quad)DBL_MAX) far = DBL_MAX;
    else if (fq < -(quad)DBL_MAX) far = -DBL_MAX;
    else far = (double)fq * (side > 0 ? (fq > 0 ? grow : 1 / grow) : (fq < 0 ? grow : 1 / grow));
  }
  double L, U;
  if (side > 0) {
    double h = fabs(A.b - xmax) / 2;
    double m = fmax(A.b, xmax), t = wn > 0.0 ? wn * (wn / (h + hypot(h, wn))) : 0.0;
    U = wide ? far : (m + t) * grow + 8 * DBL_EPSILON * (fabs(m) + t);
    if (k == 0) {
      /* lambda_1 lies in [d_1 + rho*zeta_1^2, d_1 + rho*||z||^2]. */
      double zz = 0.0;
      for (int64_t j = 0; j < n; ++j) zz += z[j] * z[j];
      L = (1.0 / (rho * zz)) / grow;
      double Ub = (1.0 / (rho * zi * zi)) * grow;
      if (Ub < U || !(U > L)) U = Ub;
    } else {
      L = xmax;              /* the pole nearest to nu, never evaluated */
    }
  } else {
    double h = fabs(A.b - xmin) / 2;
    double m = fmin(A.b, xmin), t = wn > 0.0 ? wn * (wn / (h + hypot(h, wn))) : 0.0;
    L = wide ? far : (m - t) * grow - 8 * DBL_EPSILON * (fabs(m) + t);
    U = xmin;
  }
  const double L0 = L, U0 = U;

  /* Bisection on g (decreasing on the bracket): g(mid) > 0 -> root above. */
  int it = 0;
  while (!adjacent(L, U) && it < 200) {
    double m = fmid(L, U);
    int up;
    if (wide) {
      quad gq, gpq;
      g_quad(d, z, &A, m, &gq, &gpq, NULL);
      up = gq > 0;
    } else {
      up = g_plain(&A, m) > 0;
    }
    if (up) L = m; else U = m;
    ++it;
  }
  dg.bisect_iters = it;
  double nu0 = (side > 0) ? U : L;   /* the end that is not a pole */

  /* One Newton step with a compensated sum (binary128 on the wide path). */
  double g, gp, kap, nu;
  if (wide) {
    quad gq, gpq, sa;
    g_quad(d, z, &A, nu0, &gq, &gpq, &sa);
    quad nq0 = (quad)nu0, anu = nq0 < 0 ? -nq0 : nq0, agp = gpq < 0 ? -gpq : gpq;
    nu = (double)(nq0 - gq / gpq);
    kap = (double)((fabsq(A.bq) + anu + sa) / (anu * agp));
  } else {
    g_comp(&A, nu0, &g, &gp, &kap);
    nu = nu0 - g / gp;
  }
  dg.kappa_g = kap;
  double mu = 1.0 / nu;
  double lam = sigma + mu;
  double amp = fabs(mu / lam);
  if (!(amp > 1.0)) amp = 1.0;

  if (opts.polish && kap * amp > opts.kappa_polish) {
    /* Safeguarded Newton on g evaluated in binary128.  The bracket is the
     * rigorous initial one, narrowed by the signs of the binary128 g. */
    double lo = L0, hi = U0;
    double cur = nu;
    if (!(cur >= lo && cur <= hi)) cur = nu0;
    int pit = 0;
    for (; pit < 100; ++pit) {
      quad gq, gpq;
      g_quad(d, z, &A, cur, &gq, &gpq, NULL);
      if (gq == 0) break;
      if (gq > 0) lo = cur; else hi = cur;
      double t = (double)((quad)cur - gq / gpq);
      if (!(t >= lo && t <= hi)) t = fmid(lo, hi);
      if (t == cur) break;
      cur = t;
    }
    nu = cur;
    dg.polished = 1;
    dg.polish_iters = pit;
    mu = 1.0 / nu;
    lam = sigma + mu;
  }
  if (nuq_out) {
    quad gq, gpq;
    g_quad(d, z, &A, nu, &gq, &gpq, NULL);
    *nuq_out = (quad)nu - gq / gpq;
  }

  /* Near-zero eigenvalue (eq. gamma): lambda much closer to zero than to its
   * neighbouring poles.  Then all poles are non-zero and lambda = 1/eta with
   * eta the extreme eigenvalue of A^{-1} = D^{-1} + gamma D^{-1} z z^T D^{-1},
   * gamma = -rho/(1 + rho z^T D^{-1} z), the denominator f(0) evaluated in
   * binary128. */
  double gapnb = fabs(lam - d[k]);
  if (k > 0 && fabs(lam - d[k - 1]) < gapnb) gapnb = fabs(lam - d[k - 1]);
  if (opts.nearzero > 0 && opts.nearzero * fabs(lam) < gapnb) {
    dg.nearzero = 1;
    quad f0q = 1;
    for (int64_t j = 0; j < n; ++j) {
      quad zj = (quad)z[j];
      f0q += (quad)rho * zj * zj / (quad)d[j];
    }
    double f0 = (double)f0q;
    if (f0 == 0.0) {
      dg.singular = 1;
      lam = 0.0;
    } else {
      double gam = -rho / f0;
      /* DPR1 secular function of A^{-1}: h(eta) = 1 + gamma*sum u_j^2/(e_j - eta),
       * e_j = 1/d_j, u_j = zeta_j/d_j. */
      double* e = (double*)malloc(sizeof(double) * 2 * n);
      double* u = e + n;
      double emax = -INFINITY, emin = INFINITY, emag = 0, uu = 0;
      for (int64_t j = 0; j < n; ++j) {
        e[j] = 1.0 / d[j];
        u[j] = z[j] / d[j];
        if (e[j] > emax) emax = e[j];
        if (e[j] < emin) emin = e[j];
        if (fabs(e[j]) > emag) emag = fabs(e[j]);
        uu += u[j] * u[j];
      }
      double ub = (emag + fabs(gam) * uu) * grow;   /* |eta| <= ||A^{-1}|| */
      int pos = (f0 < 0);                           /* lambda > 0 iff f(0) < 0 */
      /* for k = 1 with all poles negative the right branch starts at 0+ */
      double lo = pos ? (emax > 0 ? emax : 4.9406564584124654e-324) : -ub;
      double hi = pos ? ub : (emin < 0 ? emin : -4.9406564584124654e-324);
      int hit = 0;
      while (!adjacent(lo, hi) && hit < 200) {
        double m = fmid(lo, hi);
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += u[j] * u[j] / (e[j] - m);
        double hv = 1.0 + gam * s;
        /* h increases on the right branch and decreases on the left one */
        if ((hv < 0) == pos) lo = m; else hi = m;
        ++hit;
      }
      double eta0 = pos ? hi : lo;
      /* one compensated Newton step, as for nu */
      double s = 0.0, c = 0.0, sp = 0.0;
      for (int64_t j = 0; j < n; ++j) {
        double den = e[j] - eta0;
        double t = u[j] * u[j] / den;
        double y = s + t;
        if (fabs(s) >= fabs(t)) c += (s - y) + t; else c += (t - y) + s;
        s = y;
        sp += u[j] * u[j] / (den * den);
      }
      double hv = 1.0 + gam * (s + c);
      double hp = gam * sp;
      double eta = eta0 - hv / hp;
      lam = 1.0 / eta;
      free(e);
    }
  }

  /* Eigenvector (eq. eigenvecAi): x_j = zeta_j/(delta_j - mu), x_i = -zeta_i/mu,
   * v = x/||x||_2 with the norm accumulated in binary128. */
  quad nq = 0;
  for (int64_t j = 0; j < n; ++j) {
    double xj = (j == i) ? -zi / mu : z[j] / (A.delta[j] - mu);
    nq += (quad)xj * (quad)xj;
  }
  double xn = (double)sqrtq(nq);
  if (v_out) {
    for (int64_t j = 0; j < n; ++j) {
      double xj = (j == i) ? -zi / mu : z[j] / (A.delta[j] - mu);
      v_out[j] = xj / xn;
    }
  }
  dg.i = (int32_t)i; dg.side = side; dg.sigma = sigma;
  dg.mu = mu; dg.nu = nu; dg.lambda = lam; dg.b = A.b; dg.xnorm = xn;
  if (lambda_out) *lambda_out = lam;
  if (dg_out) *dg_out = dg;
  free(A.delta);
  return ORC_OK;
}

int oracle_dpr1eig(const double* d, const double* z, double rho, int64_t n, int64_t k,
                   const oracle_opts* opts_in, double* lambda_out, double* v_out,
                   oracle_eigdiag* dg_out) {
  return dpr1eig_at(d, z, rho, n, k, opts_in, lambda_out, v_out, dg_out, -1, NULL);
}

/* ------------------------------------------------- K_nu and the remedies */
/* ||A_i^{-1}||_2 = 1/min_j |lambda_j - d_i|, and by the interlacing
 * (eq. interlace) the minimum is taken at one of the two eigenvalues beside
 * the pole d_i: lambda_k itself or lambda_o, o = k+1 when i = k, o = k-1 when
 * i = k-1.  So K_nu of eq. (K0) for eigenpair k shifted to d_i is
 * |lambda_k - d_i| / min(|lambda_k - d_i|, |lambda_o - d_i|), the distances
 * taken from the shifted representations (sigma_j, mu_j) in binary128.  For
 * a pole p other than the shift, the same with |lambda_k - d_p|. */
static double knu_at(const double* d, int64_t n, const oracle_eigdiag* dg, int64_t k, int64_t p) {
  quad lk = fabsq(((quad)dg[k].sigma - (quad)d[p]) + (quad)dg[k].mu);
  int64_t o = (p == k) ? k + 1 : k - 1;   /* the other eigenvalue beside d_p */
  if (o < 0 || o >= n || lk == 0) return 1.0;
  quad lo = fabsq(((quad)dg[o].sigma - (quad)d[p]) + (quad)dg[o].mu);
  if (lo >= lk) return 1.0;
  return lo > 0 ? (double)(lk / lo) : INFINITY;
}

/* v = x/||x||, x_j = zeta_j/((d_j - d_i) - mu) (eq. eigenvecAi) for the
 * shifted representation (i, mu); ||x|| accumulated in binary128. */
static double vector_from(const double* d, const double* z, int64_t n, int64_t i, double mu, double* v) {
  quad nq = 0;
  for (int64_t j = 0; j < n; ++j) {
    double xj = (j == i) ? -z[i] / mu : z[j] / ((d[j] - d[i]) - mu);
    nq += (quad)xj * (quad)xj;
  }
  double xn = (double)sqrtq(nq);
  if (v)
    for (int64_t j = 0; j < n; ++j) {
      double xj = (j == i) ? -z[i] / mu : z[j] / ((d[j] - d[i]) - mu);
      v[j] = xj / xn;
    }
  return xn;
}

/* Remedy (R2): invert A - sigma I with sigma between d_i and lambda, near
 * lambda (sigma = d_i + mu (1 - t), in binary128), so that lambda - sigma is the
 * eigenvalue of A - sigma I closest to zero.  Its inverse is the DPR1 matrix
 * E + gamma u u^T with e_j = 1/(d_j - sigma), u_j = zeta_j e_j,
 * gamma = -rho/f(sigma), f(sigma) = 1 + rho sum zeta_j^2/(d_j - sigma) (the
 * same form as eq. gamma, shifted), everything in binary128 (remedy (R2)
 * forms this matrix in extended precision).  eta = 1/(lambda -
 * sigma) is its exterior eigenvalue: the root of h(eta) = 1 + gamma sum
 * u_j^2/(e_j - eta) right of every e_j when mu > 0 (then f(sigma) < 0), left of
 * every e_j when mu < 0.  Returns mu_new = lambda - d_i = (sigma - d_i) + 1/eta,
 * or NaN when no sigma on the right side of lambda is found. */
static double remedy_r2(const double* d, const double* z, double rho, int64_t n, int64_t i, double mu) {
  const int pos = mu > 0;
  for (int e = 20; e >= 2; e -= 6) {
    const quad ms = (quad)mu * (1 - ldexpq(1, -e));   /* sigma - d_i */
    const quad sg = (quad)d[i] + ms;
    quad f = 1, uu = 0, emax = -(quad)INFINITY, emin = (quad)INFINITY, emag = 0;
    for (int64_t j = 0; j < n; ++j) {
      quad dl = (quad)d[j] - sg;
      quad zj = (quad)z[j];
      f += (quad)rho * zj * zj / dl;
      quad ej = 1 / dl, uj = zj / dl;
      uu += uj * uj;
      if (ej > emax) emax = ej;
      if (ej < emin) emin = ej;
      if (fabsq(ej) > emag) emag = fabsq(ej);
    }
    if (pos ? !(f < 0) : !(f > 0)) continue;      /* sigma is not between d_i and lambda */
    const quad gam = -(quad)rho / f;
    const quad ub = (emag + fabsq(gam) * uu) * (1 + ldexpq(1, -40));
    /* bisection on the binary64 numbers of eta, h in binary128 */
    /* eta has the sign of mu: the bracket stays on that side of 0 */
    double lo, hi;
    if (pos) {
      lo = nextafter(emax > 0 ? (double)emax : 0.0, INFINITY);
      hi = nextafter((double)ub, INFINITY);
    } else {
      lo = nextafter(-(double)ub, -INFINITY);
      hi = nextafter(emin < 0 ? (double)emin : -0.0, -INFINITY);
    }
    for (int it = 0; it < 200 && !adjacent(lo, hi); ++it) {
      double m = fmid(lo, hi);
      quad hsum = 0;
      for (int64_t j = 0; j < n; ++j) {
        quad dl = (quad)d[j] - sg;
        quad ej = 1 / dl, uj = (quad)z[j] / dl;
        hsum += uj * uj / (ej - (quad)m);
      }
      quad h = 1 + gam * hsum;
      /* right branch (gamma > 0): h rises from -inf to 1, the root is above m
       * where h < 0; left branch (gamma < 0): h falls from 1 to -inf, the root
       * is above m where h > 0 */
      if (pos ? (h < 0) : (h > 0)) lo = m; else hi = m;
    }
    /* one Newton step in binary128 from the bracket end away from the poles */
    quad et = pos ? (quad)hi : (quad)lo, hs = 0, hp = 0;
    for (int64_t j = 0; j < n; ++j) {
      quad dl = (quad)d[j] - sg;
      quad ej = 1 / dl, uj = (quad)z[j] / dl, den = ej - et;
      hs += uj * uj / den;
      hp += uj * uj / (den * den);
    }
    et = et - (1 + gam * hs) / (gam * hp);
    return (double)(ms + 1 / et);
  }
  return NAN;
}

/* ------------------------------------------------------- all eigenpairs */
/* rho < 0 is reduced to rho > 0 as in Sec. 1: the eigenpairs of
 * D + rho z z^T are those of -((-D) + (-rho) z z^T); -D is put back in
 * decreasing order by reversing the index. */

int oracle_dpr1eig_all(const double* d, const double* z, double rho, int64_t n,
                       const oracle_opts* opts, double* lambda, double* V, int64_t ldv,
                       oracle_eigdiag* diags, int nthreads) {
  int rc = oracle_check(d, z, rho, n);
  if (rc != ORC_OK) return rc;
  if (V && ldv < n) return ORC_EARG;
  oracle_opts op;
  if (opts) op = *opts; else oracle_default_opts(&op);
  const double* dd = d;
  const double* zz = z;
  double r = rho;
  double *dn = NULL, *zn = NULL;
  int neg = rho < 0;
  if (neg) {
    dn = (double*)malloc(sizeof(double) * 2 * n);
    zn = dn + n;
    for (int64_t j = 0; j < n; ++j) { dn[j] = -d[n - 1 - j]; zn[j] = z[n - 1 - j]; }
    dd = dn; zz = zn; r = -rho;
  }
  /* diagnostics in the order of the solved problem (rho > 0) */
  oracle_eigdiag* dgs = (oracle_eigdiag*)calloc((size_t)n, sizeof(oracle_eigdiag));
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    double* v = V ? (double*)malloc(sizeof(double) * n) : NULL;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
    for (int64_t k = 0; k < n; ++k) {
      double lam;
      oracle_dpr1eig(dd, zz, r, n, k, &op, &lam, v, &dgs[k]);
      int64_t ko = neg ? n - 1 - k : k;
      lambda[ko] = neg ? -lam : lam;
      if (V) {
        if (neg) for (int64_t j = 0; j < n; ++j) V[ko * ldv + (n - 1 - j)] = -v[j];
        else for (int64_t j = 0; j < n; ++j) V[ko * ldv + j] = v[j];
      }
    }
    free(v);
  }
  /* K_nu of eq. (K0) for every eigenpair, from its neighbours' shifted
   * representations; with opts.remedy, Algorithm 1's last branch: where
   * K_nu > knu_thr, remedy (R1) -- the other neighbouring pole, when its K_nu
   * is smaller and below the threshold -- else remedy (R2).  The remedied
   * eigenvalue is then represented from its nearest pole d_i again (mu =
   * lambda - d_i in binary128), and v and ||x|| are recomputed from it. */
  double* kn = (double*)malloc(sizeof(double) * n);
  for (int64_t k = 0; k < n; ++k) kn[k] = (n > 1) ? knu_at(dd, n, dgs, k, dgs[k].i) : 1.0;
  for (int64_t k = 0; k < n; ++k) dgs[k].Knu = kn[k];
  if (op.remedy && n > 1) {
    int64_t* todo = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t nt = 0;
    for (int64_t k = 0; k < n; ++k)
      if (kn[k] > op.knu_thr && !dgs[k].nearzero) todo[nt++] = k;   /* eq. (gamma) keeps its lambda */
    oracle_eigdiag* upd = (oracle_eigdiag*)malloc(sizeof(oracle_eigdiag) * (nt > 0 ? nt : 1));
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
      double* v = V ? (double*)malloc(sizeof(double) * n) : NULL;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
      for (int64_t t = 0; t < nt; ++t) {
        const int64_t k = todo[t];
        oracle_eigdiag g = dgs[k];
        const int64_t i = g.i;
        const int64_t p = (i == k) ? k - 1 : k;   /* the other neighbouring pole */
        double mu_new = NAN;
        int how = 0;
        if (k >= 1 && p >= 0 && knu_at(dd, n, dgs, k, p) < kn[k] && knu_at(dd, n, dgs, k, p) <= op.knu_thr) {
          /* (R1): eigenpair k with the shift at d_p.  mu_i = (d_p - d_i) +
           * mu_p carries the absolute error of mu_p, |mu_p/mu_i| times larger
           * relative to mu_i, so nu_p is refined and carried in binary128 */
          oracle_eigdiag gp;
          double lp;
          quad nuq = 0;
          oracle_opts o1 = op;
          o1.polish = 1;
          o1.kappa_polish = 0.0;
          dpr1eig_at(dd, zz, r, n, k, &o1, &lp, NULL, &gp, p, &nuq);
          mu_new = (double)(((quad)dd[p] - (quad)dd[i]) + 1 / nuq);
          how = 1;
        } else {
          mu_new = remedy_r2(dd, zz, r, n, i, g.mu);
          how = 2;
        }
        if (mu_new == mu_new && mu_new != 0.0) {
          g.mu = mu_new;
          g.nu = 1.0 / mu_new;
          g.lambda = (double)((quad)dd[i] + (quad)mu_new);
          g.remedied = how;
          g.xnorm = vector_from(dd, zz, n, i, mu_new, v);
          const int64_t ko = neg ? n - 1 - k : k;
          lambda[ko] = neg ? -g.lambda : g.lambda;
          if (V) {
            if (neg) for (int64_t j = 0; j < n; ++j) V[ko * ldv + (n - 1 - j)] = -v[j];
            else for (int64_t j = 0; j < n; ++j) V[ko * ldv + j] = v[j];
          }
        }
        upd[t] = g;
      }
      free(v);
    }
    for (int64_t t = 0; t < nt; ++t) dgs[todo[t]] = upd[t];
    free(upd);
    free(todo);
  }
  if (diags)
    for (int64_t k = 0; k < n; ++k) diags[neg ? n - 1 - k : k] = dgs[k];
  free(kn);
  free(dgs);
  free(dn);
  return ORC_OK;
}

/* Eigenvalues only, for a bounded sample of indices (used to time the oracle
 * on a slice of a large problem). */
int oracle_dpr1eig_some(const double* d, const double* z, double rho, int64_t n,
                        const int64_t* ks, int64_t nk, const oracle_opts* opts,
                        double* lambda, double* V, int64_t ldv, oracle_eigdiag* diags,
                        int nthreads) {
  int rc = oracle_check(d, z, rho, n);
  if (rc != ORC_OK) return rc;
  if (!(rho > 0)) return ORC_EARG;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t t = 0; t < nk; ++t) {
    oracle_eigdiag dg;
    oracle_dpr1eig(d, z, rho, n, ks[t], opts, &lambda[t], V ? V + t * ldv : NULL, &dg);
    if (diags) diags[t] = dg;
  }
  return ORC_OK;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ----------------------------------------------------------- backward */
/* Reverse-mode derivative of L(Lambda, V) through A = D + rho z z^T.
 * Standard first-order perturbation of a symmetric eigendecomposition with
 * simple eigenvalues:  d lambda_k = v_k^T dA v_k,
 * d v_k = sum_{l != k} v_l (v_l^T dA v_k)/(lambda_k - lambda_l).
 * Hence Abar = V X V^T with X = diag(Lambda_bar) + F o (V^T V_bar),
 * F_lk = 1/(lambda_k - lambda_l) (l != k), and with
 * dA = diag(dd) + drho z z^T + rho (dz z^T + z dz^T):
 *   d_bar_j = Abar_jj,  rho_bar = z^T Abar z,  z_bar = rho (Abar + Abar^T) z.
 * The gaps lambda_k - lambda_l come from the shifted representation
 * (sigma_k + mu_k) - (sigma_l + mu_l) carried in binary128.  Abar is formed
 * explicitly with long double accumulation: O(n^3), for checking only.
 * V is column-major with leading dimension n; lambda_bar or V_bar may be NULL. */
int oracle_dpr1_backward(const double* d, const double* z, double rho, int64_t n,
                         const double* sigma, const double* mu, const double* V,
                         const double* lambda_bar, const double* V_bar,
                         double* d_bar, double* z_bar, double* rho_bar, int nthreads) {
  (void)d;
  long double* X = (long double*)calloc((size_t)n * n, sizeof(long double));
  long double* Ab = (long double*)calloc((size_t)n * n, sizeof(long double));
  long double* T = (long double*)calloc((size_t)n * n, sizeof(long double));
  if (!X || !Ab || !T) { free(X); free(Ab); free(T); return ORC_EARG; }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  /* X[l,k] (column-major, X[l + k n]) */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t k = 0; k < n; ++k) {
    for (int64_t l = 0; l < n; ++l) {
      if (l == k) {
        X[l + k * n] = lambda_bar ? (long double)lambda_bar[k] : 0.0L;
        continue;
      }
      if (!V_bar) continue;
      long double p = 0;
      for (int64_t j = 0; j < n; ++j) p += (long double)V[j + l * n] * (long double)V_bar[j + k * n];
      quad gap = ((quad)sigma[k] - (quad)sigma[l]) + ((quad)mu[k] - (quad)mu[l]);
      X[l + k * n] = p / (long double)gap;
    }
  }
  /* T = V X */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j) {
      long double s = 0;
      for (int64_t l = 0; l < n; ++l) s += (long double)V[j + l * n] * X[l + k * n];
      T[j + k * n] = s;
    }
  /* Abar = T V^T */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t m = 0; m < n; ++m)
    for (int64_t j = 0; j < n; ++j) {
      long double s = 0;
      for (int64_t k = 0; k < n; ++k) s += T[j + k * n] * (long double)V[m + k * n];
      Ab[j + m * n] = s;
    }
  long double rb = 0;
  for (int64_t j = 0; j < n; ++j) {
    d_bar[j] = (double)Ab[j + j * n];
    long double zs = 0;
    for (int64_t m = 0; m < n; ++m) {
      rb += (long double)z[j] * Ab[j + m * n] * (long double)z[m];
      zs += (Ab[j + m * n] + Ab[m + j * n]) * (long double)z[m];
    }
    z_bar[j] = (double)((long double)rho * zs);
  }
  *rho_bar = (double)rb;
  free(X); free(Ab); free(T);
  return ORC_OK;
}

/* The tip b of A_i^{-1} (eq. b_ob) for a given shift index i: mode 0 in
 * binary128 (rounded once to binary64), mode 2 in binary64 summed as
 * (1/rho + z_1^T D_1^{-1} z_1) + z_2^T D_2^{-1} z_2 and scaled by (1/zeta_i)^2
 * (this order reproduces the standard-precision b printed in Example 3
 * bit for bit).  Also returns K_b (knu2). */
int oracle_tip(const double* d, const double* z, double rho, int64_t n, int64_t i,
               int32_t mode, double* b_out, double* Kb_out) {
  if (n < 2 || i < 0 || i >= n) return ORC_EARG;
  double sigma = d[i], zi = z[i];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t j = 0; j < i; ++j) s1 += z[j] * z[j] / (d[j] - sigma);
  for (int64_t j = i + 1; j < n; ++j) s2 += z[j] * z[j] / (d[j] - sigma);
  double P = rho * s1, N = rho * s2;
  quad bq = b_quad(d, z, n, i, sigma, rho);
  if (mode == 0) {
    *b_out = (double)bq;
    *Kb_out = (1.0 + P - N) / fabs((double)(bq * (quad)rho * (quad)zi * (quad)zi));
  } else {
    double rzi = 1.0 / zi;
    *b_out = ((1.0 / rho + s1) + s2) * (rzi * rzi);
    *Kb_out = (1.0 + P - N) / fabs(1.0 + P + N);
  }
  return ORC_OK;
}
