/* Sanitizer run of the CPU oracle (host code only): every entry point on a few small problems,
 * including rho < 0, the exterior eigenvalue, clustered poles and tiny z_i.  Built with
 * -fsanitize=address,undefined by test_oracle_sanitized.py; prints "ok" and returns 0 when no
 * invariant fails (the sanitizers abort on their own findings). */
#include "../oracle/dpr1_oracle.c"

#include <stdio.h>

static double uni(uint64_t* s) {
  *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(*s >> 11) * 0x1.0p-53;
}

static int run_case(int64_t n, double rho, uint64_t seed, int graded) {
  double* d = malloc(sizeof(double) * n);
  double* z = malloc(sizeof(double) * n);
  double* lam = malloc(sizeof(double) * n);
  double* V = malloc(sizeof(double) * n * n);
  double* lb = malloc(sizeof(double) * n);
  double* Vb = malloc(sizeof(double) * n * n);
  double *sg = malloc(sizeof(double) * n), *mu = malloc(sizeof(double) * n);
  double *db = malloc(sizeof(double) * n), *zb = malloc(sizeof(double) * n), rb = 0.0;
  oracle_eigdiag* dg = malloc(sizeof(oracle_eigdiag) * n);
  int bad = 0;
  for (int64_t j = 0; j < n; ++j) {
    d[j] = graded ? pow(10.0, -8.0 * (double)j / (double)(n > 1 ? n - 1 : 1)) : 1.0 - 2.0 * ((double)j + 0.5 * uni(&seed)) / (double)n;
    double m = pow(10.0, -6.0 * uni(&seed));
    z[j] = (uni(&seed) < 0.5 ? -m : m);
    lb[j] = uni(&seed) - 0.5;
  }
  if (graded && n > 4) d[3] = d[2] * (1.0 - 1e-10);
  for (int64_t t = 0; t < n * n; ++t) Vb[t] = uni(&seed) - 0.5;
  int rc = oracle_dpr1eig_all(d, z, rho, n, NULL, lam, V, n, dg, 2);
  if (rc != 0) bad = 1;
  for (int64_t k = 0; !bad && k + 1 < n; ++k)
    if (!(lam[k] > lam[k + 1])) bad = 2;
  for (int64_t k = 0; !bad && k < n; ++k) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += V[k * n + j] * V[k * n + j];
    if (fabs(s - 1.0) > 1e-12) bad = 3;
  }
  int64_t ks[3] = {0, n / 2, n - 1};
  double lam3[3], V3[3 * 64];
  /* the sampled entry point takes rho > 0 only */
  if (!bad && rho > 0 && n <= 64 && oracle_dpr1eig_some(d, z, rho, n, ks, 3, NULL, lam3, V3, n, NULL, 1) != 0) bad = 4;
  for (int64_t k = 0; k < n; ++k) {
    double sgn = rho > 0 ? 1.0 : -1.0;
    sg[k] = sgn * dg[k].sigma;
    mu[k] = sgn * dg[k].mu;
  }
  if (!bad && oracle_dpr1_backward(d, z, rho, n, sg, mu, V, lb, Vb, db, zb, &rb, 2) != 0) bad = 5;
  double b = 0.0, kb = 0.0;
  if (!bad && n >= 2 && oracle_tip(d, z, fabs(rho), n, n / 2, 0, &b, &kb) != 0) bad = 6;
  if (bad) printf("case n=%lld rho=%g graded=%d failed: %d\n", (long long)n, rho, graded, bad);
  free(d); free(z); free(lam); free(V); free(lb); free(Vb); free(sg); free(mu); free(db); free(zb); free(dg);
  return bad;
}

int main(void) {
  const int64_t ns[] = {1, 2, 3, 17, 64, 129};
  const double rhos[] = {1.0, -0.7, 10.0, 1e-3};
  int bad = 0;
  uint64_t seed = 12345;
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 4; ++b)
      for (int g = 0; g < 2; ++g) bad |= run_case(ns[a], rhos[b], seed++, g);
  if (bad) return 1;
  printf("ok\n");
  return 0;
}
