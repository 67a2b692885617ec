/* Host sanitizer driver for the CPU oracle (oracle/cme_oracle.c): built
 * together with the oracle source under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitizers.py, it calls every
 * exported routine on a small ragged batch (sizes 16, 1, 64, 7: powers of
 * two and not, one mode alone), with and without threads, so that an
 * out-of-bounds access, a use of freed memory or undefined arithmetic in
 * the oracle's indexing aborts the run.  Test infrastructure only. */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;
typedef struct {
  int32_t n, reserved;
  int64_t offset;
  double kappa_ext, g0, ain_re, ain_im, sigma0, sigma1, tau_ramp;
} orc_instance;

void orc_set_threads(int n);
int orc_max_threads(void);
int orc_fwm(int n, const cplx *a, cplx *K, int truncated);
int orc_kerr_vjp(int n, const cplx *u, const cplx *w, cplx *v);
double orc_sigma(const orc_instance *p, double t);
int orc_rhs(const orc_instance *p, const double *kappa, const double *omega, double t,
            const cplx *u, cplx *f, int truncated);
int orc_run(int batch, const orc_instance *inst, const double *kappa, const double *omega,
            double h, int64_t step0, int64_t n_steps, cplx *y, int truncated, int ckpt_every,
            cplx *ckpt, int64_t total);
int orc_adjoint(int batch, const orc_instance *inst, const double *kappa, const double *omega,
                double h, int64_t step0, int64_t n_steps, const cplx *y0, const cplx *gT,
                cplx *gy0, double *g_omega, double *g_kappa, cplx *g_ain);
int orc_split_step_run(int batch, const orc_instance *inst, const double *kappa,
                       const double *omega, double h, int64_t step0, int64_t n_steps, cplx *y);
double orc_sigma_integral(const orc_instance *p, double a, double b);
int orc_rk4ip_run(int batch, const orc_instance *inst, const double *kappa, const double *omega,
                  double h, int64_t step0, int64_t n_steps, cplx *y);

static double urand(unsigned *s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0 - 0.5;
}

#define CHECK(x)                                                   \
  do {                                                             \
    if ((x) != 0) {                                                \
      fprintf(stderr, "FAILED: %s (line %d)\n", #x, __LINE__);     \
      return 1;                                                    \
    }                                                              \
  } while (0)

int main(void) {
  const int sizes[4] = {16, 1, 64, 7};
  const int B = 4;
  orc_instance inst[4];
  int64_t total = 0;
  for (int b = 0; b < B; ++b) {
    orc_instance x = {sizes[b], 0, total, 0.5, 1.0, 0.6, -0.2, 0.5, 1.5, 0.01};
    inst[b] = x;
    total += sizes[b];
  }
  unsigned seed = 13073428u;
  /* exact-size heap arrays: any overrun is caught */
  double *kap = malloc(sizeof(double) * total), *om = malloc(sizeof(double) * total);
  cplx *y = malloc(sizeof(cplx) * total), *y0 = malloc(sizeof(cplx) * total);
  cplx *gT = malloc(sizeof(cplx) * total), *gy0 = malloc(sizeof(cplx) * total);
  double *g_om = calloc(total, sizeof(double)), *g_ka = calloc(total, sizeof(double));
  cplx *g_ain = calloc(B, sizeof(cplx));
  const int steps = 6, every = 2;
  cplx *ck = malloc(sizeof(cplx) * total * (steps / every));
  for (int64_t i = 0; i < total; ++i) {
    kap[i] = 1.0 + 0.1 * urand(&seed);
    om[i] = urand(&seed);
    y0[i] = 0.3 * urand(&seed) + 0.3 * I * urand(&seed);
    gT[i] = urand(&seed) + I * urand(&seed);
  }
  for (int threads = 1; threads <= 4; threads += 3) {
    orc_set_threads(threads);
    for (int b = 0; b < B; ++b) {
      const int n = sizes[b];
      cplx *K = malloc(sizeof(cplx) * n), *v = malloc(sizeof(cplx) * n);
      cplx *f = malloc(sizeof(cplx) * n);
      const cplx *a = y0 + inst[b].offset;
      CHECK(orc_fwm(n, a, K, 0));
      CHECK(orc_fwm(n, a, K, 1));
      CHECK(orc_kerr_vjp(n, a, gT + inst[b].offset, v));
      CHECK(orc_rhs(&inst[b], kap + inst[b].offset, om + inst[b].offset, 0.003, a, f, 0));
      CHECK(orc_rhs(&inst[b], kap + inst[b].offset, om + inst[b].offset, 0.003, a, f, 1));
      if (!isfinite(orc_sigma(&inst[b], 0.2)) || !isfinite(orc_sigma_integral(&inst[b], 0.0, 0.2)))
        return 1;
      free(K);
      free(v);
      free(f);
    }
    for (int tr = 0; tr < 2; ++tr) {
      for (int64_t i = 0; i < total; ++i) y[i] = y0[i];
      CHECK(orc_run(B, inst, kap, om, 1e-3, 3, steps, y, tr, every, ck, total));
    }
    CHECK(orc_adjoint(B, inst, kap, om, 1e-3, 3, steps, y0, gT, gy0, g_om, g_ka, g_ain));
    for (int64_t i = 0; i < total; ++i) y[i] = y0[i];
    CHECK(orc_split_step_run(B, inst, kap, om, 1e-3, 3, steps, y));
    for (int64_t i = 0; i < total; ++i) y[i] = y0[i];
    CHECK(orc_rk4ip_run(B, inst, kap, om, 1e-3, 3, steps, y));
  }
  for (int64_t i = 0; i < total; ++i)
    if (!isfinite(creal(y[i])) || !isfinite(cimag(y[i])) || !isfinite(g_om[i])) return 1;
  /* invalid arguments are refused, not dereferenced */
  if (orc_run(B, inst, kap, om, -1.0, 0, steps, y, 0, 0, NULL, total) == 0) return 1;
  free(kap);
  free(om);
  free(y);
  free(y0);
  free(gT);
  free(gy0);
  free(g_om);
  free(g_ka);
  free(g_ain);
  free(ck);
  printf("oracle sanitizer driver: ok\n");
  return 0;
}
