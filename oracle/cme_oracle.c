/*
 * cme_oracle.c -- plain FP64 CPU reference for the Kerr-comb coupled mode
 * equations (CME) of Hansson, Modotto & Wabnitz, arXiv:1307.3428.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP solver; the only thing the two have in
 * common is the seeded input arrays they are handed.
 *
 * What it computes, and where each piece comes from:
 *
 *   - Four-wave-mixing (FWM) sum of Eq. (1)/(2):
 *         K_mu = sum over alpha - beta + gamma = mu of A_alpha conj(A_beta) A_gamma,
 *     evaluated through the index rewrite of Eq. (3) as two correlations:
 *         C_k  = sum_gamma conj(A_{gamma+k}) A_gamma,
 *         K_mu = sum_k A_{mu+k} C_k,
 *     i.e. O(N^2) per evaluation ("direct matrix calculation", Sec. 2).
 *     Indices are taken modulo N (cyclic): that is the sum the transform
 *     identity of Eq. (4) reproduces exactly.  A truncated variant (indices
 *     outside the mode set dropped, the literal Kronecker delta over a finite
 *     mode set) is provided as well.  No FFT is used anywhere in this file.
 *   - Right-hand side: Eq. (1) in the frame rotating with the pump and the
 *     FSR grid,
 *         f_mu = (-kappa_mu/2 + i(omega'_mu - sigma(t))) u_mu
 *                + [mu == 0] sqrt(kappa_ext) A_in + i g0 K_mu(u),
 *     with omega'_mu = omega_mu - omega_0 - mu D1 and the linear detuning ramp
 *     sigma(t) = sigma0 + (sigma1 - sigma0) min(t, tau_ramp) / tau_ramp.
 *     Storage is centred: index i holds mode mu = i - N/2 (pump at N/2).
 *   - Classic fourth-order Runge-Kutta (Sec. 2: an ordinary ODE solver with
 *     the nonlinear sum evaluated separately): stage times t, t+h/2, t+h/2,
 *     t+h and weights 1/6, 1/3, 1/3, 1/6; the time of step n is
 *     t = (step0 + n) h computed from the integer step index.
 *   - The discrete adjoint of exactly that RK4 map (not in the paper; the
 *     gradient form of the method), with the Kerr vector-Jacobian product by
 *     direct O(N^2) sums:
 *         V(w)_nu = 2 sum_d w_{nu+d} C_d + sum_s conj(w_{s-nu}) S_s,
 *         C_d = sum_b conj(u_{b+d}) u_b,  S_s = sum_a u_a u_{s-a},
 *     which is the transpose, under Re<x, y> = Re sum conj(x) y, of
 *     du -> dK(u) = 2 K-terms linear in u + the term linear in conj(u).
 *   - Interaction-picture RK4 (RK4IP): classic RK4 on the variable with the
 *     exact linear propagator of each mode factored out, so the stiff
 *     dispersion does not bound the step (see orc_rk4ip_run).
 *   - The frequency-domain split-step map (Sec. 2, the second method):
 *     Strang splitting with the linear part (loss, detuning, pump) solved
 *     exactly per mode and the Kerr part solved exactly on the transformed
 *     field, where it is a pointwise phase rotation; the transforms are naive
 *     O(N^2) DFTs.
 *
 * Precision: IEEE double throughout, built without -ffast-math.  The only
 * floating-point flag used is -fcx-limited-range, which removes C99's
 * NaN/Inf recovery branch from complex multiplication and changes no finite
 * result.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* One resonator (the symbols of Eq. (1)).  Mirrors, but is independent of,
 * the solver's own descriptor. */
typedef struct {
  int32_t n;          /* number of modes N (any N >= 1)                      */
  int32_t reserved;
  int64_t offset;     /* start of this instance in the packed mode arrays    */
  double kappa_ext;   /* external coupling loss                              */
  double g0;          /* Kerr coefficient                                     */
  double ain_re;      /* pump amplitude A_in                                  */
  double ain_im;
  double sigma0;      /* detuning omega_in - omega_0 at t = 0                 */
  double sigma1;      /* detuning at t >= tau_ramp                            */
  double tau_ramp;    /* ramp length; <= 0 means sigma = sigma0 at all times  */
} orc_instance;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

static int g_threads = 0; /* 0: OpenMP default */

/* Inner loops of one state are split over threads only from this size on:
 * below it the fork/join cost of a parallel region exceeds the work. */
#define ORC_PAR_MIN_N 512

void orc_set_threads(int n) { g_threads = n; }

int orc_max_threads(void) {
#ifdef _OPENMP
  return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * FWM sum, Eq. (3): two correlations, O(N^2).  `par` enables OpenMP over the
 * output index (only used when the caller is not already parallel).
 * ------------------------------------------------------------------------- */
static void fwm_cyclic(int n, const cplx *a, cplx *K, cplx *C, int par) {
  /* C_k = sum_gamma conj(A_{gamma+k}) A_gamma */
#pragma omp parallel for schedule(static) if (par && n >= ORC_PAR_MIN_N) num_threads(orc_max_threads())
  for (int k = 0; k < n; ++k) {
    cplx s = 0.0;
    /* gamma + k, reduced mod N: the two ranges of gamma are summed in order */
    for (int g = 0; g < n - k; ++g) s += conj(a[g + k]) * a[g];
    for (int g = n - k; g < n; ++g) s += conj(a[g + k - n]) * a[g];
    C[k] = s;
  }
  /* K_mu = sum_k A_{mu+k} C_k */
#pragma omp parallel for schedule(static) if (par && n >= ORC_PAR_MIN_N) num_threads(orc_max_threads())
  for (int mu = 0; mu < n; ++mu) {
    cplx s = 0.0;
    for (int k = 0; k < n - mu; ++k) s += a[mu + k] * C[k];
    for (int k = n - mu; k < n; ++k) s += a[mu + k - n] * C[k];
    K[mu] = s;
  }
}

/* Truncated sum: alpha, beta, gamma, mu all inside [0, N) with
 * alpha - beta + gamma = mu exactly.  C is indexed by k + (N-1), k in (-N, N). */
static void fwm_truncated(int n, const cplx *a, cplx *K, cplx *C, int par) {
#pragma omp parallel for schedule(static) if (par && n >= ORC_PAR_MIN_N) num_threads(orc_max_threads())
  for (int k = -(n - 1); k <= n - 1; ++k) {
    cplx s = 0.0;
    for (int g = 0; g < n; ++g) {
      int b = g + k;
      if (b >= 0 && b < n) s += conj(a[b]) * a[g];
    }
    C[k + n - 1] = s;
  }
#pragma omp parallel for schedule(static) if (par && n >= ORC_PAR_MIN_N) num_threads(orc_max_threads())
  for (int mu = 0; mu < n; ++mu) {
    cplx s = 0.0;
    for (int k = -(n - 1); k <= n - 1; ++k) {
      int al = mu + k;
      if (al >= 0 && al < n) s += a[al] * C[k + n - 1];
    }
    K[mu] = s;
  }
}

/* Public: K for one state.  truncated = 0: cyclic (mod N); 1: truncated. */
int orc_fwm(int n, const cplx *a, cplx *K, int truncated) {
  if (n < 1 || !a || !K) return ORC_EINVAL;
  cplx *C = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * n));
  if (!C) return ORC_ENOMEM;
  if (truncated) fwm_truncated(n, a, K, C, 1);
  else fwm_cyclic(n, a, K, C, 1);
  free(C);
  return ORC_OK;
}

/* Kerr vector-Jacobian product, cyclic: v = V(w) with
 *   V(w)_nu = 2 sum_d w_{nu+d} C_d + sum_s conj(w_{s-nu}) S_s
 *   C_d = sum_b conj(u_{b+d}) u_b,   S_s = sum_a u_a u_{s-a}.
 * The first sum transposes the two terms of dK linear in du (alpha, gamma);
 * the second transposes the term linear in conj(du) (beta). */
static void kerr_vjp_cyclic(int n, const cplx *u, const cplx *w, cplx *v, cplx *C, cplx *S,
                            int par) {
#pragma omp parallel for schedule(static) if (par && n >= ORC_PAR_MIN_N) num_threads(orc_max_threads())
  for (int d = 0; d < n; ++d) {
    cplx c = 0.0, s = 0.0;
    for (int b = 0; b < n - d; ++b) c += conj(u[b + d]) * u[b];
    for (int b = n - d; b < n; ++b) c += conj(u[b + d - n]) * u[b];
    for (int b = 0; b <= d; ++b) s += u[b] * u[d - b];
    for (int b = d + 1; b < n; ++b) s += u[b] * u[d - b + n];
    C[d] = c;
    S[d] = s;
  }
#pragma omp parallel for schedule(static) if (par && n >= ORC_PAR_MIN_N) num_threads(orc_max_threads())
  for (int nu = 0; nu < n; ++nu) {
    cplx acc = 0.0;
    for (int d = 0; d < n - nu; ++d) acc += 2.0 * w[nu + d] * C[d];
    for (int d = n - nu; d < n; ++d) acc += 2.0 * w[nu + d - n] * C[d];
    for (int s = 0; s < nu; ++s) acc += conj(w[s - nu + n]) * S[s];
    for (int s = nu; s < n; ++s) acc += conj(w[s - nu]) * S[s];
    v[nu] = acc;
  }
}

int orc_kerr_vjp(int n, const cplx *u, const cplx *w, cplx *v) {
  if (n < 1 || !u || !w || !v) return ORC_EINVAL;
  cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * n));
  if (!tmp) return ORC_ENOMEM;
  kerr_vjp_cyclic(n, u, w, v, tmp, tmp + n, 1);
  free(tmp);
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Right-hand side of Eq. (1) in the rotating frame.
 * ------------------------------------------------------------------------- */
double orc_sigma(const orc_instance *p, double t) {
  if (!(p->tau_ramp > 0.0)) return p->sigma0;
  double s = t < 0.0 ? 0.0 : (t > p->tau_ramp ? p->tau_ramp : t);
  return p->sigma0 + (p->sigma1 - p->sigma0) * (s / p->tau_ramp);
}

typedef struct {
  cplx *K, *C;    /* FWM scratch: n and 2n */
} rhs_work;

static void rhs(const orc_instance *p, const double *kappa, const double *omega, double t,
                const cplx *u, cplx *f, rhs_work *w, int truncated, int par) {
  const int n = p->n;
  if (truncated) fwm_truncated(n, u, w->K, w->C, par);
  else fwm_cyclic(n, u, w->K, w->C, par);
  const double sig = orc_sigma(p, t);
  for (int i = 0; i < n; ++i) {
    cplx L = -0.5 * kappa[i] + I * (omega[i] - sig);
    f[i] = L * u[i] + I * p->g0 * w->K[i];
  }
  f[n / 2] += sqrt(p->kappa_ext) * (p->ain_re + I * p->ain_im);
}

int orc_rhs(const orc_instance *p, const double *kappa, const double *omega, double t,
            const cplx *u, cplx *f, int truncated) {
  if (!p || p->n < 1) return ORC_EINVAL;
  rhs_work w;
  w.K = (cplx *)malloc(sizeof(cplx) * (size_t)p->n);
  w.C = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * p->n));
  if (!w.K || !w.C) { free(w.K); free(w.C); return ORC_ENOMEM; }
  rhs(p, kappa, omega, t, u, f, &w, truncated, 1);
  free(w.K); free(w.C);
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Classic RK4.  One step from y at step index `step` (t = step * h).
 * Keeps the four stage inputs u_s if `us` is given (4 * n values).
 * ------------------------------------------------------------------------- */
typedef struct {
  rhs_work rw;
  cplx *u, *k, *acc;
} rk_work;

static int rk_work_alloc(rk_work *w, int n) {
  w->rw.K = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  w->rw.C = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * n));
  w->u = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  w->k = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  w->acc = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  return (w->rw.K && w->rw.C && w->u && w->k && w->acc) ? ORC_OK : ORC_ENOMEM;
}

static void rk_work_free(rk_work *w) {
  free(w->rw.K); free(w->rw.C); free(w->u); free(w->k); free(w->acc);
}

static const double RK_C[4] = {0.0, 0.5, 0.5, 1.0};
static const double RK_W[4] = {1.0, 2.0, 2.0, 1.0};

static void rk4_step(const orc_instance *p, const double *kappa, const double *omega, double h,
                     int64_t step, cplx *y, rk_work *w, cplx *us, int truncated, int par) {
  const int n = p->n;
  const double t0 = (double)step * h;
  for (int s = 0; s < 4; ++s) {
    if (s == 0) memcpy(w->u, y, sizeof(cplx) * (size_t)n);
    else for (int i = 0; i < n; ++i) w->u[i] = y[i] + (RK_C[s] * h) * w->k[i];
    if (us) memcpy(us + (size_t)s * n, w->u, sizeof(cplx) * (size_t)n);
    rhs(p, kappa, omega, t0 + RK_C[s] * h, w->u, w->k, &w->rw, truncated, par);
    if (s == 0) for (int i = 0; i < n; ++i) w->acc[i] = w->k[i];
    else for (int i = 0; i < n; ++i) w->acc[i] += RK_W[s] * w->k[i];
  }
  for (int i = 0; i < n; ++i) y[i] += (h / 6.0) * w->acc[i];
}

static int valid_batch(int batch, const orc_instance *inst) {
  if (batch < 0 || (batch > 0 && !inst)) return 0;
  for (int b = 0; b < batch; ++b)
    if (inst[b].n < 1 || inst[b].offset < 0) return 0;
  return 1;
}

/* Advance every instance of a packed batch by n_steps RK4 steps, starting at
 * step index step0.  y: packed complex state, updated in place.
 * ckpt (optional): after every ckpt_every steps the packed state is stored,
 * [n_steps / ckpt_every][total] values. */
int orc_run(int batch, const orc_instance *inst, const double *kappa, const double *omega,
            double h, int64_t step0, int64_t n_steps, cplx *y, int truncated,
            int ckpt_every, cplx *ckpt, int64_t total) {
  if (!valid_batch(batch, inst) || !(h > 0.0) || n_steps < 0 || step0 < 0) return ORC_EINVAL;
  int status = ORC_OK;
  const int outer = batch >= orc_max_threads();
#pragma omp parallel for schedule(dynamic, 1) if (outer) num_threads(orc_max_threads())
  for (int b = 0; b < batch; ++b) {
    const orc_instance *p = &inst[b];
    rk_work w;
    if (rk_work_alloc(&w, p->n) != ORC_OK) {
      status = ORC_ENOMEM;
      rk_work_free(&w);
      continue;
    }
    cplx *yb = y + p->offset;
    for (int64_t s = 0; s < n_steps; ++s) {
      rk4_step(p, kappa + p->offset, omega + p->offset, h, step0 + s, yb, &w, NULL, truncated,
               !outer);
      if (ckpt && ckpt_every > 0 && (s + 1) % ckpt_every == 0)
        memcpy(ckpt + (size_t)((s + 1) / ckpt_every - 1) * (size_t)total + p->offset, yb,
               sizeof(cplx) * (size_t)p->n);
    }
    rk_work_free(&w);
  }
  return status;
}

/* ---------------------------------------------------------------------------
 * Discrete adjoint of orc_run (cyclic FWM).
 *
 * Given the cotangent gT = dL/dRe y(T) + i dL/dIm y(T) of the final state,
 * returns (accumulating into the given arrays):
 *   g0_out[i]    = cotangent of the initial state y(0)      (optional)
 *   g_omega[i]  += dL/domega'_i                              (optional)
 *   g_kappa[i]  += dL/dkappa_i                               (optional)
 *   g_ain[2b..] += dL/dRe A_in + i dL/dIm A_in, per instance (optional)
 *
 * Per step, backwards:  ybar' = cotangent of y_{n+1};
 *   kbar4 = h/6 ybar',           ubar4 = J4^T kbar4,
 *   kbar3 = h/3 ybar' + h ubar4, ubar3 = J3^T kbar3,
 *   kbar2 = h/3 ybar' + h/2 ubar3, ubar2 = J2^T kbar2,
 *   kbar1 = h/6 ybar' + h/2 ubar2, ubar1 = J1^T kbar1,
 *   ybar  = ybar' + ubar1 + ubar2 + ubar3 + ubar4,
 * with J_s^T w = conj(L(t_s)) w + V_s(-i g0 w) and V_s the Kerr VJP at u_s.
 * Parameter terms: omega'_i: Re(conj(kbar_s,i) i u_s,i); kappa_i:
 * Re(conj(kbar_s,i) (-u_s,i / 2)); A_in: sqrt(kappa_ext) kbar_s at mu = 0.
 * All intermediate states are kept (no checkpointing): plain and slow.
 * ------------------------------------------------------------------------- */
int orc_adjoint(int batch, const orc_instance *inst, const double *kappa, const double *omega,
                double h, int64_t step0, int64_t n_steps, const cplx *y0, const cplx *gT,
                cplx *gy0, double *g_omega, double *g_kappa, cplx *g_ain) {
  if (!valid_batch(batch, inst) || !(h > 0.0) || n_steps < 0 || step0 < 0 || !y0 || !gT)
    return ORC_EINVAL;
  int status = ORC_OK;
  const int outer = batch >= orc_max_threads();
#pragma omp parallel for schedule(dynamic, 1) if (outer) num_threads(orc_max_threads())
  for (int b = 0; b < batch; ++b) {
    const orc_instance *p = &inst[b];
    const int n = p->n;
    const double *kap = kappa + p->offset, *om = omega + p->offset;
    const double sq = sqrt(p->kappa_ext);
    rk_work w;
    int ok = rk_work_alloc(&w, n) == ORC_OK;
    cplx *traj = ok ? (cplx *)malloc(sizeof(cplx) * (size_t)n * (size_t)(n_steps + 1)) : NULL;
    cplx *us = (cplx *)malloc(sizeof(cplx) * (size_t)(4 * n));
    cplx *yb = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *ybp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *kb = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *ub = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *wp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *vv = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *C = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * n));
    if (!ok || !traj || !us || !yb || !ybp || !kb || !ub || !wp || !vv || !C) {
      status = ORC_ENOMEM;
    } else {
      /* forward, keeping every state */
      memcpy(traj, y0 + p->offset, sizeof(cplx) * (size_t)n);
      for (int64_t s = 0; s < n_steps; ++s) {
        memcpy(traj + (size_t)(s + 1) * n, traj + (size_t)s * n, sizeof(cplx) * (size_t)n);
        rk4_step(p, kap, om, h, step0 + s, traj + (size_t)(s + 1) * n, &w, NULL, 0, !outer);
      }
      memcpy(ybp, gT + p->offset, sizeof(cplx) * (size_t)n);
      cplx gain = 0.0;
      for (int64_t s = n_steps - 1; s >= 0; --s) {
        /* stage inputs u_1..u_4 of step s */
        memcpy(wp, traj + (size_t)s * n, sizeof(cplx) * (size_t)n);
        rk4_step(p, kap, om, h, step0 + s, wp, &w, us, 0, !outer);
        const double t0 = (double)(step0 + s) * h;
        for (int i = 0; i < n; ++i) yb[i] = ybp[i];
        static const double kw[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
        /* ub holds ubar_{s+1} from the previous (later) stage */
        for (int st = 3; st >= 0; --st) {
          for (int i = 0; i < n; ++i) {
            cplx v = kw[st] * h * ybp[i];
            if (st < 3) v += RK_C[st + 1] * h * ub[i];
            kb[i] = v;
          }
          const cplx *u = us + (size_t)st * n;
          const double sig = orc_sigma(p, t0 + RK_C[st] * h);
          /* J^T kbar: linear part, then Kerr VJP at u */
          for (int i = 0; i < n; ++i) wp[i] = -I * p->g0 * kb[i];
          kerr_vjp_cyclic(n, u, wp, vv, C, C + n, !outer);
          for (int i = 0; i < n; ++i) {
            cplx L = -0.5 * kap[i] + I * (om[i] - sig);
            ub[i] = conj(L) * kb[i] + vv[i];
            yb[i] += ub[i];
            if (g_omega) g_omega[p->offset + i] += creal(conj(kb[i]) * (I * u[i]));
            if (g_kappa) g_kappa[p->offset + i] += creal(conj(kb[i]) * (-0.5 * u[i]));
          }
          gain += sq * kb[n / 2];
        }
        memcpy(ybp, yb, sizeof(cplx) * (size_t)n);
      }
      if (gy0) memcpy(gy0 + p->offset, ybp, sizeof(cplx) * (size_t)n);
      if (g_ain) g_ain[b] += gain;
    }
    rk_work_free(&w);
    free(traj); free(us); free(yb); free(ybp); free(kb); free(ub); free(wp); free(vv);
    free(C);
  }
  return status;
}

/* ---------------------------------------------------------------------------
 * Frequency-domain split-step (Strang): half linear step, full Kerr step,
 * half linear step.
 *
 * Kerr part.  With a_j = sum_mu A_mu e^{+2 pi i j mu / N} (no 1/N) and, by
 * Eq. (4), K_mu = (1/N) sum_j |a_j|^2 a_j e^{-2 pi i j mu / N}, the flow
 * dA/dt = i g0 K(A) becomes da_j/dt = i g0 |a_j|^2 a_j for every j, so |a_j|
 * is constant and the exact solution is a_j(h) = a_j e^{i g0 |a_j|^2 h}.
 * Linear part.  dA_mu/dt = L_mu A_mu + [mu == 0] s with L = -kappa/2 +
 * i(omega' - sigma), s = sqrt(kappa_ext) A_in, solved exactly over each half
 * step with sigma frozen at the half step's midpoint.
 * The transforms are naive O(N^2) DFTs (no FFT).
 * ------------------------------------------------------------------------- */
static void naive_dft(int n, const cplx *x, cplx *y, double sign, int par) {
  const double w0 = sign * 2.0 * M_PI / (double)n;
#pragma omp parallel for schedule(static) if (par && n >= ORC_PAR_MIN_N) num_threads(orc_max_threads())
  for (int j = 0; j < n; ++j) {
    cplx s = 0.0;
    for (int m = 0; m < n; ++m) {
      /* reduce j*m mod n before the angle so large products stay exact */
      int64_t jm = ((int64_t)j * m) % n;
      s += x[m] * cexp(I * (w0 * (double)jm));
    }
    y[j] = s;
  }
}

static void linear_exact(const orc_instance *p, const double *kappa, const double *omega,
                         double t_mid, double dt, cplx *y) {
  const int n = p->n;
  const double sig = orc_sigma(p, t_mid);
  for (int i = 0; i < n; ++i) {
    cplx L = -0.5 * kappa[i] + I * (omega[i] - sig);
    cplx e = cexp(L * dt);
    y[i] *= e;
    if (i == n / 2) {
      cplx s = sqrt(p->kappa_ext) * (p->ain_re + I * p->ain_im);
      /* (e - 1)/L, with the L -> 0 limit dt */
      cplx phi = cabs(L * dt) > 1e-8 ? (e - 1.0) / L : dt * (1.0 + 0.5 * L * dt);
      y[i] += s * phi;
    }
  }
}

int orc_split_step_run(int batch, const orc_instance *inst, const double *kappa,
                       const double *omega, double h, int64_t step0, int64_t n_steps, cplx *y) {
  if (!valid_batch(batch, inst) || !(h > 0.0) || n_steps < 0 || step0 < 0) return ORC_EINVAL;
  int status = ORC_OK;
  const int outer = batch >= orc_max_threads();
#pragma omp parallel for schedule(dynamic, 1) if (outer) num_threads(orc_max_threads())
  for (int b = 0; b < batch; ++b) {
    const orc_instance *p = &inst[b];
    const int n = p->n;
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!a) { status = ORC_ENOMEM; continue; }
    cplx *yb = y + p->offset;
    for (int64_t s = 0; s < n_steps; ++s) {
      const double t0 = (double)(step0 + s) * h;
      linear_exact(p, kappa + p->offset, omega + p->offset, t0 + 0.25 * h, 0.5 * h, yb);
      /* to the transformed field: a_j = sum_mu A_mu e^{+2 pi i j mu/N} */
      naive_dft(n, yb, a, +1.0, !outer);
      /* exact Kerr rotation on the transformed field */
      for (int j = 0; j < n; ++j) {
        double pw = creal(a[j]) * creal(a[j]) + cimag(a[j]) * cimag(a[j]);
        a[j] *= cexp(I * (p->g0 * h * pw));
      }
      naive_dft(n, a, yb, -1.0, !outer);
      for (int i = 0; i < n; ++i) yb[i] /= (double)n;
      linear_exact(p, kappa + p->offset, omega + p->offset, t0 + 0.75 * h, 0.5 * h, yb);
    }
    free(a);
  }
  return status;
}

/* ---------------------------------------------------------------------------
 * Interaction-picture fourth-order Runge-Kutta (RK4IP).  Split the right-hand
 * side of Eq. (1) into the linear rate of each mode,
 *     L_mu(t) = -kappa_mu/2 + i(omega'_mu - sigma(t)),
 * and the rest, N(u) = i g0 K(u) + [mu == 0] sqrt(kappa_ext) A_in.  Over one
 * step from t0, with tm = t0 + h/2, the variable B(t) = exp(-int_tm^t L) A(t)
 * obeys dB/dt = exp(-int_tm^t L) N(exp(int_tm^t L) B), and classic RK4 on B,
 * mapped back to A, reads (P1 = exp(int_t0^tm L), P2 = exp(int_tm^{t0+h} L),
 * per mode; the integrals are exact because sigma is piecewise linear):
 *     yI = P1 y,              k1 = P1 N(y),
 *     k2 = N(yI + h/2 k1),    k3 = N(yI + h/2 k2),    k4 = N(P2 (yI + h k3)),
 *     y' = P2 (yI + h/6 (k1 + 2 k2 + 2 k3)) + h/6 k4.
 * The linear part, dispersion included, is integrated exactly, so the RK4
 * stability bound on h max |L| does not apply.
 * ------------------------------------------------------------------------- */

/* integral of sigma(t) over [a, b], 0 <= a <= b */
static double sigma_integral(const orc_instance *p, double a, double b) {
  if (!(p->tau_ramp > 0.0)) return p->sigma0 * (b - a);
  const double T = p->tau_ramp, slope = (p->sigma1 - p->sigma0) / T;
  double ramp; /* integral of min(t, T) */
  if (b <= T) ramp = 0.5 * (b - a) * (b + a);
  else if (a >= T) ramp = T * (b - a);
  else ramp = 0.5 * (T - a) * (T + a) + T * (b - T);
  return p->sigma0 * (b - a) + slope * ramp;
}

static void nonlinear_part(const orc_instance *p, const cplx *u, cplx *f, rhs_work *w, int par) {
  const int n = p->n;
  fwm_cyclic(n, u, w->K, w->C, par);
  for (int i = 0; i < n; ++i) f[i] = I * p->g0 * w->K[i];
  f[n / 2] += sqrt(p->kappa_ext) * (p->ain_re + I * p->ain_im);
}

double orc_sigma_integral(const orc_instance *p, double a, double b) {
  return sigma_integral(p, a, b);
}

int orc_rk4ip_run(int batch, const orc_instance *inst, const double *kappa, const double *omega,
                  double h, int64_t step0, int64_t n_steps, cplx *y) {
  if (!valid_batch(batch, inst) || !(h > 0.0) || n_steps < 0 || step0 < 0) return ORC_EINVAL;
  int status = ORC_OK;
  const int outer = batch >= orc_max_threads();
#pragma omp parallel for schedule(dynamic, 1) if (outer) num_threads(orc_max_threads())
  for (int b = 0; b < batch; ++b) {
    const orc_instance *p = &inst[b];
    const int n = p->n;
    const double *kap = kappa + p->offset, *om = omega + p->offset;
    rhs_work rw;
    rw.K = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    rw.C = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * n));
    cplx *P1 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *P2 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *yi = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *u = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *k = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *acc = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!rw.K || !rw.C || !P1 || !P2 || !yi || !u || !k || !acc) {
      status = ORC_ENOMEM;
    } else {
      cplx *yb = y + p->offset;
      for (int64_t s = 0; s < n_steps; ++s) {
        const double t0 = (double)(step0 + s) * h, tm = t0 + 0.5 * h, t1 = t0 + h;
        const double S1 = sigma_integral(p, t0, tm), S2 = sigma_integral(p, tm, t1);
        for (int i = 0; i < n; ++i) {
          const double mag = exp(-0.25 * h * kap[i]);
          P1[i] = mag * cexp(I * (0.5 * h * om[i] - S1));
          P2[i] = mag * cexp(I * (0.5 * h * om[i] - S2));
        }
        nonlinear_part(p, yb, k, &rw, !outer);
        for (int i = 0; i < n; ++i) {
          yi[i] = P1[i] * yb[i];
          acc[i] = P1[i] * k[i];
          u[i] = yi[i] + (0.5 * h) * acc[i];
        }
        nonlinear_part(p, u, k, &rw, !outer);
        for (int i = 0; i < n; ++i) {
          acc[i] += 2.0 * k[i];
          u[i] = yi[i] + (0.5 * h) * k[i];
        }
        nonlinear_part(p, u, k, &rw, !outer);
        for (int i = 0; i < n; ++i) {
          acc[i] += 2.0 * k[i];
          u[i] = P2[i] * (yi[i] + h * k[i]);
        }
        nonlinear_part(p, u, k, &rw, !outer);
        for (int i = 0; i < n; ++i) yb[i] = P2[i] * (yi[i] + (h / 6.0) * acc[i]) + (h / 6.0) * k[i];
      }
    }
    free(rw.K); free(rw.C); free(P1); free(P2); free(yi); free(u); free(k); free(acc);
  }
  return status;
}
