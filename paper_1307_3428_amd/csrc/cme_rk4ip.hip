// cme_rk4ip.hip -- interaction-picture fourth-order Runge-Kutta (RK4IP) on
// the two-level transform of cme_fft.hpp.
//
// The right-hand side of Eq. (1) is split into the linear rate of each mode,
// L_mu(t) = -kappa_mu/2 + i(omega'_mu - sigma(t)), integrated exactly, and
// N(u) = i (g0/N) DFT(|a|^2 a) + [mu = 0] pump with a = IDFT(u) (Eq. (4)),
// taken by the RK4 stages.  Over one step from t0 (tm = t0 + h/2), with the
// half-step propagators P1 = exp(int_t0^tm L), P2 = exp(int_tm^{t0+h} L):
//   yI = P1 y,             k1 = P1 N(y),
//   k2 = N(yI + h/2 k1),   k3 = N(yI + h/2 k2),   k4 = N(P2 (yI + h k3)),
//   y' = P2 (yI + h/6 (k1 + 2 k2 + 2 k3)) + h/6 k4
// (classic RK4 on exp(-int_tm^t L) A).  P = D exp(-i int sigma), where the
// per-mode factor D = exp((-kappa/2 + i omega') h/2) is formed once per
// launch (FP64, then rounded) and the detuning phase is one scalar per half
// step (the integral of the piecewise-linear ramp in closed form).  The
// dispersion therefore does not bound the step as it does for classic RK4.
// Same workgroup layout and transforms as the wave kernels (cme_wave.hpp);
// four transform pairs per step, no adjoint.  The same step runs on the lean
// transforms (cme_lean.hip, N = 4096) and the staged ones (cme_staged.hip,
// N >= 8192).
#include <type_traits>

#include "cme_wave.hpp"

namespace cme {

namespace {

template <typename Real, int N, int E, int V, int PS, int TP>
__global__ void __launch_bounds__((WaveShape<Real, N, E, V, PS, TP>::THREADS)) rk4ip_wave(RunArgs a) {
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  using WP = WavePlan<N, E, V, TP>;
  constexpr int W = WP::W;
  __shared__ cx<Real> lds[SH::IPB * SH::PER_INST];

  const int lane = (int)threadIdx.x & 63;
  const int wv = (int)threadIdx.x >> 6;
  const int sub = W == 1 ? wv : 0;
  const int w = W == 1 ? 0 : wv;
  const int slot = (int)blockIdx.x * SH::IPB + sub;
  if constexpr (W == 1) {
    if (slot >= a.count) return;  // waves of a W = 1 group never synchronise
  }
  const int id = a.order[slot];
  const DevInst d = a.inst[id];
  cx<Real> *X = lds + sub * SH::PER_INST;
  cx<Real> *Y = SH::TWO ? X + SH::WV * SH::LB1 : X;
  cx<Real> *A = reinterpret_cast<cx<Real> *>(a.A) + d.offset;
  const double *kap = a.kappa + d.offset;
  const double *omg = a.omega + d.offset;

  WaveTwiddles<N, E, V, TP, Real> tw;
  load_wave_twiddles<N, E, V>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  const double h = a.h;
  cx<Real> y[E], acc[E], v[E], dm[E];
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = WP::mode(w, lane, m);
    y[m] = A[i];
    const double mag = exp(-0.25 * h * kap[i]);
    double sn, cs;
    sincos(0.5 * h * omg[i], &sn, &cs);
    dm[m] = {(Real)(mag * cs), (Real)(mag * sn)};
  });
  const bool pump_owner = (w == 0 && lane == 0);
  const Real gn = (Real)d.g0n;
  const cx<Real> pump = {(Real)d.pump_re, (Real)d.pump_im};
  const Real hh = (Real)(0.5 * h), hf = (Real)h, h6 = (Real)(h / 6.0);
  cx<Real> *ckpt = reinterpret_cast<cx<Real> *>(a.ckpt);
  int32_t to_ckpt = a.ckpt_every;
  int64_t ckpt_slot = 0;

  // v <- N(v): inverse transform, cube, forward transform, i g0/N, pump
  auto nonlinear = [&]() {
    fft_fwdpath<N, E, V, TP, +1, PS, !SH::TWO>(v, X, tw, w, lane);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const Real p = v[m].re * v[m].re + v[m].im * v[m].im;
      v[m] = {p * v[m].re, p * v[m].im};
    });
    fft_backpath<N, E, V, TP, -1, PS>(v, X, Y, tw, w, lane);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      cx<Real> q = {-gn * v[m].im, gn * v[m].re};
      if constexpr (m == E / 2) {
        if (pump_owner) q = cadd(q, pump);
      }
      v[m] = q;
    });
  };

  for (int64_t n = 0; n < a.n_steps; ++n) {
    const double t0 = (double)(a.step0 + n) * h, tm = t0 + 0.5 * h, t1 = t0 + h;
    double sn, cs;
    sincos(-sigma_integral(d.sigma0, d.sigma1, d.tau_ramp, t0, tm), &sn, &cs);
    const cx<Real> c1 = {(Real)cs, (Real)sn};
    sincos(-sigma_integral(d.sigma0, d.sigma1, d.tau_ramp, tm, t1), &sn, &cs);
    const cx<Real> c2 = {(Real)cs, (Real)sn};
    // k1 = P1 N(y), yI = P1 y
    sfor<0, E>([&](auto mi) { v[decltype(mi)::value] = y[decltype(mi)::value]; });
    nonlinear();
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const cx<Real> p1 = cmul(dm[m], c1);
      acc[m] = cmul(p1, v[m]);
      y[m] = cmul(p1, y[m]);
      v[m] = {y[m].re + hh * acc[m].re, y[m].im + hh * acc[m].im};
    });
    // k2 = N(yI + h/2 k1)
    nonlinear();
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      acc[m] = {acc[m].re + (Real)2 * v[m].re, acc[m].im + (Real)2 * v[m].im};
      v[m] = {y[m].re + hh * v[m].re, y[m].im + hh * v[m].im};
    });
    // k3 = N(yI + h/2 k2)
    nonlinear();
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      acc[m] = {acc[m].re + (Real)2 * v[m].re, acc[m].im + (Real)2 * v[m].im};
      v[m] = cmul(cmul(dm[m], c2), cx<Real>{y[m].re + hf * v[m].re, y[m].im + hf * v[m].im});
    });
    // k4 = N(P2 (yI + h k3)); y' = P2 (yI + h/6 acc) + h/6 k4
    nonlinear();
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const cx<Real> z = cmul(cmul(dm[m], c2), cx<Real>{y[m].re + h6 * acc[m].re,
                                                       y[m].im + h6 * acc[m].im});
      y[m] = {z.re + h6 * v[m].re, z.im + h6 * v[m].im};
    });
    if (ckpt != nullptr && --to_ckpt == 0) {
      to_ckpt = a.ckpt_every;
      cx<Real> *dst = ckpt + ckpt_slot * a.total + d.offset;
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        dst[WP::mode(w, lane, m)] = y[m];
      });
      ++ckpt_slot;
    }
  }
  bool bad = false;
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    A[WP::mode(w, lane, m)] = y[m];
    bad |= !(isfinite(y[m].re) && isfinite(y[m].im));
  });
  if (bad) atomicOr(&a.flags[id], 1);
}

template <typename Real, int N, int E, int V, int PS, int TP>
hipError_t launch_rk4ip(const RunArgs &a, hipStream_t st) {
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  if (a.stages != nullptr) return hipErrorInvalidValue;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((rk4ip_wave<Real, N, E, V, PS, TP>), dim3(grid), dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

template <typename Real, int N, int E, int V, int PS, int TP = 0> constexpr Variant rk4ip_variant() {
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  return Variant{std::is_same<Real, double>::value ? 0 : 1, N, E, V, PS, TP, 7, SH::IPB,
                 SH::THREADS, SH::LDS_BYTES, &launch_rk4ip<Real, N, E, V, PS, TP>, nullptr};
}

// (N, E, V, PS): the wave kernel shapes; one default per size and precision
const Variant kRk4ipVariants[] = {
    rk4ip_variant<double, 128, 2, 1, 1>(),   rk4ip_variant<double, 256, 4, 1, 2>(),
    rk4ip_variant<double, 512, 4, 1, 2>(),   rk4ip_variant<double, 1024, 4, 1, 2>(),
    rk4ip_variant<double, 2048, 8, 1, 3>(),  rk4ip_variant<double, 4096, 8, 1, 3>(),
    rk4ip_variant<double, 8192, 16, 2, 3>(), rk4ip_variant<float, 128, 2, 1, 1>(),
    rk4ip_variant<float, 256, 4, 1, 2>(),    rk4ip_variant<float, 512, 8, 1, 3>(),
    rk4ip_variant<float, 1024, 8, 1, 3>(),   rk4ip_variant<float, 2048, 8, 1, 3>(),
    rk4ip_variant<float, 4096, 8, 1, 3>(),   rk4ip_variant<float, 8192, 16, 2, 3>(),
};

}  // namespace

const Variant *variants_rk4ip(int *count) {
  *count = (int)(sizeof(kRk4ipVariants) / sizeof(kRk4ipVariants[0]));
  return kRk4ipVariants;
}

}  // namespace cme
