// cme_split.hip -- frequency-domain split-step time stepping (the paper's
// second method, Sec. 2): Strang splitting of Eq. (1) into its linear part,
// solved exactly per mode, and the four-wave-mixing part, solved exactly on
// the transformed field.
//
// One step of size h from t0:
//   1. half linear step, dA_mu/dt = L_mu A_mu + [mu = 0] s over h/2 with
//      L_mu = -kappa_mu/2 + i(omega'_mu - sigma(t0 + h/4)) frozen:
//        A_mu <- e^{L_mu h/2} A_mu + [mu = 0] s (e^{L_mu h/2} - 1) / L_mu,
//      s = sqrt(kappa_ext) A_in (the limit h/2 (1 + L h/4) where |L h/2| is
//      tiny);
//   2. a = IDFT(A) (Eq. (4), no 1/N): the Kerr flow dA/dt = i g0 K(A) is
//      da_j/dt = i g0 |a_j|^2 a_j, whose exact solution keeps |a_j| and
//      rotates the phase: a_j <- a_j e^{i g0 h |a_j|^2};
//   3. A = DFT(a) / N;
//   4. half linear step with sigma(t0 + 3h/4).
// e^{L_mu h/2} = e^{(-kappa_mu/2 + i omega'_mu) h/2} e^{-i sigma h/2}: the
// first factor is formed once per launch, the second once per half step.
// Two transforms per step (RK4 needs eight); second-order accurate in h.
// The transform is that of cme_lean.hpp; FP64 or FP32 (the linear factors
// formed in FP64 and rounded, the pump mode's half step in FP64); N = 128 ...
// 4096 (the staged transforms of cme_staged.hip take the same map above, FP64).
#include <type_traits>

#include "cme_internal.hpp"
#include "cme_lean.hpp"

namespace cme {

template <typename Real, int N, int E, int PS, int IPB_ = 0> struct SplitShape {
  using LP = LeanPlan<N, E>;
  static constexpr int W = LP::W;
  static constexpr int WV = LP::WV;
  static constexpr int IPB = IPB_ > 0 ? IPB_ : (W == 1 ? 4 : 1);
  static constexpr int LB1 = LdsLen<LP::N1, PS>::value;
  static constexpr int LIMIT = 160 * 1024;
  static constexpr int ONE = IPB * WV * LB1 * (int)sizeof(cx<Real>);
  static constexpr bool TWO = WV > 1 && 2 * ONE <= LIMIT;
  static constexpr int PER_INST = (TWO ? 2 : 1) * WV * LB1;
  static constexpr int LDS_BYTES = IPB * PER_INST * (int)sizeof(cx<Real>);
  static constexpr int THREADS = IPB * 64 * W;
  static_assert(LDS_BYTES <= LIMIT, "LDS over the gfx950 per-workgroup limit");
};

template <typename Real, int N, int E, int PS, int IPB_ = 0>
__global__ void __launch_bounds__((SplitShape<Real, N, E, PS, IPB_>::THREADS)) split_lean(RunArgs a) {
  using SH = SplitShape<Real, N, E, PS, IPB_>;
  using WP = WavePlan<N, E, 1, 0>;
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

  LeanTw<N, E, Real> tw;
  load_lean_twiddles<N, E>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  const double h = a.h, hh = 0.5 * a.h;
  // f = e^{(-kappa/2 + i omega') h/2} per mode
  cx<Real> y[E], f[E], v[E];
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = WP::mode(w, lane, m);
    y[m] = A[i];
    const double mag = exp(-0.5 * kap[i] * hh);
    double sn, cs;
    sincos(omg[i] * hh, &sn, &cs);
    f[m] = {(Real)(mag * cs), (Real)(mag * sn)};
  });
  const bool pump_owner = (w == 0 && lane == 0);  // mode N/2 sits in slot E/2
  const double lre = -0.5 * kap[N / 2], lim0 = omg[N / 2];
  const cx<double> pump = {d.pump_re, d.pump_im};
  const double gh = d.g0n * (double)N * h;  // g0 h
  const Real ghr = (Real)gh;                 // the Kerr rotation runs in Real
  const Real inv_n = (Real)1 / (Real)N;

  auto half_linear = [&](double t_mid) {
    const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t_mid);
    double sn, cs;
    sincos(-sig * hh, &sn, &cs);
    const cx<Real> c = {(Real)cs, (Real)sn};
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const cx<Real> e = cmul(f[m], c);
      if constexpr (m == E / 2 && std::is_same<Real, float>::value) {
        if (pump_owner) {
          // FP32: the pump mode's half-step coefficients e = exp(L h/2) and
          // s (e - 1) / L with L = lre + i (lim0 - sig) depend on sigma(t);
          // they are formed in FP64 (in FP32, e - 1 would lose digits) and
          // rounded once, the update of the state is FP32
          const double li = lim0 - sig;
          const double mg = exp(lre * hh);
          double s2, c2;
          sincos(li * hh, &s2, &c2);
          const cx<double> ed = {mg * c2, mg * s2};
          cx<double> phi;
          if (sqrt(lre * lre + li * li) * hh > 1e-8) {
            const double den = lre * lre + li * li;
            phi = {((ed.re - 1.0) * lre + ed.im * li) / den, (ed.im * lre - (ed.re - 1.0) * li) / den};
          } else {
            phi = {hh * (1.0 + 0.5 * lre * hh), hh * (0.5 * li * hh)};
          }
          const cx<double> sp = cmul(pump, phi);
          y[m] = cadd(cmul(y[m], cx<Real>{(Real)ed.re, (Real)ed.im}),
                      cx<Real>{(Real)sp.re, (Real)sp.im});
        } else {
          y[m] = cmul(y[m], e);
        }
      } else {
        y[m] = cmul(y[m], e);
        if constexpr (m == E / 2) {
          if (pump_owner) {
            // (e - 1) / L with L = lre + i (lim0 - sig), or its small-|L h/2| limit
            const cx<double> L = {lre, lim0 - sig};
            const double lh = sqrt(L.re * L.re + L.im * L.im) * hh;
            cx<double> phi;
            if (lh > 1e-8) {
              const cx<double> em1 = {e.re - 1.0, e.im};
              const double den = L.re * L.re + L.im * L.im;
              phi = {(em1.re * L.re + em1.im * L.im) / den, (em1.im * L.re - em1.re * L.im) / den};
            } else {
              phi = {hh * (1.0 + 0.5 * L.re * hh), hh * (0.5 * L.im * hh)};
            }
            const cx<double> pp = cmul(pump, phi);
            y[m] = {y[m].re + (Real)pp.re, y[m].im + (Real)pp.im};
          }
        }
      }
    });
  };

  cx<Real> *ckpt = reinterpret_cast<cx<Real> *>(a.ckpt);
  int32_t to_ckpt = a.ckpt_every;
  int64_t ckpt_slot = 0;
  for (int64_t n = 0; n < a.n_steps; ++n) {
    const double t0 = (double)(a.step0 + n) * h;
    half_linear(t0 + 0.25 * h);
    sfor<0, E>([&](auto mi) { v[decltype(mi)::value] = y[decltype(mi)::value]; });
    lean_fwdpath<N, E, +1, PS, !SH::TWO>(v, X, tw, w, lane);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      Real sn, cs;
      const Real ph = ghr * (v[m].re * v[m].re + v[m].im * v[m].im);
      if constexpr (std::is_same<Real, float>::value) sincosf(ph, &sn, &cs);
      else sincos(ph, &sn, &cs);
      v[m] = cmul(v[m], cx<Real>{cs, sn});
    });
    lean_backpath<N, E, -1, PS>(v, X, Y, tw, w, lane);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      y[m] = {v[m].re * inv_n, v[m].im * inv_n};
    });
    half_linear(t0 + 0.75 * h);
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

template <typename Real, int N, int E, int PS, int IPB_ = 0>
hipError_t launch_split(const RunArgs &a, hipStream_t st) {
  using SH = SplitShape<Real, N, E, PS, IPB_>;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((split_lean<Real, N, E, PS, IPB_>), dim3(grid), dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

template <typename Real, int N, int E, int PS, int IPB_ = 0> constexpr Variant split_variant() {
  using SH = SplitShape<Real, N, E, PS, IPB_>;
  return Variant{std::is_same<Real, double>::value ? 0 : 1, N, E, 1, PS, 0, 4, SH::IPB,
                 SH::THREADS, SH::LDS_BYTES,
                 &launch_split<Real, N, E, PS, IPB_>, nullptr};
}

// (N, E, PS[, instances per workgroup]): one wavefront per instance up to
// N = 256, then E = 8.  Single-wavefront instances run one per workgroup by
// default (each on its own CU when the batch is small: the paper's Fig. 1
// set steps 10% faster than with four per workgroup) or four per workgroup.
static const Variant kSplitVariants[] = {
    split_variant<double, 128, 2, 1, 1>(), split_variant<double, 256, 4, 2, 1>(),
    split_variant<double, 128, 2, 1>(),    split_variant<double, 256, 4, 2>(),
    split_variant<double, 512, 8, 3>(),    split_variant<double, 1024, 8, 3>(),
    split_variant<double, 2048, 8, 3>(),   split_variant<double, 4096, 8, 3>(),
    // FP32 state and transforms (the linear factors formed in FP64, the pump
    // mode's half step in FP64)
    split_variant<float, 128, 2, 1, 1>(), split_variant<float, 256, 4, 2, 1>(),
    split_variant<float, 512, 8, 3>(),    split_variant<float, 1024, 8, 3>(),
    split_variant<float, 2048, 8, 3>(),   split_variant<float, 4096, 8, 3>(),
};

const Variant *variants_split(int *count) {
  *count = (int)(sizeof(kSplitVariants) / sizeof(kSplitVariants[0]));
  return kSplitVariants;
}

}  // namespace cme
