// cme_dual.hip -- persistent RK4 kernel with two independent transform chains.
//
// Same RK4 map as cme_wave.hip, evaluated in a different but mathematically
// identical order.  With L(t) = -kappa/2 + i(omega' - sigma(t)), p the pump
// at mu = 0, a hat for the unnormalised inverse transform (Eq. (4)) and
// K = DFT(b) / N the four-wave-mixing sum of b = |a|^2 a:
//
//   k_s           = L(t_s) u_s + p + i g0 K_s                   (mode domain)
//   IDFT(k_s)     = IDFT(L(t_s) u_s + p) + i g0 b_s            (IDFT(DFT(b)) = N b)
//   a_{s+1}       = IDFT(u_{s+1}) = IDFT(y) + c_{s+1} h IDFT(k_s)
//
// so a step needs the transforms
//   R0: IDFT(y)  and  IDFT(L_1 y + p)          (independent)
//   R1: DFT(b_1)
//   R2: DFT(b_2) and IDFT(L_2 u_2 + p)         (independent)
//   R3: DFT(b_3) and IDFT(L_3 u_3 + p)         (independent)
//   R4: DFT(b_4)
// -- eight transforms in five dependent rounds, one workgroup barrier per
// round, and in three rounds two transforms whose instruction streams
// interleave (one transform's LDS traffic overlaps the other's arithmetic).
// IDFT(y) is recomputed from the mode amplitudes every step, so the state is
// still only A and split runs stay bit-identical.
//
// LDS: two sets of two transform contexts, alternated round by round, so
// that one barrier per round separates every reuse of a context; when two
// sets do not fit, one set plus a barrier at the start of every round.
#include "cme_fft.hpp"
#include "cme_internal.hpp"

namespace cme {

namespace {
__device__ constexpr double kCd[4] = {0.0, 0.5, 0.5, 1.0};
}  // namespace

template <typename Real, int N, int E, int PS, int TP> struct DualShape {
  using WP = WavePlan<N, E, 1, TP>;
  static constexpr int W = WP::W;
  static constexpr int WV = WP::WV;
  static constexpr int IPB = W == 1 ? 4 : 1;
  static constexpr int LB1 = LdsLen<WP::N1, PS>::value;
  static constexpr int CTX = WV * LB1;
  static constexpr int LIMIT = 160 * 1024;
  static constexpr int NSET = IPB * 4 * CTX * (int)sizeof(cx<Real>) <= LIMIT ? 2 : 1;
  static constexpr int PER_INST = NSET * 2 * CTX;
  static constexpr int LDS_BYTES = IPB * PER_INST * (int)sizeof(cx<Real>);
  static constexpr int THREADS = IPB * WP::T;
  static_assert(LDS_BYTES <= LIMIT, "LDS over the gfx950 per-workgroup limit");
  static_assert(THREADS <= 1024, "workgroup too large");
  static_assert(TP == 0 || PS == 3, "register-transpose sub-transforms use the 1-in-8 padded region");
};

template <typename Real, int N, int E, int PS, int TP>
__global__ void __launch_bounds__((DualShape<Real, N, E, PS, TP>::THREADS)) rk4_dual(RunArgs a) {
  using SH = DualShape<Real, N, E, PS, TP>;
  using WP = WavePlan<N, E, 1, TP>;
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
  cx<Real> *const base = lds + sub * SH::PER_INST;
  cx<Real> *A = reinterpret_cast<cx<Real> *>(a.A) + d.offset;
  const double *kap = a.kappa + d.offset;
  const double *omg = a.omega + d.offset;

  WaveTwiddles<N, E, 1, TP, Real> tw;
  load_wave_twiddles<N, E, 1>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  // mode domain: y, k, acc; transformed domain: yt = IDFT(y), bt = |a|^2 a;
  // va, vb: the two transform chains
  cx<Real> y[E], k[E], acc[E], yt[E], bt[E], va[E], vb[E];
  Real lr[E];
  double om[E];
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = WP::mode(w, lane, m);
    y[m] = A[i];
    lr[m] = (Real)(-0.5 * kap[i]);
    om[m] = omg[i];
  });
  const bool pump_owner = (w == 0 && lane == 0);
  const Real gn = (Real)d.g0n;                 // g0 / N (mode domain)
  const Real gt = (Real)(d.g0n * (double)N);   // g0     (transformed domain)
  const cx<Real> pump = {(Real)d.pump_re, (Real)d.pump_im};
  const double h = a.h;
  cx<Real> *ckpt = reinterpret_cast<cx<Real> *>(a.ckpt);
  cx<Real> *stages = reinterpret_cast<cx<Real> *>(a.stages);
  int32_t to_ckpt = a.ckpt_every;
  int64_t ckpt_slot = 0;
  int round = 0;

  // context c (0: chain a, 1: chain b) of the current round
  auto ctx = [&](int c) { return base + (((round & (SH::NSET - 1)) * 2) + c) * SH::CTX; };
  auto begin_round = [&]() {
    if constexpr (SH::NSET == 1) {
      if (round > 0) cross_sync<W>();
    }
  };
  // q = L(sig) u + p for mode slot m
  auto lin = [&](const cx<Real> u, int m, double sig, bool pump_slot) {
    const Real det = (Real)(om[m] - sig);
    cx<Real> q = {lr[m] * u.re - det * u.im, lr[m] * u.im + det * u.re};
    if (pump_slot && pump_owner) q = cadd(q, pump);
    return q;
  };
  auto store_stage = [&](int64_t n, int s, const cx<Real> *u) {
    if (stages != nullptr) {
      cx<Real> *st = stages + ((int64_t)n * 4 + s) * a.total + d.offset;
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        st[WP::mode(w, lane, m)] = u[m];
      });
    }
  };

  for (int64_t n = 0; n < a.n_steps; ++n) {
    const double t0 = (double)(a.step0 + n) * h;
    // ---- R0: yt = IDFT(y), vb = IDFT(L_1 y + p)
    const double sig0 = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0);
    store_stage(n, 0, y);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      va[m] = y[m];
      vb[m] = lin(y[m], m, sig0, m == E / 2);
    });
    begin_round();
    {
      cx<Real> *ca = ctx(0), *cb = ctx(1);
      fwd_phase1<N, E, 1, TP, +1, PS>(va, ca, tw, w, lane);
      fwd_phase1<N, E, 1, TP, +1, PS>(vb, cb, tw, w, lane);
      cross_sync<W>();
      fwd_phase2<N, E, 1, TP, +1, PS>(va, ca, tw, w, lane);
      fwd_phase2<N, E, 1, TP, +1, PS>(vb, cb, tw, w, lane);
    }
    ++round;
    // ---- R1: DFT(b_1), b_1 = |yt|^2 yt
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      yt[m] = va[m];
      const Real p = va[m].re * va[m].re + va[m].im * va[m].im;
      bt[m] = {p * va[m].re, p * va[m].im};
      va[m] = bt[m];
    });
    begin_round();
    {
      cx<Real> *ca = ctx(0);
      back_phase1<N, E, 1, TP, -1, PS>(va, ca, tw, w, lane);
      cross_sync<W>();
      back_phase2<N, E, 1, TP, -1, PS>(va, ca, tw, w, lane);
    }
    ++round;
    {
      const Real c1h = (Real)(kCd[1] * h);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const cx<Real> q = lin(y[m], m, sig0, m == E / 2);
        const cx<Real> kn = {q.re - gn * va[m].im, q.im + gn * va[m].re};
        k[m] = kn;
        acc[m] = kn;
        const cx<Real> kt = {vb[m].re - gt * bt[m].im, vb[m].im + gt * bt[m].re};
        va[m] = {yt[m].re + c1h * kt.re, yt[m].im + c1h * kt.im};  // a_2
      });
    }
    // ---- R2, R3: DFT(b_s) and IDFT(L_s u_s + p), s = 2, 3
    sfor<1, 3>([&](auto si) {
      constexpr int s = decltype(si)::value;  // 0-based stage index
      const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + kCd[s] * h);
      const Real ch = (Real)(kCd[s] * h);
      const Real cnh = (Real)(kCd[s + 1] * h);
      cx<Real> u[E];
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const Real pw = va[m].re * va[m].re + va[m].im * va[m].im;
        bt[m] = {pw * va[m].re, pw * va[m].im};
        va[m] = bt[m];
        u[m] = {y[m].re + ch * k[m].re, y[m].im + ch * k[m].im};
        vb[m] = lin(u[m], m, sig, m == E / 2);
      });
      store_stage(n, s, u);
      begin_round();
      {
        cx<Real> *ca = ctx(0), *cb = ctx(1);
        back_phase1<N, E, 1, TP, -1, PS>(va, ca, tw, w, lane);
        fwd_phase1<N, E, 1, TP, +1, PS>(vb, cb, tw, w, lane);
        cross_sync<W>();
        back_phase2<N, E, 1, TP, -1, PS>(va, ca, tw, w, lane);
        fwd_phase2<N, E, 1, TP, +1, PS>(vb, cb, tw, w, lane);
      }
      ++round;
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const cx<Real> uu = {y[m].re + ch * k[m].re, y[m].im + ch * k[m].im};
        const cx<Real> q = lin(uu, m, sig, m == E / 2);
        const cx<Real> kn = {q.re - gn * va[m].im, q.im + gn * va[m].re};
        k[m] = kn;
        acc[m] = {acc[m].re + (Real)2 * kn.re, acc[m].im + (Real)2 * kn.im};
        const cx<Real> kt = {vb[m].re - gt * bt[m].im, vb[m].im + gt * bt[m].re};
        va[m] = {yt[m].re + cnh * kt.re, yt[m].im + cnh * kt.im};  // a_{s+2}
      });
    });
    // ---- R4: DFT(b_4)
    {
      const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + kCd[3] * h);
      const Real ch = (Real)(kCd[3] * h);
      cx<Real> u[E];
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const Real pw = va[m].re * va[m].re + va[m].im * va[m].im;
        va[m] = {pw * va[m].re, pw * va[m].im};
        u[m] = {y[m].re + ch * k[m].re, y[m].im + ch * k[m].im};
      });
      store_stage(n, 3, u);
      begin_round();
      {
        cx<Real> *ca = ctx(0);
        back_phase1<N, E, 1, TP, -1, PS>(va, ca, tw, w, lane);
        cross_sync<W>();
        back_phase2<N, E, 1, TP, -1, PS>(va, ca, tw, w, lane);
      }
      ++round;
      const Real h6 = (Real)(h / 6.0);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const cx<Real> q = lin(u[m], m, sig, m == E / 2);
        const cx<Real> kn = {q.re - gn * va[m].im, q.im + gn * va[m].re};
        const cx<Real> ac = {acc[m].re + kn.re, acc[m].im + kn.im};
        y[m] = {y[m].re + h6 * ac.re, y[m].im + h6 * ac.im};
      });
    }
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

template <typename Real, int N, int E, int PS, int TP>
hipError_t launch_dual_fwd(const RunArgs &a, hipStream_t st) {
  using SH = DualShape<Real, N, E, PS, TP>;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((rk4_dual<Real, N, E, PS, TP>), dim3(grid), dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

// defined in cme_wave.hip: the reverse kernel does not depend on how the
// forward trajectory was evaluated
template <typename Real, int N, int E, int V, int PS, int TP>
hipError_t launch_wave_adj(const AdjArgs &a, hipStream_t st);

template <typename Real, int N, int E, int PS, int TP> constexpr Variant dual_variant() {
  using SH = DualShape<Real, N, E, PS, TP>;
  return Variant{std::is_same<Real, double>::value ? 0 : 1, N, E, 1, PS, TP, 2, SH::IPB,
                 SH::THREADS, SH::LDS_BYTES, &launch_dual_fwd<Real, N, E, PS, TP>,
                 &launch_wave_adj<Real, N, E, 1, PS, TP>};
}

static const Variant kDualVariants[] = {
    dual_variant<double, 512, 8, 3, 0>(),  dual_variant<double, 512, 8, 3, 1>(),
    dual_variant<double, 1024, 8, 3, 0>(), dual_variant<double, 1024, 8, 3, 1>(),
    dual_variant<double, 2048, 8, 3, 0>(), dual_variant<double, 2048, 8, 3, 1>(),
    dual_variant<double, 2048, 8, 3, 2>(), dual_variant<double, 4096, 8, 3, 0>(),
    dual_variant<double, 4096, 8, 3, 1>(),
};

const Variant *variants_dual(int *count) {
  *count = (int)(sizeof(kDualVariants) / sizeof(kDualVariants[0]));
  return kDualVariants;
}

}  // namespace cme
