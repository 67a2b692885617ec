// cme_lean.hip -- two-level kernels with a small register footprint, so that
// two wavefronts share each SIMD: classic RK4 (cyclic or padded sum), its
// reverse sweep, and the interaction-picture RK4.
//
// The kernels of cme_wave.hpp keep every per-thread twiddle of the two-level
// transform in registers and, with the RK4 state, need more than 256
// registers per lane at E = 8: one wavefront per SIMD, whose LDS waits and
// arithmetic cannot overlap.  These use the transform of cme_lean.hpp
// (twiddles rebuilt on use), and the RK4 state is y, the weighted
// derivative sum, and the stage input u (the transform works on a copy),
// i.e. the previous derivative is not kept: u of the next stage is formed as
// soon as a derivative is known.  The arithmetic per stage is that of
// cme_wave.hpp (Eq. (4) for the four-wave-mixing sum, Eq. (1) for the
// derivative); only the rounding of the rebuilt twiddles differs.
#include "cme_internal.hpp"
#include "cme_lean.hpp"

namespace cme {

namespace {
__device__ constexpr double kLeanC[4] = {0.0, 0.5, 0.5, 1.0};
__device__ constexpr double kLeanW[4] = {1.0, 2.0, 2.0, 1.0};
}  // namespace

template <typename Real, int N, int E, int PS> struct LeanShape {
  using LP = LeanPlan<N, E>;
  static constexpr int W = LP::W;
  static constexpr int WV = LP::WV;
  static constexpr int IPB = W == 1 ? 4 : 1;
  static constexpr int LB1 = LdsLen<LP::N1, PS>::value;
  static constexpr int LIMIT = 160 * 1024;
  // two exchange buffers when two workgroups still fit a CU (or one
  // workgroup already fills two waves per SIMD)
  static constexpr int ONE = IPB * WV * LB1 * (int)sizeof(cx<Real>);
  static constexpr bool TWO = WV > 1 && (4 * ONE <= LIMIT || (W >= 8 && 2 * ONE <= LIMIT));
  static constexpr int NBUF = TWO ? 2 : 1;
  static constexpr int PER_INST = NBUF * WV * LB1;
  static constexpr int LDS_BYTES = IPB * PER_INST * (int)sizeof(cx<Real>);
  static constexpr int THREADS = IPB * 64 * W;
  static_assert(LDS_BYTES <= LIMIT, "LDS over the gfx950 per-workgroup limit");
  static_assert(THREADS <= 1024, "workgroup too large");
};

// REC: record the stage inputs and inverse transforms for the adjoint
// PAD: the alias-free truncated sum, as in the wave kernels: the instance's
// N/2 modes at transform indices [N/4, 3N/4), the derivative zero elsewhere.
template <typename Real, int N, int E, int PS, bool REC, bool PAD = false>
__global__ void __launch_bounds__((LeanShape<Real, N, E, PS>::THREADS))
    __attribute__((amdgpu_waves_per_eu(2))) rk4_lean(RunArgs a) {
  using SH = LeanShape<Real, N, E, PS>;
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
  static_assert(!(PAD && REC), "padded plans have no adjoint");
  constexpr int Q4 = N / 4;
  auto in_band = [](int i) { return !PAD || (i >= Q4 && i < 3 * Q4); };
  auto phys = [](int i) { return PAD ? i - Q4 : i; };  // index in the caller's state
  cx<Real> *A = reinterpret_cast<cx<Real> *>(a.A) + (PAD ? d.a_offset : d.offset);
  const double *kap = a.kappa + d.offset;
  const double *omg = a.omega + d.offset;

  LeanTw<N, E, Real> tw;
  load_lean_twiddles<N, E>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  cx<Real> y[E], acc[E], u[E], v[E];
  Real lr[E];
  double om[E];
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = WP::mode(w, lane, m);
    y[m] = in_band(i) ? A[phys(i)] : cx<Real>{(Real)0, (Real)0};
    lr[m] = (Real)(-0.5 * kap[i]);
    om[m] = omg[i];
  });
  const bool pump_owner = (w == 0 && lane == 0);
  const Real gn = (Real)d.g0n;
  const cx<Real> pump = {(Real)d.pump_re, (Real)d.pump_im};
  const double h = a.h;
  cx<Real> *ckpt = reinterpret_cast<cx<Real> *>(a.ckpt);
  cx<Real> *stages = reinterpret_cast<cx<Real> *>(a.stages);
  int32_t to_ckpt = a.ckpt_every;
  int64_t ckpt_slot = 0;

  for (int64_t n = 0; n < a.n_steps; ++n) {
    const double t0 = (double)(a.step0 + n) * h;
    sfor<0, 4>([&](auto si) {
      constexpr int s = decltype(si)::value;
      const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + kLeanC[s] * h);
      if constexpr (s == 0) {
        sfor<0, E>([&](auto mi) { u[decltype(mi)::value] = y[decltype(mi)::value]; });
      }
      if constexpr (REC) {
        cx<Real> *st = stages + stage_offset(n, s, a.total) + d.offset;
        sfor<0, E>([&](auto mi) {
          constexpr int m = decltype(mi)::value;
          st[WP::mode(w, lane, m)] = u[m];
        });
      }
      sfor<0, E>([&](auto mi) { v[decltype(mi)::value] = u[decltype(mi)::value]; });
      lean_fwdpath<N, E, +1, PS, !SH::TWO>(v, X, tw, w, lane);
      if constexpr (REC) {
        cx<Real> *st = stages + stage_offset(n, s, a.total) + a.total + d.offset;
        sfor<0, E>([&](auto mi) {
          constexpr int m = decltype(mi)::value;
          st[WP::tslot(w, lane, m)] = v[m];
        });
      }
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const Real p = v[m].re * v[m].re + v[m].im * v[m].im;
        v[m] = {p * v[m].re, p * v[m].im};
      });
      lean_backpath<N, E, -1, PS>(v, X, Y, tw, w, lane);
      const Real chn = (Real)(kLeanC[s < 3 ? s + 1 : 3] * h);
      const Real h6 = (Real)(h / 6.0);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const Real det = (Real)(om[m] - sig);
        cx<Real> kn = {lr[m] * u[m].re - det * u[m].im - gn * v[m].im,
                       lr[m] * u[m].im + det * u[m].re + gn * v[m].re};
        if constexpr (m == E / 2) {
          if (pump_owner) kn = cadd(kn, pump);
        }
        if constexpr (PAD) {
          if (!in_band(WP::mode(w, lane, m))) kn = {(Real)0, (Real)0};
        }
        if constexpr (s == 0) acc[m] = kn;
        else {
          const Real wt = (Real)kLeanW[s];
          acc[m] = {acc[m].re + wt * kn.re, acc[m].im + wt * kn.im};
        }
        if constexpr (s < 3) u[m] = {y[m].re + chn * kn.re, y[m].im + chn * kn.im};
        else y[m] = {y[m].re + h6 * acc[m].re, y[m].im + h6 * acc[m].im};
      });
    });
    if (ckpt != nullptr && --to_ckpt == 0) {
      to_ckpt = a.ckpt_every;
      cx<Real> *dst = ckpt + ckpt_slot * a.total + (PAD ? d.a_offset : d.offset);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const int i = WP::mode(w, lane, m);
        if (in_band(i)) dst[phys(i)] = y[m];
      });
      ++ckpt_slot;
    }
  }
  bool bad = false;
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = WP::mode(w, lane, m);
    if (in_band(i)) A[phys(i)] = y[m];
    bad |= !(isfinite(y[m].re) && isfinite(y[m].im));
  });
  if (bad) atomicOr(&a.flags[id], 1);
}

// Reverse sweep over one checkpoint segment (the discrete adjoint of the
// RK4 map of rk4_lean, steps in reverse).  Per stage, from the cotangent
// ybar' of the step's output and ubar_{s+1} of the later stage:
//   kbar_s = w_s h ybar' + c_{s+1} h ubar_{s+1}
//   ubar_s = conj(L_s) kbar_s + V(-i g0 kbar_s),
//   V(w') = DFT[2 |a_s|^2 z + a_s^2 conj(z)],  z = IDFT(w') / N,
// with a_s = IDFT(u_s) read back from the stage buffer (stored by the
// forward recompute), so a stage costs two transforms; ybar = ybar' +
// sum_s ubar_s, and the parameter gradients accumulate
//   gbar_omega += Re(conj(kbar) i u),  gbar_kappa -= Re(conj(kbar) u) / 2,
//   gbar_Ain   += sqrt(kappa_ext) kbar at mu = 0.
// The 1/N of z is folded into g0/N.
template <typename Real, int N, int E, int PS>
__global__ void __launch_bounds__((LeanShape<Real, N, E, PS>::THREADS)) rk4_lean_reverse(AdjArgs a) {
  using SH = LeanShape<Real, N, E, PS>;
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
  const double *kap = a.kappa + d.offset;
  const double *omg = a.omega + d.offset;
  cx<Real> *gA = reinterpret_cast<cx<Real> *>(a.gA) + d.offset;
  const cx<Real> *stages = reinterpret_cast<const cx<Real> *>(a.stages);

  LeanTw<N, E, Real> tw;
  load_lean_twiddles<N, E>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  cx<Real> yb1[E], yb[E], ub[E], z[E];
  Real lr[E], gom[E], gka[E];
  double om[E];
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = WP::mode(w, lane, m);
    yb1[m] = gA[i];
    lr[m] = (Real)(-0.5 * kap[i]);
    om[m] = omg[i];
    gom[m] = (Real)0;
    gka[m] = (Real)0;
    ub[m] = {(Real)0, (Real)0};
  });
  const bool pump_owner = (w == 0 && lane == 0);
  cx<Real> gain = {(Real)0, (Real)0};
  const Real gn = (Real)d.g0n;
  const double h = a.h;

  for (int nn = a.n_seg - 1; nn >= 0; --nn) {
    const double t0 = (double)(a.step_first + nn) * h;
    sfor<0, E>([&](auto mi) { yb[decltype(mi)::value] = yb1[decltype(mi)::value]; });
    sfor<0, 4>([&](auto ri) {
      constexpr int s = 3 - decltype(ri)::value;
      const Real wb = (Real)(kLeanW[s] / 6.0 * h);
      const Real cn = (Real)(s < 3 ? kLeanC[s < 3 ? s + 1 : 3] * h : 0.0);
      // the stage record is loaded first, so that its latency hides behind
      // the transforms
      const cx<Real> *rec = stages + stage_offset(nn, s, a.total) + d.offset;
      cx<Real> ar[E], ur[E];
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        ar[m] = rec[a.total + WP::tslot(w, lane, m)];
        ur[m] = rec[WP::mode(w, lane, m)];
      });
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        cx<Real> kv = {wb * yb1[m].re, wb * yb1[m].im};
        if constexpr (s < 3) kv = {kv.re + cn * ub[m].re, kv.im + cn * ub[m].im};
        z[m] = {gn * kv.im, -gn * kv.re};
      });
      lean_fwdpath<N, E, +1, PS, !SH::TWO>(z, X, tw, w, lane);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const cx<Real> av = ar[m], zv = z[m];
        const Real p2 = (Real)2 * (av.re * av.re + av.im * av.im);
        const cx<Real> a2 = {av.re * av.re - av.im * av.im, (Real)2 * av.re * av.im};
        z[m] = {p2 * zv.re + a2.re * zv.re + a2.im * zv.im,
                p2 * zv.im + a2.im * zv.re - a2.re * zv.im};
      });
      lean_backpath<N, E, -1, PS>(z, X, Y, tw, w, lane);
      const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + kLeanC[s] * h);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        cx<Real> kv = {wb * yb1[m].re, wb * yb1[m].im};
        if constexpr (s < 3) kv = {kv.re + cn * ub[m].re, kv.im + cn * ub[m].im};
        const cx<Real> u = ur[m];
        const Real det = (Real)(om[m] - sig);
        const cx<Real> unew = {lr[m] * kv.re + det * kv.im + z[m].re,
                               lr[m] * kv.im - det * kv.re + z[m].im};
        ub[m] = unew;
        yb[m] = cadd(yb[m], unew);
        gom[m] += kv.im * u.re - kv.re * u.im;
        gka[m] -= (Real)0.5 * (kv.re * u.re + kv.im * u.im);
        if constexpr (m == E / 2) {
          if (pump_owner) gain = cadd(gain, kv);
        }
      });
    });
    sfor<0, E>([&](auto mi) { yb1[decltype(mi)::value] = yb[decltype(mi)::value]; });
  }
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = WP::mode(w, lane, m);
    gA[i] = yb1[m];
    if (a.g_omega) a.g_omega[d.offset + i] += (double)gom[m];
    if (a.g_kappa) a.g_kappa[d.offset + i] += (double)gka[m];
  });
  if (pump_owner && a.g_ain) {
    a.g_ain[2 * id] += d.sqrt_kext * (double)gain.re;
    a.g_ain[2 * id + 1] += d.sqrt_kext * (double)gain.im;
  }
}

template <typename Real, int N, int E, int PS>
hipError_t launch_lean_adj(const AdjArgs &a, hipStream_t st) {
  using SH = LeanShape<Real, N, E, PS>;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((rk4_lean_reverse<Real, N, E, PS>), dim3(grid), dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

template <typename Real, int N, int E, int PS>
hipError_t launch_lean_fwd(const RunArgs &a, hipStream_t st) {
  using SH = LeanShape<Real, N, E, PS>;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  if (a.stages)
    hipLaunchKernelGGL((rk4_lean<Real, N, E, PS, true>), dim3(grid), dim3(SH::THREADS), 0, st, a);
  else
    hipLaunchKernelGGL((rk4_lean<Real, N, E, PS, false>), dim3(grid), dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

// Interaction-picture RK4 (the step of cme_rk4ip.hip) on the lean
// transforms, for eight wavefronts per instance at two per SIMD: the state y
// (y_I after the first stage), the accumulated k, the transform array and the
// per-mode factor exp((-kappa/2 + i omega') h/2) per thread.
template <typename Real, int N, int E, int PS>
__global__ void __launch_bounds__((LeanShape<Real, N, E, PS>::THREADS))
    __attribute__((amdgpu_waves_per_eu(2))) rk4ip_lean(RunArgs a) {
  using SH = LeanShape<Real, N, E, PS>;
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

  // v <- N(v) = i (g0/N) DFT(|IDFT v|^2 IDFT v) + pump
  auto nonlinear = [&]() {
    lean_fwdpath<N, E, +1, PS, !SH::TWO>(v, X, tw, w, lane);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const Real p = v[m].re * v[m].re + v[m].im * v[m].im;
      v[m] = {p * v[m].re, p * v[m].im};
    });
    lean_backpath<N, E, -1, PS>(v, X, Y, tw, w, lane);
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
    sfor<0, E>([&](auto mi) { v[decltype(mi)::value] = y[decltype(mi)::value]; });
    nonlinear();  // k1 = P1 N(y), yI = P1 y
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const cx<Real> p1 = cmul(dm[m], c1);
      acc[m] = cmul(p1, v[m]);
      y[m] = cmul(p1, y[m]);
      v[m] = {y[m].re + hh * acc[m].re, y[m].im + hh * acc[m].im};
    });
    nonlinear();  // k2 = N(yI + h/2 k1)
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      acc[m] = {acc[m].re + (Real)2 * v[m].re, acc[m].im + (Real)2 * v[m].im};
      v[m] = {y[m].re + hh * v[m].re, y[m].im + hh * v[m].im};
    });
    nonlinear();  // k3 = N(yI + h/2 k2)
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      acc[m] = {acc[m].re + (Real)2 * v[m].re, acc[m].im + (Real)2 * v[m].im};
      v[m] = cmul(cmul(dm[m], c2), cx<Real>{y[m].re + hf * v[m].re, y[m].im + hf * v[m].im});
    });
    nonlinear();  // k4 = N(P2 (yI + h k3)); y' = P2 (yI + h/6 acc) + h/6 k4
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

template <typename Real, int N, int E, int PS>
hipError_t launch_rk4ip_lean(const RunArgs &a, hipStream_t st) {
  using SH = LeanShape<Real, N, E, PS>;
  if (a.stages) return hipErrorInvalidValue;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((rk4ip_lean<Real, N, E, PS>), dim3(grid), dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

// interaction-picture RK4 (kind 12)
template <typename Real, int N, int E, int PS> constexpr Variant rk4ip_lean_variant() {
  using SH = LeanShape<Real, N, E, PS>;
  return Variant{std::is_same<Real, double>::value ? 0 : 1, N, E, 1, PS, 0, 12, SH::IPB,
                 SH::THREADS, SH::LDS_BYTES, &launch_rk4ip_lean<Real, N, E, PS>, nullptr};
}

template <typename Real, int N, int E, int PS>
hipError_t launch_lean_pad(const RunArgs &a, hipStream_t st) {
  using SH = LeanShape<Real, N, E, PS>;
  if (a.stages) return hipErrorInvalidValue;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((rk4_lean<Real, N, E, PS, false, true>), dim3(grid), dim3(SH::THREADS), 0,
                     st, a);
  return hipGetLastError();
}

// padded sum (kind 11): transform length N for instances of N/2 modes
template <typename Real, int N, int E, int PS> constexpr Variant lean_pad_variant() {
  using SH = LeanShape<Real, N, E, PS>;
  return Variant{0, N, E, 1, PS, 0, 11, SH::IPB, SH::THREADS, SH::LDS_BYTES,
                 &launch_lean_pad<Real, N, E, PS>, nullptr};
}

template <typename Real, int N, int E, int PS> constexpr Variant lean_variant() {
  using SH = LeanShape<Real, N, E, PS>;
  return Variant{std::is_same<Real, double>::value ? 0 : 1, N, E, 1, PS, 0, 3, SH::IPB,
                 SH::THREADS, SH::LDS_BYTES, &launch_lean_fwd<Real, N, E, PS>,
                 &launch_lean_adj<Real, N, E, PS>};
}

// The wave kernels with E = 8, V = 1 and Stockham sub-transforms store their
// stage records in the same slot order and use this reverse sweep too.
template hipError_t launch_lean_adj<double, 512, 8, 3>(const AdjArgs &, hipStream_t);
template hipError_t launch_lean_adj<double, 1024, 8, 3>(const AdjArgs &, hipStream_t);
template hipError_t launch_lean_adj<double, 2048, 8, 3>(const AdjArgs &, hipStream_t);
template hipError_t launch_lean_adj<double, 4096, 8, 3>(const AdjArgs &, hipStream_t);

static const Variant kLeanVariants[] = {
    lean_variant<double, 512, 8, 3>(),
    lean_variant<double, 1024, 8, 3>(),
    lean_variant<double, 2048, 8, 3>(),
    lean_variant<double, 4096, 8, 3>(),
    // the padded sum for 2048-mode instances: eight wavefronts, two per SIMD
    // (the default there; listed ahead of the wave kernel's padded variant)
    lean_pad_variant<double, 4096, 8, 3>(),
    // the interaction-picture RK4 at N = 4096 (the default there)
    rk4ip_lean_variant<double, 4096, 8, 3>(),
};

const Variant *variants_lean(int *count) {
  *count = (int)(sizeof(kLeanVariants) / sizeof(kLeanVariants[0]));
  return kLeanVariants;
}

}  // namespace cme
