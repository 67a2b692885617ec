// cme_wave.hpp -- persistent RK4 kernels on the two-level (wave-decomposed)
// transform of cme_fft.hpp.
//
// One instance per workgroup of W wavefronts (W = N / (64 E)), or, when one
// wavefront holds a whole instance (W = 1), four instances per workgroup that
// never synchronise with each other.  Per transform there is one workgroup
// barrier (the transpose across waves); all other exchanges are wave-local.
// The RK4 stage arithmetic is the one described in cme_kernels.hip: per
// stage u = y + c h k, a = inverse transform (Eq. (4)), b = |a|^2 a,
// NK = forward transform, k = (-kappa/2 + i(omega' - sigma)) u + i (g0/N) NK
// + pump at mu = 0, acc += w k; then y += h/6 acc.
#pragma once

#include <type_traits>

#include "cme_fft.hpp"
#include "cme_internal.hpp"

namespace cme {

// RK4 nodes c_s, derivative weights (times 6) and weights
__device__ constexpr double kCw[4] = {0.0, 0.5, 0.5, 1.0};
__device__ constexpr double kWrw[4] = {1.0, 2.0, 2.0, 1.0};
__device__ constexpr double kWbw[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

template <typename Real, int N, int E, int V, int PS, int TP> struct WaveShape {
  using WP = WavePlan<N, E, V, TP>;
  static constexpr int W = WP::W;
  static constexpr int WV = WP::WV;
  static constexpr int IPB = W == 1 ? 4 : 1;
  static constexpr int LB1 = LdsLen<WP::N1, PS>::value;
  static constexpr int LIMIT = 160 * 1024;
  static constexpr bool TWO = WV > 1 && 2 * IPB * WV * LB1 * (int)sizeof(cx<Real>) <= LIMIT;
  static constexpr int NBUF = TWO ? 2 : 1;
  static constexpr int PER_INST = NBUF * WV * LB1;
  static constexpr int LDS_BYTES = IPB * PER_INST * (int)sizeof(cx<Real>);
  static constexpr int THREADS = IPB * WP::T;
  static_assert(LDS_BYTES <= LIMIT, "LDS over the gfx950 per-workgroup limit");
  static_assert(THREADS <= 1024, "workgroup too large");
  static_assert(TP == 0 || PS == 3, "register-transpose sub-transforms use the 1-in-8 padded region");
};

// REC: record the stage inputs and inverse transforms for the adjoint
// (a separate instantiation, so the plain run carries none of its code).
// PAD: alias-free truncated sum -- the instance's N/2 modes sit in the middle
// of this N-point transform (transform index i <-> mode i - N/4 of the
// caller's state), the other half stays zero (its derivative is masked), so
// the cyclic sum of Eq. (4) over 2x padding equals the literal sum of Eq. (2)
// over the instance's own modes.
template <typename Real, int N, int E, int V, int PS, int TP, bool REC, bool PAD = false>
__global__ void __launch_bounds__((WaveShape<Real, N, E, V, PS, TP>::THREADS)) rk4_wave(RunArgs a) {
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
  static_assert(!(PAD && REC), "padded plans have no adjoint");
  constexpr int Q4 = N / 4;
  // caller's state of this instance, and where transform index i lives in it
  cx<Real> *A = reinterpret_cast<cx<Real> *>(a.A) + (PAD ? d.a_offset : d.offset);
  auto in_band = [](int i) { return !PAD || (i >= Q4 && i < 3 * Q4); };
  auto phys = [](int i) { return PAD ? i - Q4 : i; };
  const double *kap = a.kappa + d.offset;
  const double *omg = a.omega + d.offset;

  WaveTwiddles<N, E, V, TP, Real> tw;
  load_wave_twiddles<N, E, V>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  cx<Real> y[E], k[E], acc[E], v[E];
  Real lr[E];
  double om[E];
  bool band[E];
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = WP::mode(w, lane, m);
    band[m] = in_band(i);
    y[m] = band[m] ? A[phys(i)] : cx<Real>{(Real)0, (Real)0};
    lr[m] = (Real)(-0.5 * kap[i]);
    om[m] = omg[i];
    k[m] = {(Real)0, (Real)0};
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
      const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + kCw[s] * h);
      const Real ch = (Real)(kCw[s] * h);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        if constexpr (s == 0) v[m] = y[m];
        else v[m] = {y[m].re + ch * k[m].re, y[m].im + ch * k[m].im};
      });
      if constexpr (REC) {
        cx<Real> *st = stages + stage_offset(n, s, a.total) + d.offset;
        sfor<0, E>([&](auto mi) {
          constexpr int m = decltype(mi)::value;
          st[WP::mode(w, lane, m)] = v[m];
        });
      }
      fft_fwdpath<N, E, V, TP, +1, PS, !SH::TWO>(v, X, tw, w, lane);
      if constexpr (REC && V == 1 && TP == 0) {
        {
          cx<Real> *st = stages + stage_offset(n, s, a.total) + a.total + d.offset;
          sfor<0, E>([&](auto mi) {
            constexpr int m = decltype(mi)::value;
            st[WP::tslot(w, lane, m)] = v[m];
          });
        }
      }
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const Real p = v[m].re * v[m].re + v[m].im * v[m].im;
        v[m] = {p * v[m].re, p * v[m].im};
      });
      fft_backpath<N, E, V, TP, -1, PS>(v, X, Y, tw, w, lane);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        cx<Real> u;
        if constexpr (s == 0) u = y[m];
        else u = {y[m].re + ch * k[m].re, y[m].im + ch * k[m].im};
        const Real det = (Real)(om[m] - sig);
        cx<Real> kn = {lr[m] * u.re - det * u.im - gn * v[m].im,
                       lr[m] * u.im + det * u.re + gn * v[m].re};
        if constexpr (m == E / 2) {
          if (pump_owner) kn = cadd(kn, pump);
        }
        if constexpr (PAD) {
          if (!band[m]) kn = {(Real)0, (Real)0};
        }
        k[m] = kn;
        if constexpr (s == 0) acc[m] = kn;
        else {
          const Real wt = (Real)kWrw[s];
          acc[m] = {acc[m].re + wt * kn.re, acc[m].im + wt * kn.im};
        }
      });
    });
    const Real h6 = (Real)(h / 6.0);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      y[m] = {y[m].re + h6 * acc[m].re, y[m].im + h6 * acc[m].im};
    });
    if (ckpt != nullptr && --to_ckpt == 0) {
      to_ckpt = a.ckpt_every;
      cx<Real> *dst = ckpt + ckpt_slot * a.total + (PAD ? d.a_offset : d.offset);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const int i = WP::mode(w, lane, m);
        if (band[m]) dst[phys(i)] = y[m];
      });
      ++ckpt_slot;
    }
  }
  bool bad = false;
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = WP::mode(w, lane, m);
    if (band[m]) A[phys(i)] = y[m];
    bad |= !(isfinite(y[m].re) && isfinite(y[m].im));
  });
  if (bad) atomicOr(&a.flags[id], 1);
}

template <typename Real, int N, int E, int V, int PS, int TP>
__global__ void __launch_bounds__((WaveShape<Real, N, E, V, PS, TP>::THREADS)) rk4_wave_reverse(AdjArgs a) {
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
    if (slot >= a.count) return;
  }
  const int id = a.order[slot];
  const DevInst d = a.inst[id];
  cx<Real> *X = lds + sub * SH::PER_INST;
  cx<Real> *Y = SH::TWO ? X + SH::WV * SH::LB1 : X;
  const double *kap = a.kappa + d.offset;
  const double *omg = a.omega + d.offset;
  cx<Real> *gA = reinterpret_cast<cx<Real> *>(a.gA) + d.offset;
  const cx<Real> *stages = reinterpret_cast<const cx<Real> *>(a.stages);

  WaveTwiddles<N, E, V, TP, Real> tw;
  load_wave_twiddles<N, E, V>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  cx<Real> yb1[E], yb[E], ub[E], z[E], fa[E];
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
      const Real wb = (Real)(kWbw[s] * h);
      const Real cn = (Real)(s < 3 ? kCw[s < 3 ? s + 1 : 3] * h : 0.0);
      // kbar = w_s h ybar' + c_{s+1} h ubar_{s+1}; z <- (-i g0/N) kbar
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        cx<Real> kv = {wb * yb1[m].re, wb * yb1[m].im};
        if constexpr (s < 3) kv = {kv.re + cn * ub[m].re, kv.im + cn * ub[m].im};
        z[m] = {gn * kv.im, -gn * kv.re};
      });
      const cx<Real> *us = stages + stage_offset(nn, s, a.total) + d.offset;
      fft_fwdpath<N, E, V, TP, +1, PS, true>(z, X, tw, w, lane);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        fa[m] = us[WP::mode(w, lane, m)];
      });
      fft_fwdpath<N, E, V, TP, +1, PS, true>(fa, X, tw, w, lane);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const cx<Real> av = fa[m], zv = z[m];
        const Real p2 = (Real)2 * (av.re * av.re + av.im * av.im);
        const cx<Real> a2 = {av.re * av.re - av.im * av.im, (Real)2 * av.re * av.im};
        z[m] = {p2 * zv.re + a2.re * zv.re + a2.im * zv.im,
                p2 * zv.im + a2.im * zv.re - a2.re * zv.im};
      });
      fft_backpath<N, E, V, TP, -1, PS>(z, X, Y, tw, w, lane);
      const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + kCw[s] * h);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        cx<Real> kv = {wb * yb1[m].re, wb * yb1[m].im};
        if constexpr (s < 3) kv = {kv.re + cn * ub[m].re, kv.im + cn * ub[m].im};
        const cx<Real> u = us[WP::mode(w, lane, m)];
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

template <typename Real, int N, int E, int V, int PS, int TP>
hipError_t launch_wave_fwd(const RunArgs &a, hipStream_t st) {
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  if (a.stages)
    hipLaunchKernelGGL((rk4_wave<Real, N, E, V, PS, TP, true>), dim3(grid), dim3(SH::THREADS), 0,
                       st, a);
  else
    hipLaunchKernelGGL((rk4_wave<Real, N, E, V, PS, TP, false>), dim3(grid), dim3(SH::THREADS), 0,
                       st, a);
  return hipGetLastError();
}

template <typename Real, int N, int E, int V, int PS, int TP>
hipError_t launch_wave_adj(const AdjArgs &a, hipStream_t st) {
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((rk4_wave_reverse<Real, N, E, V, PS, TP>), dim3(grid), dim3(SH::THREADS), 0,
                     st, a);
  return hipGetLastError();
}

template <typename Real, int N, int E, int V, int PS, int TP>
hipError_t launch_wave_pad(const RunArgs &a, hipStream_t st) {
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((rk4_wave<Real, N, E, V, PS, TP, false, true>), dim3(grid), dim3(SH::THREADS),
                     0, st, a);
  return hipGetLastError();
}

// Padded-sum variant (kind 5): transform size N for instances of N/2 modes.
template <typename Real, int N, int E, int V, int PS, int TP = 0> constexpr Variant pad_variant() {
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  return Variant{std::is_same<Real, double>::value ? 0 : 1, N, E, V, PS, TP, 5, SH::IPB,
                 SH::THREADS, SH::LDS_BYTES, &launch_wave_pad<Real, N, E, V, PS, TP>, nullptr};
}

// defined in cme_lean.hip (FP64, E = 8, PS = 3): the reverse sweep that
// reads the stored time-domain stage fields (two transforms per stage)
template <typename Real, int N, int E, int PS>
hipError_t launch_lean_adj(const AdjArgs &a, hipStream_t st);

// The reverse (adjoint) kernels exist in FP64 only.  Variants that store the
// time-domain stage fields in the lean slot order (E = 8, V = 1, Stockham
// sub-transforms, 1-in-8 padding) share the lean reverse sweep; the others
// recompute the field from the stage input.
template <typename Real, int N, int E, int V, int PS, int TP> constexpr AdjLaunch wave_adj_ptr() {
  if constexpr (!std::is_same<Real, double>::value) return nullptr;
  else if constexpr (E == 8 && V == 1 && TP == 0 && PS == 3 && N >= 512 && N <= 4096)
    return &launch_lean_adj<Real, N, E, PS>;
  else return &launch_wave_adj<Real, N, E, V, PS, TP>;
}

template <typename Real, int N, int E, int V, int PS, int TP = 0> constexpr Variant wave_variant() {
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  return Variant{std::is_same<Real, double>::value ? 0 : 1, N, E, V, PS, TP, 1, SH::IPB,
                 SH::THREADS, SH::LDS_BYTES, &launch_wave_fwd<Real, N, E, V, PS, TP>,
                 wave_adj_ptr<Real, N, E, V, PS, TP>()};
}

}  // namespace cme

