// cme_kernels.hip -- persistent RK4 kernels for the coupled mode equations.
//
// One team of T = N / E threads integrates one instance (resonator) for all
// requested steps without leaving the chip: the state y, the RK4 accumulator
// and the previous stage slope live in the registers of the thread that owns
// each mode (mode i = t + m T), and the two transforms of every stage go
// through the team's LDS buffers (cme_fft.hpp).  Per RK4 stage (Sec. 2 of
// Hansson, Modotto & Wabnitz, arXiv:1307.3428):
//   u  = y + c_s h k                     (registers)
//   a  = sum_mu u_mu e^{+2 pi i j mu/N}  (inverse transform, Eq. (4))
//   b  = |a|^2 a                         (registers)
//   NK = sum_j b_j e^{-2 pi i j mu/N}    (forward transform; K = NK / N)
//   k  = (-kappa/2 + i(omega' - sigma(t_s))) u + i (g0/N) NK + [mu=0] pump
//   acc += w_s k
// then y += h/6 acc.  Eq. (1) in the rotating frame is the equation solved.
//
// The reverse kernel is the discrete adjoint of the same map (not in the
// paper): per stage, from the stored stage input u_s,
//   kbar = (weights) ybar' + c h ubar_next,
//   z    = inverse transform of (-i g0/N) kbar,  a = inverse transform of u_s,
//   V    = forward transform of (2|a|^2 z + a^2 conj(z)),
//   ubar = conj(L(t_s)) kbar + V,  ybar += ubar,
// with the parameter gradients accumulated in registers.
#include "cme_fft.hpp"
#include "cme_internal.hpp"

namespace cme {

// RK4 nodes and weights (classic Butcher tableau)
__device__ constexpr double kC[4] = {0.0, 0.5, 0.5, 1.0};
__device__ constexpr double kWr[4] = {1.0, 2.0, 2.0, 1.0};   // forward accumulation weights
__device__ constexpr double kWb[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

template <typename Real, int N, int E, int PS> struct KernelShape {
  using PL = FftPlan<N, E>;
  static constexpr int T = PL::T;
  static constexpr int IPB = T >= 64 ? 1 : 64 / T;
  static constexpr int LB = LdsLen<N, PS>::value;
  static constexpr int LDS_LIMIT = 160 * 1024;
  static constexpr bool PING = 2 * IPB * LB * (int)sizeof(cx<Real>) <= LDS_LIMIT;
  static constexpr int NBUF = PING ? 2 : 1;
  static constexpr int LDS_BYTES = IPB * NBUF * LB * (int)sizeof(cx<Real>);
  static constexpr int THREADS = IPB * T;
  // a workgroup of one wavefront orders its LDS exchanges without a
  // workgroup barrier (one wavefront's LDS operations execute in order)
  static constexpr int SYNC = THREADS <= 64 ? SYNC_WAVE : SYNC_BLOCK;
  static_assert(LDS_BYTES <= LDS_LIMIT, "LDS over the gfx950 per-workgroup limit");
  static_assert(THREADS <= 1024, "workgroup too large");
};

template <typename Real, int N, int E, int PS>
__global__ void __launch_bounds__((KernelShape<Real, N, E, PS>::THREADS))
    rk4_persistent(RunArgs a) {
  using SH = KernelShape<Real, N, E, PS>;
  using PL = FftPlan<N, E>;
  constexpr int T = SH::T;
  constexpr bool PING = SH::PING;
  constexpr int X = PL::P - 1;  // LDS exchanges per transform
  __shared__ cx<Real> lds[SH::IPB][SH::NBUF][SH::LB];

  const int sub = SH::IPB == 1 ? 0 : (int)threadIdx.x / T;
  const int t = SH::IPB == 1 ? (int)threadIdx.x : (int)threadIdx.x % T;
  const int slot = (int)blockIdx.x * SH::IPB + sub;
  const bool active = slot < a.count;
  const int id = a.order[active ? slot : a.count - 1];
  const DevInst d = a.inst[id];
  cx<Real> *buf0 = lds[sub][0];
  cx<Real> *buf1 = lds[sub][SH::NBUF - 1];
  cx<Real> *A = reinterpret_cast<cx<Real> *>(a.A) + d.offset;
  const double *kap = a.kappa + d.offset;
  const double *omg = a.omega + d.offset;

  cx<Real> tw[PL::NTW];
  load_twiddles<N, E>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), t);

  cx<Real> y[E], k[E], acc[E], v[E];
  Real lr[E];
  double om[E];
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = t + m * T;
    y[m] = A[i];
    lr[m] = (Real)(-0.5 * kap[i]);
    om[m] = omg[i];
    k[m] = {(Real)0, (Real)0};
  });
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
      const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + kC[s] * h);
      const Real ch = (Real)(kC[s] * h);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        if constexpr (s == 0) v[m] = y[m];
        else v[m] = {y[m].re + ch * k[m].re, y[m].im + ch * k[m].im};
      });
      if (stages != nullptr && active) {
        cx<Real> *st = stages + stage_offset(n, s, a.total) + d.offset;
        sfor<0, E>([&](auto mi) { st[t + decltype(mi)::value * T] = v[decltype(mi)::value]; });
      }
      fft_team<N, E, +1, PS, PING, 0, SH::SYNC>(v, buf0, buf1, tw, t);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const Real p = v[m].re * v[m].re + v[m].im * v[m].im;
        v[m] = {p * v[m].re, p * v[m].im};
      });
      fft_team<N, E, -1, PS, PING, (X & 1), SH::SYNC>(v, buf0, buf1, tw, t);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        cx<Real> u;
        if constexpr (s == 0) u = y[m];
        else u = {y[m].re + ch * k[m].re, y[m].im + ch * k[m].im};
        const Real det = (Real)(om[m] - sig);
        cx<Real> kn = {lr[m] * u.re - det * u.im - gn * v[m].im,
                       lr[m] * u.im + det * u.re + gn * v[m].re};
        if constexpr (m == E / 2) {
          if (t == 0) kn = cadd(kn, pump);
        }
        k[m] = kn;
        if constexpr (s == 0) acc[m] = kn;
        else {
          const Real w = (Real)kWr[s];
          acc[m] = {acc[m].re + w * kn.re, acc[m].im + w * kn.im};
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
      if (active) {
        cx<Real> *dst = ckpt + ckpt_slot * a.total + d.offset;
        sfor<0, E>([&](auto mi) { dst[t + decltype(mi)::value * T] = y[decltype(mi)::value]; });
      }
      ++ckpt_slot;
    }
  }
  if (active) {
    bool bad = false;
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      A[t + m * T] = y[m];
      bad |= !(isfinite(y[m].re) && isfinite(y[m].im));
    });
    if (bad) atomicOr(&a.flags[id], 1);
  }
}

template <typename Real, int N, int E, int PS>
__global__ void __launch_bounds__((KernelShape<Real, N, E, PS>::THREADS))
    rk4_reverse(AdjArgs a) {
  using SH = KernelShape<Real, N, E, PS>;
  using PL = FftPlan<N, E>;
  constexpr int T = SH::T;
  constexpr bool PING = SH::PING;
  constexpr int X = PL::P - 1;
  __shared__ cx<Real> lds[SH::IPB][SH::NBUF][SH::LB];

  const int sub = SH::IPB == 1 ? 0 : (int)threadIdx.x / T;
  const int t = SH::IPB == 1 ? (int)threadIdx.x : (int)threadIdx.x % T;
  const int slot = (int)blockIdx.x * SH::IPB + sub;
  const bool active = slot < a.count;
  const int id = a.order[active ? slot : a.count - 1];
  const DevInst d = a.inst[id];
  cx<Real> *buf0 = lds[sub][0];
  cx<Real> *buf1 = lds[sub][SH::NBUF - 1];
  const double *kap = a.kappa + d.offset;
  const double *omg = a.omega + d.offset;
  cx<Real> *gA = reinterpret_cast<cx<Real> *>(a.gA) + d.offset;
  const cx<Real> *stages = reinterpret_cast<const cx<Real> *>(a.stages);

  cx<Real> tw[PL::NTW];
  load_twiddles<N, E>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), t);

  cx<Real> yb1[E], yb[E], ub[E], kb[E], z[E], fa[E];
  Real lr[E], gom[E], gka[E];
  double om[E];
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = t + m * T;
    yb1[m] = gA[i];
    lr[m] = (Real)(-0.5 * kap[i]);
    om[m] = omg[i];
    gom[m] = (Real)0;
    gka[m] = (Real)0;
  });
  cx<Real> gain = {(Real)0, (Real)0};
  const Real gn = (Real)d.g0n;
  const double h = a.h;

  for (int nn = a.n_seg - 1; nn >= 0; --nn) {
    const double t0 = (double)(a.step_first + nn) * h;
    sfor<0, E>([&](auto mi) { yb[decltype(mi)::value] = yb1[decltype(mi)::value]; });
    sfor<0, 4>([&](auto ri) {
      constexpr int s = 3 - decltype(ri)::value;
      const Real wb = (Real)(kWb[s] * h);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        cx<Real> kv = {wb * yb1[m].re, wb * yb1[m].im};
        if constexpr (s < 3) {
          const Real cn = (Real)(kC[s + 1] * h);
          kv = {kv.re + cn * ub[m].re, kv.im + cn * ub[m].im};
        }
        kb[m] = kv;
        // z <- (-i g0/N) kbar, then inverse transform
        z[m] = {gn * kv.im, -gn * kv.re};
      });
      const cx<Real> *us = stages + stage_offset(nn, s, a.total) + d.offset;
      fft_team<N, E, +1, PS, PING, 0, SH::SYNC>(z, buf0, buf1, tw, t);
      sfor<0, E>([&](auto mi) { fa[decltype(mi)::value] = us[t + decltype(mi)::value * T]; });
      fft_team<N, E, +1, PS, PING, (X & 1), SH::SYNC>(fa, buf0, buf1, tw, t);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const cx<Real> av = fa[m], zv = z[m];
        const Real p2 = (Real)2 * (av.re * av.re + av.im * av.im);
        const cx<Real> a2 = {av.re * av.re - av.im * av.im, (Real)2 * av.re * av.im};
        // 2|a|^2 z + a^2 conj(z)
        z[m] = {p2 * zv.re + a2.re * zv.re + a2.im * zv.im,
                p2 * zv.im + a2.im * zv.re - a2.re * zv.im};
      });
      fft_team<N, E, -1, PS, PING, (2 * X) & 1, SH::SYNC>(z, buf0, buf1, tw, t);
      const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + kC[s] * h);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const cx<Real> kv = kb[m];
        const cx<Real> u = us[t + m * T];
        const Real det = (Real)(om[m] - sig);
        const cx<Real> unew = {lr[m] * kv.re + det * kv.im + z[m].re,
                               lr[m] * kv.im - det * kv.re + z[m].im};
        ub[m] = unew;
        yb[m] = cadd(yb[m], unew);
        gom[m] += kv.im * u.re - kv.re * u.im;
        gka[m] -= (Real)0.5 * (kv.re * u.re + kv.im * u.im);
        if constexpr (m == E / 2) {
          if (t == 0) gain = cadd(gain, kv);
        }
      });
      // the next stage's first transform writes buffer 0 again; parity of
      // this stage's 3 X exchanges may be odd, so fence it
      if constexpr (PING && ((3 * X) & 1)) team_sync<SH::SYNC>();
    });
    sfor<0, E>([&](auto mi) { yb1[decltype(mi)::value] = yb[decltype(mi)::value]; });
  }
  if (active) {
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const int i = t + m * T;
      gA[i] = yb1[m];
      if (a.g_omega) a.g_omega[d.offset + i] += (double)gom[m];
      if (a.g_kappa) a.g_kappa[d.offset + i] += (double)gka[m];
    });
    if (t == 0 && a.g_ain) {
      // d(pump)/dA_in = sqrt(kappa_ext): dL/dA_in = sqrt(kappa_ext) sum kbar at mu = 0
      a.g_ain[2 * id] += d.sqrt_kext * (double)gain.re;
      a.g_ain[2 * id + 1] += d.sqrt_kext * (double)gain.im;
    }
  }
}

template <typename Real, int N, int E, int PS>
hipError_t launch_fwd(const RunArgs &a, hipStream_t st) {
  using SH = KernelShape<Real, N, E, PS>;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((rk4_persistent<Real, N, E, PS>), dim3(grid), dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

template <typename Real, int N, int E, int PS>
hipError_t launch_adj(const AdjArgs &a, hipStream_t st) {
  using SH = KernelShape<Real, N, E, PS>;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((rk4_reverse<Real, N, E, PS>), dim3(grid), dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

#define CME_PS(E) (ilog2(E))
#define CME_V64(N, E)                                                                       \
  Variant{0, N, E, 1, CME_PS(E), 0, 0, KernelShape<double, N, E, CME_PS(E)>::IPB,              \
          KernelShape<double, N, E, CME_PS(E)>::THREADS,                                    \
          KernelShape<double, N, E, CME_PS(E)>::LDS_BYTES, &launch_fwd<double, N, E, CME_PS(E)>, \
          &launch_adj<double, N, E, CME_PS(E)>}

// FP32 team kernels (forward only: the reverse path is FP64).
#define CME_V32(N, E)                                                                      \
  Variant{1, N, E, 1, CME_PS(E), 0, 0, KernelShape<float, N, E, CME_PS(E)>::IPB,              \
          KernelShape<float, N, E, CME_PS(E)>::THREADS,                                    \
          KernelShape<float, N, E, CME_PS(E)>::LDS_BYTES, &launch_fwd<float, N, E, CME_PS(E)>, \
          nullptr}

// Team kernels cover the sizes where one instance is smaller than a
// wavefront's worth of threads (several instances share a wavefront).
static const Variant kVariants[] = {
    CME_V64(16, 4),  CME_V64(32, 4),  CME_V64(64, 4),  CME_V64(64, 8),
    CME_V64(128, 4), CME_V64(128, 8), CME_V64(256, 8), CME_V32(16, 4),
    CME_V32(32, 4),  CME_V32(64, 4),  CME_V32(128, 4), CME_V32(256, 8),
};

const Variant *variants_team(int *count) {
  *count = (int)(sizeof(kVariants) / sizeof(kVariants[0]));
  return kVariants;
}

}  // namespace cme
