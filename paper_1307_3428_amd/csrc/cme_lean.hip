// cme_lean.hip -- two-level RK4 kernels with a small register footprint, so
// that two wavefronts share each SIMD.
//
// The kernels of cme_wave.hip keep every per-thread twiddle of the two-level
// transform in registers and, with the RK4 state, need more than 256
// registers per lane at E = 8: one wavefront per SIMD, whose LDS waits and
// arithmetic cannot overlap.  Here
//   * each wave-local Stockham pass keeps only the powers b^(2^i) of its
//     twiddle base b = exp(-2 pi i k / (NS R)) and forms b^r, r < R, on use;
//   * the cross-wave twiddles exp(-2 pi i n1 k2 / N) are applied on the side
//     of the exchange where a thread holds one n1 and all k2 (on both paths),
//     from the powers of exp(-2 pi i n1 / N) for the thread's first n1 and
//     compile-time rotations exp(-2 pi i 64 q k2 / N) for the others;
//   * the RK4 state is y, the weighted derivative sum, and the stage input u
//     (the transform works on a copy), i.e. the previous derivative is not
//     kept: u of the next stage is formed as soon as a derivative is known.
// The arithmetic per stage is that of cme_wave.hip (Eq. (4) for the
// four-wave-mixing sum, Eq. (1) for the derivative); only the rounding of
// the rebuilt twiddles differs.
#include "cme_fft.hpp"
#include "cme_internal.hpp"

namespace cme {

namespace {
__device__ constexpr double kLeanC[4] = {0.0, 0.5, 0.5, 1.0};
__device__ constexpr double kLeanW[4] = {1.0, 2.0, 2.0, 1.0};
}  // namespace

constexpr int flog2(int x) {
  int r = 0;
  while ((2 << r) <= x) ++r;
  return r;
}

template <typename Real> __device__ __forceinline__ cx<Real> csqr(cx<Real> a) {
  const Real d = a.re + a.re;
  return {a.re * a.re - a.im * a.im, d * a.im};
}

// t[r] = b^r, r = 1..R-1, from b: powers of two by squaring, any other r as
// (r without its top bit) times (its top bit).
// The base passes through an empty asm statement first, so that the powers
// are formed where they are used instead of being hoisted out of the time
// loop into registers.
template <int R, typename Real>
__device__ __forceinline__ void pow_fill(cx<Real> (&t)[R], cx<Real> b) {
  asm volatile("" : "+v"(b.re), "+v"(b.im));
  sfor<1, R>([&](auto ri) {
    constexpr int r = decltype(ri)::value;
    constexpr int top = 1 << flog2(r);
    if constexpr (r == 1) t[r] = b;
    else if constexpr (top == r) t[r] = csqr(t[r / 2]);
    else t[r] = cmul(t[r - top], t[top]);
  });
}

// lpad<PS>(i0 + c) as lpad<PS>(i0) + (c + c / 2^PS) when the constant c
// cannot carry into the padded bits: c a multiple of 2^PS, or i0 a multiple
// of 2^PS and c < 2^PS.  Keeps one address register per access group, the
// rest become instruction offsets.
template <int PS, int C, bool ALIGNED>
__device__ __forceinline__ int lpad_off(int padded_i0) {
  static_assert(PS == 0 || C % (1 << PS) == 0 || (ALIGNED && C < (1 << PS)),
                "constant step may carry into the padding bits");
  if constexpr (PS == 0) return padded_i0 + C;
  else return padded_i0 + C + (C >> PS);
}

template <int N, int E> struct LeanPlan {
  using WP = WavePlan<N, E, 1, 0>;
  using Sub = FftPlan<WP::N1, E>;
  static constexpr int N1 = WP::N1, WV = WP::WV, Q = WP::Q, W = WP::W;
  static constexpr int LWV = WV > 1 ? ilog2(WV) : 0;
  // powers kept per pass p >= 1: log2 of its radix
  static constexpr int npow(int p) { return p == 0 ? 0 : 1; }
  static constexpr int powoff(int p) {
    int o = 0;
    for (int i = 0; i < p; ++i) o += npow(i);
    return o;
  }
  static constexpr int NSUB = powoff(Sub::P) > 0 ? powoff(Sub::P) : 1;
  static constexpr int NX = 1;
  static constexpr bool ok() {
    for (int p = 0; p < Sub::P; ++p)
      if (Sub::qd(p) != 1) return false;
    return true;
  }
  static_assert(ok(), "every sub-transform pass must have one twiddle base per thread");
  static_assert(WV == 1 || (N / 64 <= 64 && 64 % (N / 64) == 0),
                "cross-wave rotations are multiples of 2 pi / (N / 64), N / 64 dividing 64");
};

template <int N, int E, typename Real> struct LeanTw {
  cx<Real> sub[LeanPlan<N, E>::NSUB];
  cx<Real> x[LeanPlan<N, E>::NX];
};

// tab[i] = exp(-2 pi i i / N), i < N
template <int N, int E, typename Real>
__device__ __forceinline__ void load_lean_twiddles(LeanTw<N, E, Real> &tw,
                                                   const cx<Real> *__restrict__ tab, int w,
                                                   int l) {
  using LP = LeanPlan<N, E>;
  using PL = typename LP::Sub;
  constexpr int TS = LP::WV;  // the sub-transform table is every WV-th entry
  sfor<1, PL::P>([&](auto pi) {
    constexpr int p = decltype(pi)::value;
    constexpr int R = PL::radix(p), NSp = PL::ns(p);
    constexpr int STRIDE = LP::N1 / (NSp * R);
    const int k = l & (NSp - 1);
    sfor<0, LP::npow(p)>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      tw.sub[LP::powoff(p) + i] = tab[(k << i) * STRIDE * TS];
    });
  });
  if constexpr (LP::WV > 1) {
    const int n1 = l + 64 * w * LP::Q;
    tw.x[0] = tab[n1];
  }
}

// One wave-local transform of length N1 = 64 E in place in reg (one region
// of LdsLen<N1, PS> elements), sign S; as fft_wave_multi with V = 1 but with
// the twiddles rebuilt per pass.
template <int N, int E, int S, int PS, typename Real>
__device__ __forceinline__ void fft_wave_lean(cx<Real> (&v)[E], cx<Real> *reg,
                                              const LeanTw<N, E, Real> &tw, int l) {
  using LP = LeanPlan<N, E>;
  using PL = typename LP::Sub;
  constexpr int T = 64;
  sfor<0, PL::P>([&](auto pi) {
    constexpr int p = decltype(pi)::value;
    constexpr int R = PL::radix(p), NSp = PL::ns(p);
    constexpr int Qb = E / R;
    constexpr bool LAST = p == PL::P - 1;
    if constexpr (p > 0) {
      const int r0 = lpad<PS>(l);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        v[m] = reg[lpad_off<PS, m * T, false>(r0)];
      });
    }
    if constexpr (!LAST) wave_sync();  // in place: reads before writes
    cx<Real> t[R];
    if constexpr (NSp > 1) pow_fill<R>(t, tw.sub[LP::powoff(p)]);
    sfor<0, Qb>([&](auto qi) {
      constexpr int q = decltype(qi)::value;
      cx<Real> z[R];
      sfor<0, R>([&](auto ri) { z[decltype(ri)::value] = v[q + decltype(ri)::value * Qb]; });
      if constexpr (NSp > 1) {
        sfor<1, R>([&](auto ri) {
          constexpr int r = decltype(ri)::value;
          z[r] = ctw<S>(z[r], t[r]);
        });
      }
      dft_reg<R, S>(z);
      if constexpr (LAST) {
        sfor<0, R>([&](auto ri) { v[q + decltype(ri)::value * Qb] = z[decltype(ri)::value]; });
      } else {
        const int j = l + q * T;
        const int k = j & (NSp - 1);
        const int b0 = lpad<PS>((j - k) * R + k);
        // (j - k) R + k is a multiple of R when NS = 1
        sfor<0, R>([&](auto ri) {
          constexpr int r = decltype(ri)::value;
          reg[lpad_off<PS, r * NSp, NSp == 1 && R % (1 << PS) == 0>(b0)] = z[r];
        });
      }
    });
    if constexpr (!LAST) wave_sync();
  });
}

// z[r] *= exp(S 2 pi i n1 r / N) for r = 1..WV-1, n1 = l + 64 (w Q + i):
// t holds exp(-2 pi i n1_0 r / N); slot i adds the rotation 64 i r / N.
template <int N, int E, int S, int I, typename Real>
__device__ __forceinline__ void cross_twiddle(cx<Real> (&z)[(LeanPlan<N, E>::WV)],
                                              const cx<Real> (&t)[(LeanPlan<N, E>::WV)]) {
  constexpr int WV = LeanPlan<N, E>::WV;
  constexpr int L = N / 64;
  sfor<1, WV>([&](auto ri) {
    constexpr int r = decltype(ri)::value;
    z[r] = ctw<S>(z[r], t[r]);
    if constexpr (I > 0) z[r] = twc<S, (I * r) % L, L>(z[r]);
  });
}

// Forward path (mode order in, scrambled order out), sign S.
template <int N, int E, int S, int PS, bool PRE, typename Real>
__device__ __forceinline__ void lean_fwdpath(cx<Real> (&v)[E], cx<Real> *X,
                                             const LeanTw<N, E, Real> &tw, int w, int l) {
  using LP = LeanPlan<N, E>;
  constexpr int LB1 = LdsLen<LP::N1, PS>::value;
  constexpr int WV = LP::WV, Q = LP::Q;
  if constexpr (WV > 1) {
    if constexpr (PRE) cross_sync<LP::W>();
    cx<Real> t[WV];
    pow_fill<WV>(t, tw.x[0]);
    const int c0 = lpad<PS>(l + 64 * w * Q);
    sfor<0, Q>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      cx<Real> z[WV];
      sfor<0, WV>([&](auto ri) { z[decltype(ri)::value] = v[i + Q * decltype(ri)::value]; });
      dft_reg<WV, S>(z);
      cross_twiddle<N, E, S, i>(z, t);
      const int n1 = lpad_off<PS, 64 * i, false>(c0);
      sfor<0, WV>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        X[r * LB1 + n1] = z[r];
      });
    });
    cross_sync<LP::W>();
    const int r0 = w * LB1 + lpad<PS>(l);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      v[m] = X[lpad_off<PS, 64 * m, false>(r0)];
    });
  }
  fft_wave_lean<N, E, S, PS>(v, X + w * LB1, tw, l);
}

// Back path (scrambled order in, mode order out), sign S.  The wave-local
// transform runs in X (own region), the exchange goes through Y.
template <int N, int E, int S, int PS, typename Real>
__device__ __forceinline__ void lean_backpath(cx<Real> (&v)[E], cx<Real> *X, cx<Real> *Y,
                                              const LeanTw<N, E, Real> &tw, int w, int l) {
  using LP = LeanPlan<N, E>;
  constexpr int LB1 = LdsLen<LP::N1, PS>::value;
  constexpr int WV = LP::WV, Q = LP::Q;
  fft_wave_lean<N, E, S, PS>(v, X + w * LB1, tw, l);
  if constexpr (WV > 1) {
    if (Y == X) wave_sync();  // own region: the transform's last reads come first
    const int r0 = w * LB1 + lpad<PS>(l);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      Y[lpad_off<PS, 64 * m, false>(r0)] = v[m];
    });
    cross_sync<LP::W>();
    cx<Real> t[WV];
    pow_fill<WV>(t, tw.x[0]);
    const int c0 = lpad<PS>(l + 64 * w * Q);
    sfor<0, Q>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const int n1 = lpad_off<PS, 64 * i, false>(c0);
      cx<Real> z[WV];
      sfor<0, WV>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        z[r] = Y[r * LB1 + n1];
      });
      cross_twiddle<N, E, S, i>(z, t);
      dft_reg<WV, S>(z);
      sfor<0, WV>([&](auto ri) { v[i + Q * decltype(ri)::value] = z[decltype(ri)::value]; });
    });
  }
}

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

template <typename Real, int N, int E, int PS>
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
  cx<Real> *A = reinterpret_cast<cx<Real> *>(a.A) + d.offset;
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
    y[m] = A[i];
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
      if (stages != nullptr) {
        cx<Real> *st = stages + stage_offset(n, s, a.total) + d.offset;
        sfor<0, E>([&](auto mi) {
          constexpr int m = decltype(mi)::value;
          st[WP::mode(w, lane, m)] = u[m];
        });
      }
      sfor<0, E>([&](auto mi) { v[decltype(mi)::value] = u[decltype(mi)::value]; });
      lean_fwdpath<N, E, +1, PS, !SH::TWO>(v, X, tw, w, lane);
      if (stages != nullptr) {
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
  hipLaunchKernelGGL((rk4_lean<Real, N, E, PS>), dim3(grid), dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
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
};

const Variant *variants_lean(int *count) {
  *count = (int)(sizeof(kLeanVariants) / sizeof(kLeanVariants[0]));
  return kLeanVariants;
}

}  // namespace cme
