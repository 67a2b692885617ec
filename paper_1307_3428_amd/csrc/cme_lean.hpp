// cme_lean.hpp -- two-level transform with a small register footprint.
//
// As fft_fwdpath / fft_backpath of cme_fft.hpp (one wave-local sub-transform
// per wave, V = 1), but
//   * each wave-local Stockham pass keeps one twiddle base per thread,
//     b = exp(-2 pi i k / (NS R)), and forms b^r, r < R, on use;
//   * the cross-wave twiddles exp(-2 pi i n1 k2 / N) are applied on the side
//     of the exchange where a thread holds one n1 and all k2 (on both paths),
//     from the powers of exp(-2 pi i n1 / N) for the thread's first n1 and
//     compile-time rotations exp(-2 pi i 64 q k2 / N) for the others;
//   * LDS addresses are one register plus instruction offsets.
#pragma once

#include "cme_fft.hpp"

namespace cme {

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

}  // namespace cme
