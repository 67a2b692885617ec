// cme_fft.hpp -- workgroup-resident complex FFT for gfx950 (CDNA4).
//
// Used twice per Runge-Kutta stage to evaluate the four-wave-mixing sum as in
// Eq. (4) of Hansson, Modotto & Wabnitz (arXiv:1307.3428): an inverse
// transform of the mode amplitudes, the pointwise cube, and a forward
// transform.  The transforms are radix-E Stockham passes (E = elements per
// thread, a power of two) whose data live in registers inside a pass and are
// exchanged between passes through LDS.
//
// Ownership.  A team of T = N / E threads holds one length-N sequence; thread
// t owns elements t + m T, m = 0..E-1, in registers.  In every pass the
// thread's butterflies j = t + q T (q < E / R for radix R) read exactly those
// elements, and in the final pass the Stockham output index of those
// butterflies is again t + m T.  So a transform takes its input from and
// leaves its output in the same registers: only the E - 1 exchanges between
// passes touch LDS, and the RK4 state of mode t + m T can stay in the owning
// thread's registers for the whole run.
//
// Pass (Stockham, decimation in time, natural order in and out), with
// NS = product of the earlier radices and k = j mod NS:
//   z_r  = x[j + r N / R] * exp(s 2 pi i r k / (NS R)),   r = 0..R-1
//   Z    = DFT_R with sign s of z
//   y[(j - k) R + k + r NS] = Z_r.
// The radices are E, except one smaller pass (N / E^P) when N is not a power
// of E; it is placed second.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace cme {

// ---------------------------------------------------------------------------
// Complex values and compile-time loops
// ---------------------------------------------------------------------------
template <typename Real> struct alignas(2 * sizeof(Real)) cx {
  Real re, im;
};

template <typename Real>
__device__ __forceinline__ cx<Real> cadd(cx<Real> a, cx<Real> b) { return {a.re + b.re, a.im + b.im}; }
template <typename Real>
__device__ __forceinline__ cx<Real> csub(cx<Real> a, cx<Real> b) { return {a.re - b.re, a.im - b.im}; }
// a * w
template <typename Real>
__device__ __forceinline__ cx<Real> cmul(cx<Real> a, cx<Real> w) {
  return {a.re * w.re - a.im * w.im, a.re * w.im + a.im * w.re};
}
// a * conj(w)
template <typename Real>
__device__ __forceinline__ cx<Real> cmulc(cx<Real> a, cx<Real> w) {
  return {a.re * w.re + a.im * w.im, a.im * w.re - a.re * w.im};
}
// a * exp(s i theta) given w = exp(-i theta): s = -1 -> a w, s = +1 -> a conj(w)
template <int S, typename Real>
__device__ __forceinline__ cx<Real> ctw(cx<Real> a, cx<Real> w) {
  if constexpr (S < 0) return cmul(a, w);
  else return cmulc(a, w);
}

template <int I> using ic = std::integral_constant<int, I>;

// Synchronisation scope of an LDS exchange: the whole workgroup (s_barrier),
// or one wavefront.  LDS operations of one wavefront execute in program
// order, so a wave-local exchange needs no barrier instruction; the fences
// and the wave barrier only keep the compiler from reordering the accesses.
enum { SYNC_BLOCK = 0, SYNC_WAVE = 1 };

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int SYNC> __device__ __forceinline__ void team_sync() {
  if constexpr (SYNC == SYNC_BLOCK) __syncthreads();
  else wave_sync();
}

// f(ic<B>), f(ic<B+1>), ..., f(ic<E-1>) with compile-time indices
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f) {
  if constexpr (B < E) {
    f(ic<B>{});
    sfor<B + 1, E>(f);
  }
}

constexpr int ilog2(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

// cos and sin of 2 pi j / 64 for j = 0..16, correctly rounded to double.
struct Trig64 {
  static constexpr double c[17] = {
      1.0,                0.9951847266721969, 0.9807852804032304, 0.9569403357322088,
      0.9238795325112867, 0.881921264348355,  0.8314696123025452, 0.773010453362737,
      0.7071067811865476, 0.6343932841636455, 0.5555702330196022, 0.47139673682599764,
      0.3826834323650898, 0.2902846772544624, 0.19509032201612828, 0.0980171403295606,
      0.0};
  // cos(2 pi j / 64) for any j (reduced mod 64)
  static constexpr double cosj(int j) {
    j = ((j % 64) + 64) % 64;
    const int q = j / 16, r = j % 16;
    return q == 0 ? c[r] : q == 1 ? -c[16 - r] : q == 2 ? -c[r] : c[16 - r];
  }
  static constexpr double sinj(int j) {
    j = ((j % 64) + 64) % 64;
    const int q = j / 16, r = j % 16;
    return q == 0 ? c[16 - r] : q == 1 ? c[r] : q == 2 ? -c[16 - r] : -c[r];
  }
};

// a * exp(S 2 pi i K / L), K and L compile-time, L a power of two dividing 64.
// Multiplications by 0 or +-1 are never emitted: quarter turns are swaps and
// sign flips, eighth turns two adds and two multiplies.
template <int S, int K, int L, typename Real>
__device__ __forceinline__ cx<Real> twc(cx<Real> a) {
  static_assert(64 % L == 0, "twiddle denominator must divide 64");
  constexpr int k = ((K % L) + L) % L;
  constexpr int j = k * (64 / L);  // angle 2 pi j / 64
  if constexpr (j == 0) {
    return a;
  } else if constexpr (j == 32) {
    return {-a.re, -a.im};
  } else if constexpr (j == 16 || j == 48) {
    // exp(S i pi/2 * (1 or 3)) = +-i
    constexpr int sg = (j == 16 ? 1 : -1) * (S > 0 ? 1 : -1);
    if constexpr (sg > 0) return {-a.im, a.re};
    else return {a.im, -a.re};
  } else if constexpr (j % 8 == 0) {
    // odd multiple of pi/4: (cs + i ss) / sqrt(2)
    constexpr Real r = (Real)0.7071067811865476;
    constexpr int cs = Trig64::cosj(j) > 0 ? 1 : -1;
    constexpr int ss = (Trig64::sinj(j) > 0 ? 1 : -1) * (S > 0 ? 1 : -1);
    const Real xr = cs > 0 ? a.re : -a.re, xi = cs > 0 ? a.im : -a.im;
    const Real yr = ss > 0 ? a.im : -a.im, yi = ss > 0 ? a.re : -a.re;
    return {r * (xr - yr), r * (xi + yi)};
  } else {
    constexpr Real c = (Real)Trig64::cosj(j);
    constexpr Real s = (Real)(S > 0 ? Trig64::sinj(j) : -Trig64::sinj(j));
    return {a.re * c - a.im * s, a.re * s + a.im * c};
  }
}

constexpr int bitrev(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
  return r;
}

// In-register DFT of size R (power of two <= 64), sign S, natural order:
// Z_k = sum_r z_r exp(S 2 pi i r k / R).  Radix-2 decimation in time on the
// bit-reversed input (the permutation only renames registers).
template <int R, int S, typename Real>
__device__ __forceinline__ void dft_reg(cx<Real> (&z)[R]) {
  if constexpr (R == 1) {
    return;
  } else {
    constexpr int B = ilog2(R);
    cx<Real> w[R];
    sfor<0, R>([&](auto i) { w[bitrev(decltype(i)::value, B)] = z[decltype(i)::value]; });
    sfor<1, B + 1>([&](auto lv) {
      constexpr int len = 1 << decltype(lv)::value;
      constexpr int half = len / 2;
      sfor<0, R / len>([&](auto g) {
        constexpr int base = decltype(g)::value * len;
        sfor<0, half>([&](auto kk) {
          constexpr int k = decltype(kk)::value;
          const cx<Real> a = w[base + k];
          const cx<Real> b = twc<S, k, len>(w[base + k + half]);
          w[base + k] = cadd(a, b);
          w[base + k + half] = csub(a, b);
        });
      });
    });
    sfor<0, R>([&](auto i) { z[decltype(i)::value] = w[decltype(i)::value]; });
  }
}

// Fused multiply-add a * b + c in the type's own precision.
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// A twiddle w in the multiply-add form (c, t) with w = c (1 + i t).  Where
// Re w is zero (w = +-i) c is a tiny positive number and t = Im w / c, so
// that c t = Im w and c u stays the product to rounding for any operand far
// below the overflow threshold.
template <typename Real> __device__ __forceinline__ cx<Real> fma_form(cx<Real> w) {
  constexpr Real tiny = sizeof(Real) == 8 ? (Real)0x1p-500 : (Real)0x1p-60;
  const Real c = fabs(w.re) < tiny ? tiny : w.re;
  return {c, w.im / c};
}

// Radix-2 butterfly a, x -> a + w x, a - w x with w = c (1 + i t) given as
// ct = (c, t), or conj(w) for S > 0: u = x (1 + i t), then a +- c u, six
// fused multiply-adds in place of a complex multiply and four adds.
template <int S, typename Real>
__device__ __forceinline__ void fma_bfly(cx<Real> &a, cx<Real> &x, cx<Real> ct) {
  const Real t = S < 0 ? ct.im : -ct.im;
  const Real ur = fmar(-t, x.im, x.re), ui = fmar(t, x.re, x.im);
  x = {fmar(-ct.re, ur, a.re), fmar(-ct.re, ui, a.im)};
  a = {fmar(ct.re, ur, a.re), fmar(ct.re, ui, a.im)};
}

// Z_k = sum_r z_r (b^r exp(S 2 pi i r k / R)) for R a power of two, with b
// (conj(b) for S > 0) the pass's twiddle base: the radix-2
// decimation-in-time DFT of the twiddled inputs.  The butterflies of the
// level of length len combine two sub-sequences whose common factors differ
// by b^(R / len), so that factor joins the level's rotation:
// w = b^(R / len) exp(-2 pi i kk / len) for butterfly kk < len / 2, held at
// ct[len / 2 + kk] in the multiply-add form.
template <int R, int S, typename Real>
__device__ __forceinline__ void dft_reg_fma(cx<Real> (&z)[R], const cx<Real> *ct) {
  constexpr int B = ilog2(R);
  cx<Real> w[R];
  sfor<0, R>([&](auto i) { w[bitrev(decltype(i)::value, B)] = z[decltype(i)::value]; });
  sfor<1, B + 1>([&](auto lv) {
    constexpr int len = 1 << decltype(lv)::value;
    constexpr int half = len / 2;
    sfor<0, R / len>([&](auto g) {
      constexpr int base = decltype(g)::value * len;
      sfor<0, half>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        fma_bfly<S>(w[base + k], w[base + k + half], ct[half + k]);
      });
    });
  });
  sfor<0, R>([&](auto i) { z[decltype(i)::value] = w[decltype(i)::value]; });
}

// ---------------------------------------------------------------------------
// Pass plan for length N with E elements per thread
// ---------------------------------------------------------------------------
template <int N, int E> struct FftPlan {
  static_assert((N & (N - 1)) == 0 && (E & (E - 1)) == 0 && E >= 2 && E <= N, "bad plan");
  static constexpr int T = N / E;  // threads per sequence
  static constexpr int LN = ilog2(N), LE = ilog2(E);
  static constexpr int PFULL = LN / LE;
  static constexpr int REM = 1 << (LN - PFULL * LE);
  static constexpr int P = PFULL + (REM > 1 ? 1 : 0);
  static constexpr int REMPOS = REM > 1 ? 1 : -1;

  static constexpr int radix(int p) { return p == REMPOS ? REM : E; }
  static constexpr int ns(int p) {
    int s = 1;
    for (int i = 0; i < p; ++i) s *= radix(i);
    return s;
  }
  // number of distinct twiddle index sets per pass: k = (t + q T) mod NS
  // depends on q only while NS > T
  static constexpr int qd(int p) {
    const int q = E / radix(p);
    const int d = ns(p) > T ? ns(p) / T : 1;
    return q < d ? q : d;
  }
  static constexpr int ntw(int p) { return p == 0 ? 0 : qd(p) * (radix(p) - 1); }
  static constexpr int twoff(int p) {
    int o = 0;
    for (int i = 0; i < p; ++i) o += ntw(i);
    return o;
  }
  static constexpr int NTW = twoff(P) > 0 ? twoff(P) : 1;
};

// LDS index with one padding element every 2^PS elements (PS = 0: none)
template <int PS> __device__ __forceinline__ int lpad(int i) {
  if constexpr (PS == 0) return i;
  else return i + (i >> PS);
}
template <int N, int PS> struct LdsLen {
  static constexpr int value = PS == 0 ? N : N + (N >> PS);
};

// Load the per-thread twiddles of every pass from the table
// tab[i * TS] = exp(-2 pi i i / N), i < N (TS: stride of a longer table).
template <int N, int E, int TS = 1, typename Real>
__device__ __forceinline__ void load_twiddles(cx<Real> (&tw)[(FftPlan<N, E>::NTW)],
                                              const cx<Real> *__restrict__ tab, int t) {
  using PL = FftPlan<N, E>;
  sfor<1, PL::P>([&](auto pi) {
    constexpr int p = decltype(pi)::value;
    constexpr int R = PL::radix(p), NSp = PL::ns(p), QD = PL::qd(p), OFF = PL::twoff(p);
    constexpr int STRIDE = N / (NSp * R);
    sfor<0, QD>([&](auto qi) {
      constexpr int q = decltype(qi)::value;
      const int k = (t + q * PL::T) & (NSp - 1);
      sfor<1, R>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        tw[OFF + q * (R - 1) + (r - 1)] = tab[r * k * STRIDE * TS];
      });
    });
  });
}

// One transform of sign S (S = +1: a_j = sum_m x_m e^{+2 pi i j m / N};
// S = -1: e^{-...}; no scaling) of the sequence held as v[m] = x[t + m T].
// LDS: with PING (two buffers) each exchange alternates buffers starting at
// parity PAR0 and needs one synchronisation; with a single buffer each
// exchange is fenced on both sides.  SYNC selects workgroup or wave scope
// (a wave-scope team is exactly one wavefront).
template <int N, int E, int S, int PS, bool PING, int PAR0, int SYNC = SYNC_BLOCK,
          typename Real>
__device__ __forceinline__ void fft_team(cx<Real> (&v)[E], cx<Real> *buf0, cx<Real> *buf1,
                                         const cx<Real> (&tw)[(FftPlan<N, E>::NTW)], int t) {
  using PL = FftPlan<N, E>;
  constexpr int T = PL::T;
  sfor<0, PL::P>([&](auto pi) {
    constexpr int p = decltype(pi)::value;
    constexpr int R = PL::radix(p), NSp = PL::ns(p), QD = PL::qd(p), OFF = PL::twoff(p);
    constexpr int Q = E / R;
    constexpr bool LAST = p == PL::P - 1;
    if constexpr (p > 0) {
      cx<Real> *src = (PING && ((PAR0 + p - 1) & 1)) ? buf1 : buf0;
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        v[m] = src[lpad<PS>(t + m * T)];
      });
    }
    if constexpr (!LAST && !PING) {
      // single buffer: every thread must be done reading it (in the previous
      // pass, or in the last pass of the previous transform) before it is
      // overwritten
      team_sync<SYNC>();
    }
    cx<Real> *dst = (PING && ((PAR0 + p) & 1)) ? buf1 : buf0;
    sfor<0, Q>([&](auto qi) {
      constexpr int q = decltype(qi)::value;
      cx<Real> z[R];
      sfor<0, R>([&](auto ri) { z[decltype(ri)::value] = v[q + decltype(ri)::value * Q]; });
      if constexpr (NSp > 1) {
        constexpr int qq = q % QD;
        sfor<1, R>([&](auto ri) {
          constexpr int r = decltype(ri)::value;
          z[r] = ctw<S>(z[r], tw[OFF + qq * (R - 1) + (r - 1)]);
        });
      }
      dft_reg<R, S>(z);
      if constexpr (LAST) {
        sfor<0, R>([&](auto ri) { v[q + decltype(ri)::value * Q] = z[decltype(ri)::value]; });
      } else {
        const int j = t + q * T;
        const int k = j & (NSp - 1);
        const int base = (j - k) * R + k;
        sfor<0, R>([&](auto ri) {
          constexpr int r = decltype(ri)::value;
          dst[lpad<PS>(base + r * NSp)] = z[r];
        });
      }
    });
    if constexpr (!LAST) team_sync<SYNC>();
  });
}

template <int N, int E> constexpr int fft_exchanges() { return FftPlan<N, E>::P - 1; }

// ---------------------------------------------------------------------------
// Two-level transform for a workgroup of W wavefronts (T = 64 W threads),
// each wavefront running V independent wave-local sub-transforms.
//
// N = WV N1 with WV = W V "virtual waves" and N1 = 64 ES (ES = E / V modes
// per thread per sub-transform).  Index maps n = n1 + N1 n2 (input side) and
// k = k2 + WV k1 (output side):
//   X[k2 + WV k1] = sum_n1 e^{s 2pi i n1 k1 / N1} e^{s 2pi i n1 k2 / N}
//                   sum_n2 x[n1 + N1 n2] e^{s 2pi i n2 k2 / WV}.
// Forward path (input in mode order, output scrambled):
//   (a) WV-point DFTs over n2 in registers, (b) twiddles e^{s 2pi i n1 k2/N},
//   (c) one transpose across waves through LDS (the only workgroup barrier),
//   then the N1-point transform over n1 for k2 = w V + v, v < V, inside wave
//   w; its exchanges are wave-local, and the V sub-transforms of a wave are
//   independent, so the LDS traffic of one overlaps the arithmetic of another.
// Back path: the mirror image (wave-local N1-point transforms, twiddles,
// transpose across waves, WV-point DFTs in registers), taking the scrambled
// order to mode order.  The pointwise cube of Eq. (4) does not care about the
// order of the transformed field, so an inverse transform on the forward path
// followed by a forward transform on the back path returns the four-wave-
// mixing sum in the registers that held the mode amplitudes.
//
// Ownership: lane l of wave w holds, in slot m = i + Q n2 (Q = E / WV),
//   mode n = l + 64 (w Q + i) + N1 n2,
// and on the scrambled side, in slot m = v ES + j, the element
//   k = (w V + v) + WV (l + 64 j).
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Register transposes between the slots a thread holds and its lane bits.
//
// xpose<C>(a, b): for a pair of register slots (a: slot bit 0, b: slot bit 1)
// exchange that slot bit with lane bit C, i.e. afterwards lane l holds in
// slot bit s the value lane (l with bit C := s) held in slot bit (l's bit C).
// Lane bits 5 and 4 use v_permlane32_swap / v_permlane16_swap (one
// instruction per 32-bit word pair), bits 3 and 2 DPP row rotations with
// bank masks (two), bits 1 and 0 DPP quad permutes plus a select (four).
// No LDS is involved.
// ---------------------------------------------------------------------------
template <int C> __device__ __forceinline__ void xpose_u32(uint32_t &a, uint32_t &b, int lane) {
  if constexpr (C == 5) {
    auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  } else if constexpr (C == 4) {
    auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  } else if constexpr (C == 3) {
    // partner = lane ^ 8 = rotation by 8 inside a row of 16; banks 2,3 hold bit 3 set
    const uint32_t na = __builtin_amdgcn_update_dpp(a, b, 0x128, 0xF, 0xC, false);
    const uint32_t nb = __builtin_amdgcn_update_dpp(b, a, 0x128, 0xF, 0x3, false);
    a = na;
    b = nb;
  } else if constexpr (C == 2) {
    // lanes with bit 2 set (banks 1, 3) take from lane - 4 (row_ror:4), the
    // others from lane + 4 (row_ror:12)
    const uint32_t na = __builtin_amdgcn_update_dpp(a, b, 0x124, 0xF, 0xA, false);
    const uint32_t nb = __builtin_amdgcn_update_dpp(b, a, 0x12C, 0xF, 0x5, false);
    a = na;
    b = nb;
  } else {
    // quad_perm [2,3,0,1] (lane ^ 2) or [1,0,3,2] (lane ^ 1)
    constexpr int QP = C == 1 ? 0x4E : 0xB1;
    const uint32_t pb = __builtin_amdgcn_mov_dpp(b, QP, 0xF, 0xF, false);
    const uint32_t pa = __builtin_amdgcn_mov_dpp(a, QP, 0xF, 0xF, false);
    const bool hi = (lane >> C) & 1;
    const uint32_t na = hi ? pb : a, nb = hi ? b : pa;
    a = na;
    b = nb;
  }
}

template <int C, typename Real>
__device__ __forceinline__ void xpose(cx<Real> &a, cx<Real> &b, int lane) {
  constexpr int NW = (int)(sizeof(cx<Real>) / 4);
  uint32_t wa[NW], wb[NW];
  __builtin_memcpy(wa, &a, sizeof(a));
  __builtin_memcpy(wb, &b, sizeof(b));
  sfor<0, NW>([&](auto di) { xpose_u32<C>(wa[decltype(di)::value], wb[decltype(di)::value], lane); });
  __builtin_memcpy(&a, wa, sizeof(a));
  __builtin_memcpy(&b, wb, sizeof(b));
}

// Exchange the three slot bits of v[0..7] with lane bits C0+2, C0+1, C0:
// afterwards slot = old (lane >> C0) & 7 and (lane >> C0) & 7 = old slot.
template <int C0, typename Real>
__device__ __forceinline__ void xpose8(cx<Real> *v, int lane) {
  sfor<0, 4>([&](auto si) {
    constexpr int s = decltype(si)::value;
    xpose<C0 + 2>(v[s], v[s + 4], lane);
  });
  sfor<0, 4>([&](auto si) {
    constexpr int s = (decltype(si)::value & 1) + 4 * (decltype(si)::value >> 1);
    xpose<C0 + 1>(v[s], v[s + 2], lane);
  });
  sfor<0, 4>([&](auto si) {
    constexpr int s = 2 * decltype(si)::value;
    xpose<C0>(v[s], v[s + 1], lane);
  });
}

// Exchange slot bits with lane bits 0..2 through the wave's LDS region
// (padded one element in 8): lane l, slot s -> lane (l & 56) | s, slot l & 7.
template <typename Real>
__device__ __forceinline__ void xpose8_lo_lds(cx<Real> *v, cx<Real> *reg, int lane) {
  wave_sync();  // earlier reads of the region come first
  sfor<0, 8>([&](auto si) {
    constexpr int s = decltype(si)::value;
    reg[lpad<3>(8 * (lane & 56) + 8 * s + (lane & 7))] = v[s];
  });
  wave_sync();
  sfor<0, 8>([&](auto si) {
    constexpr int s = decltype(si)::value;
    v[s] = reg[lpad<3>(8 * lane + s)];
  });
}

// 512-point transforms on one wavefront (64 lanes x 8 slots), three radix-8
// passes over the slots with register/LDS transposes in between.  With digits
// n = n0 + 8 n1 + 64 n2 (n0 = lane & 7, n1 = lane >> 3, n2 = slot):
//   X[k0 + 8 k1 + 64 k2] = sum_n0 w512^{n0 k0} w64^{n0 k1} w8^{n0 k2}
//                          sum_n1 w64^{n1 k0} w8^{n1 k1} sum_n2 w8^{n2 k0} x[n]
// (w_M = e^{s 2pi i / M}).  Forward path: natural order in (lane l, slot s
// holds element l + 64 s), digit-permuted order out (lane l, slot s holds
// element (l >> 3) + 8 (l & 7) + 64 s).  Back path: the mirror image.
// Twiddles per lane (s = 1..7): A = w512^{l s}, B = w64^{(l & 7) s},
// C = w512^{(8 (l & 7) + (l >> 3)) s}, D = w64^{(l >> 3) s}, stored as
// e^{-2 pi i .} and conjugated by ctw for s = +1.
template <typename Real> struct Tw512 {
  cx<Real> a[7], b[7], c[7], d[7];
};

// tab[i * TS] = exp(-2 pi i i / 512)
template <int TS, typename Real>
__device__ __forceinline__ void load_tw512(Tw512<Real> &t, const cx<Real> *__restrict__ tab,
                                           int lane) {
  const int lo = lane & 7, hi = lane >> 3, sw = 8 * lo + hi;
  sfor<1, 8>([&](auto si) {
    constexpr int s = decltype(si)::value;
    t.a[s - 1] = tab[(lane * s) * TS];
    t.b[s - 1] = tab[(8 * lo * s) * TS];
    t.c[s - 1] = tab[(sw * s) * TS];
    t.d[s - 1] = tab[(8 * hi * s) * TS];
  });
}

template <int S, typename Real>
__device__ __forceinline__ void twiddle7(cx<Real> *v, const cx<Real> (&w)[7]) {
  sfor<1, 8>([&](auto si) {
    constexpr int s = decltype(si)::value;
    v[s] = ctw<S>(v[s], w[s - 1]);
  });
}

// LO_LDS: exchange lane bits 0..2 through LDS (one store + one load per
// element) instead of DPP (about four instructions per 32-bit word).
template <int S, bool LO_LDS, typename Real>
__device__ __forceinline__ void fft512_fwd(cx<Real> *v, cx<Real> *reg, const Tw512<Real> &t,
                                           int lane) {
  cx<Real>(&z)[8] = *reinterpret_cast<cx<Real>(*)[8]>(v);
  dft_reg<8, S>(z);
  twiddle7<S>(v, t.a);
  xpose8<3>(v, lane);
  dft_reg<8, S>(z);
  twiddle7<S>(v, t.b);
  if constexpr (LO_LDS) xpose8_lo_lds(v, reg, lane);
  else xpose8<0>(v, lane);
  dft_reg<8, S>(z);
}

template <int S, bool LO_LDS, typename Real>
__device__ __forceinline__ void fft512_back(cx<Real> *v, cx<Real> *reg, const Tw512<Real> &t,
                                            int lane) {
  cx<Real>(&z)[8] = *reinterpret_cast<cx<Real>(*)[8]>(v);
  dft_reg<8, S>(z);
  twiddle7<S>(v, t.c);
  if constexpr (LO_LDS) xpose8_lo_lds(v, reg, lane);
  else xpose8<0>(v, lane);
  dft_reg<8, S>(z);
  twiddle7<S>(v, t.d);
  xpose8<3>(v, lane);
  dft_reg<8, S>(z);
}

// Synchronisation of the cross-wave exchange: a workgroup barrier, or a wave
// fence when the whole instance lives in one wavefront (W = 1).
template <int W> __device__ __forceinline__ void cross_sync() {
  if constexpr (W == 1) wave_sync();
  else __syncthreads();
}

template <int N, int E, int V, int TP = 0> struct WavePlan {
  static constexpr int TPOL = TP;  // 0: Stockham sub-transforms; 1, 2: fft512 (1: low bits via LDS)
  static constexpr int T = N / E;
  static constexpr int W = T / 64;
  static constexpr int ES = E / V;
  static constexpr int N1 = 64 * ES;
  static constexpr int WV = W * V;
  static constexpr int Q = E / WV;
  using Sub = FftPlan<N1, ES>;
  static_assert(T % 64 == 0 && W >= 1 && E % V == 0 && E % WV == 0 && WV <= 64,
                "bad wave plan");
  static_assert(TP == 0 || ES == 8, "register-transpose sub-transforms need 8 modes per thread");
  static constexpr int NTX = WV > 1 ? Q * (WV - 1) : 1;  // cross twiddles, forward path
  static constexpr int NTY = WV > 1 ? E : 1;             // cross twiddles, back path
  __device__ static int mode(int w, int l, int m) {
    return l + 64 * (w * Q + m % Q) + N1 * (m / Q);
  }
  // storage position of the element a thread holds in slot m on the
  // transformed (scrambled) side: a bijection onto [0, N) with lanes
  // contiguous, used to save and reload time-domain fields
  __device__ static int tslot(int w, int l, int m) { return l + 64 * (w + W * m); }
};

template <int N, int E, int V, int TP, typename Real> struct WaveTwiddles {
  using WP = WavePlan<N, E, V, TP>;
  cx<Real> sub[TP == 0 ? WP::Sub::NTW : 1];
  Tw512<Real> t512;  // used when TP > 0 (the optimiser drops it otherwise)
  cx<Real> x[WP::NTX];
  cx<Real> y[WP::NTY];
};

// tab[i] = exp(-2 pi i i / N), i < N
template <int N, int E, int V, int TP, typename Real>
__device__ __forceinline__ void load_wave_twiddles(WaveTwiddles<N, E, V, TP, Real> &tw,
                                                   const cx<Real> *__restrict__ tab, int w,
                                                   int l) {
  using WP = WavePlan<N, E, V, TP>;
  if constexpr (TP == 0) load_twiddles<WP::N1, WP::ES, WP::WV>(tw.sub, tab, l);
  else load_tw512<N / 512>(tw.t512, tab, l);
  if constexpr (WP::WV > 1) {
    sfor<0, WP::Q>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const int n1 = l + 64 * (w * WP::Q + i);
      sfor<1, WP::WV>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        tw.x[i * (WP::WV - 1) + r - 1] = tab[n1 * r];
      });
    });
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      constexpr int v = m / WP::ES, j = m % WP::ES;
      tw.y[m] = tab[(l + 64 * j) * (w * V + v)];
    });
  }
}

// V independent wave-local transforms of length N1 = 64 ES, in place in the
// regions reg + v * LB1.  Each pass first issues the reads of all V
// sequences, then computes and writes them one after the other, so the reads
// of sequence v+1 and the writes of sequence v overlap the arithmetic.
template <int N1, int ES, int V, int S, int PS, typename Real>
__device__ __forceinline__ void fft_wave_multi(cx<Real> (&v)[V * ES], cx<Real> *reg,
                                               const cx<Real> (&tw)[(FftPlan<N1, ES>::NTW)],
                                               int l) {
  using PL = FftPlan<N1, ES>;
  constexpr int T = 64;
  constexpr int LB1 = LdsLen<N1, PS>::value;
  sfor<0, PL::P>([&](auto pi) {
    constexpr int p = decltype(pi)::value;
    constexpr int R = PL::radix(p), NSp = PL::ns(p), QD = PL::qd(p), OFF = PL::twoff(p);
    constexpr int Qb = ES / R;
    constexpr bool LAST = p == PL::P - 1;
    if constexpr (p > 0) {
      sfor<0, V>([&](auto vi) {
        constexpr int vv = decltype(vi)::value;
        sfor<0, ES>([&](auto mi) {
          constexpr int m = decltype(mi)::value;
          v[vv * ES + m] = reg[vv * LB1 + lpad<PS>(l + m * T)];
        });
      });
    }
    if constexpr (!LAST) wave_sync();  // in place: reads before writes
    sfor<0, V>([&](auto vi) {
      constexpr int vv = decltype(vi)::value;
      sfor<0, Qb>([&](auto qi) {
        constexpr int q = decltype(qi)::value;
        cx<Real> z[R];
        sfor<0, R>([&](auto ri) {
          z[decltype(ri)::value] = v[vv * ES + q + decltype(ri)::value * Qb];
        });
        if constexpr (NSp > 1) {
          constexpr int qq = q % QD;
          sfor<1, R>([&](auto ri) {
            constexpr int r = decltype(ri)::value;
            z[r] = ctw<S>(z[r], tw[OFF + qq * (R - 1) + (r - 1)]);
          });
        }
        dft_reg<R, S>(z);
        if constexpr (LAST) {
          sfor<0, R>([&](auto ri) {
            v[vv * ES + q + decltype(ri)::value * Qb] = z[decltype(ri)::value];
          });
        } else {
          const int j = l + q * T;
          const int k = j & (NSp - 1);
          const int base = (j - k) * R + k;
          sfor<0, R>([&](auto ri) {
            constexpr int r = decltype(ri)::value;
            reg[vv * LB1 + lpad<PS>(base + r * NSp)] = z[r];
          });
        }
      });
    });
    if constexpr (!LAST) wave_sync();
  });
}

// ---------------------------------------------------------------------------
// The two-level transforms split at their workgroup barrier, so that two
// independent transforms can share one barrier and interleave their work:
//   forward path = fwd_phase1, barrier, fwd_phase2;
//   back path    = back_phase1, barrier, back_phase2.
// Each transform uses one context X of WV regions (LB1 elements each): the
// forward path writes all regions before the barrier and then works in its
// own regions; the back path works and writes in its own regions before the
// barrier and reads all regions after it.  A caller that reuses a context
// must put another barrier between the last reads of one use and the first
// writes of the next.
// ---------------------------------------------------------------------------
template <int N, int E, int V, int TP, int S, int PS, typename Real>
__device__ __forceinline__ void fwd_phase1(cx<Real> (&v)[E], cx<Real> *X,
                                           const WaveTwiddles<N, E, V, TP, Real> &tw, int w,
                                           int l) {
  using WP = WavePlan<N, E, V, TP>;
  constexpr int LB1 = LdsLen<WP::N1, PS>::value;
  constexpr int WV = WP::WV, Q = WP::Q;
  if constexpr (WV > 1) {
    sfor<0, Q>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      cx<Real> z[WV];
      sfor<0, WV>([&](auto ri) { z[decltype(ri)::value] = v[i + Q * decltype(ri)::value]; });
      dft_reg<WV, S>(z);
      const int n1 = l + 64 * (w * Q + i);
      sfor<1, WV>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        z[r] = ctw<S>(z[r], tw.x[i * (WV - 1) + r - 1]);
      });
      sfor<0, WV>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        X[r * LB1 + lpad<PS>(n1)] = z[r];
      });
    });
  }
}

template <int N, int E, int V, int TP, int S, int PS, typename Real>
__device__ __forceinline__ void fwd_phase2(cx<Real> (&v)[E], cx<Real> *X,
                                           const WaveTwiddles<N, E, V, TP, Real> &tw, int w,
                                           int l) {
  using WP = WavePlan<N, E, V, TP>;
  constexpr int LB1 = LdsLen<WP::N1, PS>::value;
  constexpr int WV = WP::WV, ES = WP::ES;
  if constexpr (WV > 1) {
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      constexpr int vv = m / ES, j = m % ES;
      v[m] = X[(w * V + vv) * LB1 + lpad<PS>(l + 64 * j)];
    });
  }
  if constexpr (TP == 0) {
    fft_wave_multi<WP::N1, ES, V, S, PS>(v, X + w * V * LB1, tw.sub, l);
  } else {
    sfor<0, V>([&](auto vi) {
      constexpr int vv = decltype(vi)::value;
      fft512_fwd<S, TP == 1>(v + vv * 8, X + (w * V + vv) * LB1, tw.t512, l);
    });
  }
}

template <int N, int E, int V, int TP, int S, int PS, typename Real>
__device__ __forceinline__ void back_phase1(cx<Real> (&v)[E], cx<Real> *X,
                                            const WaveTwiddles<N, E, V, TP, Real> &tw, int w,
                                            int l) {
  using WP = WavePlan<N, E, V, TP>;
  constexpr int LB1 = LdsLen<WP::N1, PS>::value;
  constexpr int WV = WP::WV, ES = WP::ES;
  if constexpr (TP == 0) {
    fft_wave_multi<WP::N1, ES, V, S, PS>(v, X + w * V * LB1, tw.sub, l);
  } else {
    sfor<0, V>([&](auto vi) {
      constexpr int vv = decltype(vi)::value;
      fft512_back<S, TP == 1>(v + vv * 8, X + (w * V + vv) * LB1, tw.t512, l);
    });
  }
  if constexpr (WV > 1) {
    wave_sync();  // the transform's last reads of the region come first
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      constexpr int vv = m / ES, j = m % ES;
      X[(w * V + vv) * LB1 + lpad<PS>(l + 64 * j)] = ctw<S>(v[m], tw.y[m]);
    });
  }
}

template <int N, int E, int V, int TP, int S, int PS, typename Real>
__device__ __forceinline__ void back_phase2(cx<Real> (&v)[E], cx<Real> *X,
                                            const WaveTwiddles<N, E, V, TP, Real> &tw, int w,
                                            int l) {
  using WP = WavePlan<N, E, V, TP>;
  constexpr int LB1 = LdsLen<WP::N1, PS>::value;
  constexpr int WV = WP::WV, Q = WP::Q;
  if constexpr (WV > 1) {
    sfor<0, Q>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const int n1 = l + 64 * (w * Q + i);
      cx<Real> z[WV];
      sfor<0, WV>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        z[r] = X[r * LB1 + lpad<PS>(n1)];
      });
      dft_reg<WV, S>(z);
      sfor<0, WV>([&](auto ri) { v[i + Q * decltype(ri)::value] = z[decltype(ri)::value]; });
    });
  }
}

// Forward path of sign S.  X: WV regions of LB1 = padded N1 elements.
// PRE: issue a workgroup barrier before the cross-wave writes (needed when
// another wave may still be reading X).
template <int N, int E, int V, int TP, int S, int PS, bool PRE, typename Real>
__device__ __forceinline__ void fft_fwdpath(cx<Real> (&v)[E], cx<Real> *X,
                                            const WaveTwiddles<N, E, V, TP, Real> &tw, int w,
                                            int l) {
  using WP = WavePlan<N, E, V, TP>;
  constexpr int LB1 = LdsLen<WP::N1, PS>::value;
  constexpr int WV = WP::WV, Q = WP::Q, ES = WP::ES;
  if constexpr (WV > 1) {
    if constexpr (PRE) cross_sync<WP::W>();
    sfor<0, Q>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      cx<Real> z[WV];
      sfor<0, WV>([&](auto ri) { z[decltype(ri)::value] = v[i + Q * decltype(ri)::value]; });
      dft_reg<WV, S>(z);
      const int n1 = l + 64 * (w * Q + i);
      sfor<1, WV>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        z[r] = ctw<S>(z[r], tw.x[i * (WV - 1) + r - 1]);
      });
      sfor<0, WV>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        X[r * LB1 + lpad<PS>(n1)] = z[r];
      });
    });
    cross_sync<WP::W>();
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      constexpr int vv = m / ES, j = m % ES;
      v[m] = X[(w * V + vv) * LB1 + lpad<PS>(l + 64 * j)];
    });
  }
  if constexpr (TP == 0) {
    fft_wave_multi<WP::N1, ES, V, S, PS>(v, X + w * V * LB1, tw.sub, l);
  } else {
    sfor<0, V>([&](auto vi) {
      constexpr int vv = decltype(vi)::value;
      fft512_fwd<S, TP == 1>(v + vv * 8, X + (w * V + vv) * LB1, tw.t512, l);
    });
  }
}

// Back path of sign S.  The wave-local transforms run in X (own regions); the
// cross-wave exchange goes through Y (may equal X only if the caller fences
// the next forward path with PRE).
template <int N, int E, int V, int TP, int S, int PS, typename Real>
__device__ __forceinline__ void fft_backpath(cx<Real> (&v)[E], cx<Real> *X, cx<Real> *Y,
                                             const WaveTwiddles<N, E, V, TP, Real> &tw, int w,
                                             int l) {
  using WP = WavePlan<N, E, V, TP>;
  constexpr int LB1 = LdsLen<WP::N1, PS>::value;
  constexpr int WV = WP::WV, Q = WP::Q, ES = WP::ES;
  if constexpr (TP == 0) {
    fft_wave_multi<WP::N1, ES, V, S, PS>(v, X + w * V * LB1, tw.sub, l);
  } else {
    sfor<0, V>([&](auto vi) {
      constexpr int vv = decltype(vi)::value;
      fft512_back<S, TP == 1>(v + vv * 8, X + (w * V + vv) * LB1, tw.t512, l);
    });
  }
  if constexpr (WV > 1) {
    if (Y == X) wave_sync();  // own regions: the transform's last reads come first
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      constexpr int vv = m / ES, j = m % ES;
      Y[(w * V + vv) * LB1 + lpad<PS>(l + 64 * j)] = ctw<S>(v[m], tw.y[m]);
    });
    cross_sync<WP::W>();
    sfor<0, Q>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const int n1 = l + 64 * (w * Q + i);
      cx<Real> z[WV];
      sfor<0, WV>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        z[r] = Y[r * LB1 + lpad<PS>(n1)];
      });
      dft_reg<WV, S>(z);
      sfor<0, WV>([&](auto ri) { v[i + Q * decltype(ri)::value] = z[decltype(ri)::value]; });
    });
  }
}

}  // namespace cme
