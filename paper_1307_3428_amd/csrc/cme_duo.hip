// cme_duo.hip -- RK4 kernel evaluating each step as four rounds of two
// independent transforms, interleaved inside every wavefront.
//
// Same RK4 map as cme_wave.hpp, in a different but mathematically identical
// order.  With L_s = -kappa/2 + i(omega' - sigma(t_s)), p the pump at mu = 0,
// W_s = L_s u_s + p, IDFT the unnormalised inverse transform of Eq. (4) and
// K'_s = DFT(b_s) (so the four-wave-mixing term is (g0/N) K'_s):
//   k_s        = W_s + i (g0/N) K'_s,           b_s = |a_s|^2 a_s,
//   a_s        = IDFT(u_s),  IDFT(k_s) = IDFT(W_s) + i g0 b_s  (IDFT DFT = N),
//   a_{s+1}    = IDFT(y + c_{s+1} h W_s) + c_{s+1} h i g0 b_s.
// Hence:
//   R0: a_1 = IDFT(y), V_1 = IDFT(y + h/2 W_1)      (W_1 = L_1 y + p)
//       a_2 = V_1 + h/2 i g0 b_1
//   R1: K'_1, K'_2             (forward transforms of b_1 and b_2)
//       k_1, u_2, W_2, k_2, u_3, W_3
//   R2: a_3 = IDFT(u_3), V_3 = IDFT(y + h W_3)
//       a_4 = V_3 + h i g0 b_3
//   R3: K'_3, K'_4             (forward transforms of b_3 and b_4)
//       k_3, u_4, W_4, k_4;  y += h/6 (k_1 + 2 k_2 + 2 k_3 + k_4).
// Only two arrays live across rounds R2 and R3: y + h W_3 and
// y + h/6 (k_1 + 2 k_2 + 2 W_3), which stand for y, the accumulator and W_3.
// Eight transforms in four rounds; the two of a round have the same
// direction and structure, so their passes are interleaved: while one
// transform's LDS exchange is in flight the wave computes the other's
// butterflies.  One workgroup barrier per round (two buffer sets, used by
// alternate rounds).  The transform is that of cme_lean.hpp.
#include <type_traits>

#include "cme_internal.hpp"
#include "cme_lean.hpp"

namespace cme {

// Butterflies of pass p of the wave-local transform of sign S on v (twiddles
// t[r] = b^r of the pass), results back in v: v[q + r Qb] = Z_r of butterfly q.
// FMA: t holds the level twiddles of dft_reg_fma in place of the powers.
template <int N, int E, int S, int p, bool FMA = false, typename Real>
__device__ __forceinline__ void lean_compute(cx<Real> (&v)[E], const cx<Real> *t) {
  using PL = typename LeanPlan<N, E>::Sub;
  constexpr int R = PL::radix(p), NSp = PL::ns(p), Qb = E / R;
  sfor<0, Qb>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    cx<Real> z[R];
    sfor<0, R>([&](auto ri) { z[decltype(ri)::value] = v[q + decltype(ri)::value * Qb]; });
    if constexpr (FMA && NSp > 1) {
      dft_reg_fma<R, S>(z, t);
    } else {
      if constexpr (NSp > 1) {
        sfor<1, R>([&](auto ri) {
          constexpr int r = decltype(ri)::value;
          z[r] = ctw<S>(z[r], t[r]);
        });
      }
      dft_reg<R, S>(z);
    }
    sfor<0, R>([&](auto ri) { v[q + decltype(ri)::value * Qb] = z[decltype(ri)::value]; });
  });
}

// Stockham scatter of pass p (not the last) to the wave's region reg.
template <int N, int E, int PS, int p, typename Real>
__device__ __forceinline__ void lean_scatter(const cx<Real> (&v)[E], cx<Real> *reg, int l) {
  using PL = typename LeanPlan<N, E>::Sub;
  constexpr int R = PL::radix(p), NSp = PL::ns(p), Qb = E / R;
  constexpr int T = 64;
  sfor<0, Qb>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    const int j = l + q * T;
    const int k = j & (NSp - 1);
    const int b0 = lpad<PS>((j - k) * R + k);
    sfor<0, R>([&](auto ri) {
      constexpr int r = decltype(ri)::value;
      reg[lpad_off<PS, r * NSp, NSp == 1 && R % (1 << PS) == 0>(b0)] = v[q + r * Qb];
    });
  });
}

template <int PS, int E, typename Real>
__device__ __forceinline__ void lean_gather(cx<Real> (&v)[E], const cx<Real> *reg, int l) {
  const int r0 = lpad<PS>(l);
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    v[m] = reg[lpad_off<PS, m * 64, false>(r0)];
  });
}

// Scheduling: the instructions emitted since the last full scheduling
// barrier are ordered as NDS times (one LDS instruction, then NV VALU
// instructions), so that one sequence's exchange drains from the LDS queue
// while the other's butterflies execute (a wave issues in order: LDS
// instructions bunched together stall it on the full queue).
template <int NDS, int NV> __device__ __forceinline__ void interleave_ds_valu() {
  sfor<0, NDS>([&](auto) {
    __builtin_amdgcn_sched_group_barrier(0x080, 1, 0);  // DS read or write
    __builtin_amdgcn_sched_group_barrier(0x002, NV, 0);  // VALU
  });
  __builtin_amdgcn_sched_barrier(0);
}

// Orders a wave's LDS scatter before its gather for the compiler (the
// hardware executes one wavefront's LDS instructions in order).  Unlike
// wave_sync it has no wave barrier, which would end the scheduling region
// and keep the gather from interleaving with the other sequence's VALU work.
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Twiddles of the paired transforms, from one of two sources: LeanTw (one
// base per pass, powers formed on use) or FullTw (every power held in
// registers: the paired kernels run one wavefront per SIMD, so they have the
// register file to spare and save the arithmetic).
template <int N, int E, typename Real> struct FullTw {
  using LP = LeanPlan<N, E>;
  using PL = typename LP::Sub;
  cx<Real> sub[PL::P][E];                  // pass p >= 1: b_p^r, r < radix(p)
  cx<Real> x[(LP::WV > 1 ? LP::WV : 1)];  // b_x^r, r < WV
};

// tab[i] = exp(-2 pi i i / N), i < N
template <int N, int E, typename Real>
__device__ __forceinline__ void load_full_twiddles(FullTw<N, E, Real> &tw,
                                                   const cx<Real> *__restrict__ tab, int w,
                                                   int l) {
  using LP = LeanPlan<N, E>;
  using PL = typename LP::Sub;
  constexpr int TS = LP::WV;
  sfor<1, PL::P>([&](auto pi) {
    constexpr int p = decltype(pi)::value;
    constexpr int R = PL::radix(p), NSp = PL::ns(p);
    constexpr int STRIDE = LP::N1 / (NSp * R);
    const int k = l & (NSp - 1);
    sfor<1, R>([&](auto ri) {
      constexpr int r = decltype(ri)::value;
      tw.sub[p][r] = tab[r * k * STRIDE * TS];
    });
  });
  if constexpr (LP::WV > 1) {
    const int n1 = l + 64 * w * LP::Q;
    sfor<1, LP::WV>([&](auto ri) {
      constexpr int r = decltype(ri)::value;
      tw.x[r] = tab[r * n1];
    });
  }
}

// FT = 2, the multiply-add form: the level twiddles of dft_reg_fma for each
// pass p >= 1 (entry half + kk for the level of length 2 half: w =
// b_p^(R / len) exp(-2 pi i kk / len)), and the cross-wave twiddles of each
// group i of the thread's elements with the group's rotation folded in
// (b_x^r exp(-2 pi i r i / (N / 64)) = tab[r (n1 + 64 i)]), so that each is
// one complex multiply.
// XG = false: one set of cross-wave powers for all groups (the rotation of
// each group applied on use), for kernels without the registers to spare.
template <int N, int E, typename Real, bool XG = true> struct FmaTw {
  using LP = LeanPlan<N, E>;
  using PL = typename LP::Sub;
  cx<Real> sub[PL::P][E];
  cx<Real> x[XG ? LP::Q : 1][(LP::WV > 1 ? LP::WV : 1)];
};

template <int N, int E, bool XG, typename Real>
__device__ __forceinline__ void load_fma_twiddles(FmaTw<N, E, Real, XG> &tw,
                                                  const cx<Real> *__restrict__ tab, int w,
                                                  int l) {
  using LP = LeanPlan<N, E>;
  using PL = typename LP::Sub;
  constexpr int TS = LP::WV;
  sfor<1, PL::P>([&](auto pi) {
    constexpr int p = decltype(pi)::value;
    constexpr int R = PL::radix(p), NSp = PL::ns(p);
    constexpr int STRIDE = LP::N1 / (NSp * R);
    const int k = l & (NSp - 1);
    sfor<1, ilog2(R) + 1>([&](auto lv) {
      constexpr int len = 1 << decltype(lv)::value, half = len / 2;
      sfor<0, half>([&](auto kki) {
        constexpr int kk = decltype(kki)::value;
        tw.sub[p][half + kk] =
            fma_form(tab[((R / len) * k * STRIDE * TS + kk * (N / len)) & (N - 1)]);
      });
    });
  });
  if constexpr (LP::WV > 1) {
    const int n1 = l + 64 * w * LP::Q;
    sfor<0, (XG ? LP::Q : 1)>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      sfor<1, LP::WV>([&](auto ri) {
        constexpr int r = decltype(ri)::value;
        tw.x[i][r] = tab[(r * (n1 + 64 * i)) & (N - 1)];
      });
    });
  }
}

// IsFmaTw: the multiply-add pass twiddles; CombTw: cross-wave twiddles per group
template <typename TW> struct IsFmaTw : std::false_type {};
template <int N, int E, typename Real, bool XG>
struct IsFmaTw<FmaTw<N, E, Real, XG>> : std::true_type {};
template <typename TW> struct CombTw : std::false_type {};
template <int N, int E, typename Real> struct CombTw<FmaTw<N, E, Real, true>> : std::true_type {};

template <int N, int E, bool XG, typename Real>
__device__ __forceinline__ void load_twiddle_source(FmaTw<N, E, Real, XG> &tw, const cx<Real> *tab,
                                                    int w, int l) {
  load_fma_twiddles<N, E>(tw, tab, w, l);
}
template <int N, int E, typename Real>
__device__ __forceinline__ void load_twiddle_source(LeanTw<N, E, Real> &tw, const cx<Real> *tab,
                                                    int w, int l) {
  load_lean_twiddles<N, E>(tw, tab, w, l);
}
template <int N, int E, typename Real>
__device__ __forceinline__ void load_twiddle_source(FullTw<N, E, Real> &tw, const cx<Real> *tab,
                                                    int w, int l) {
  load_full_twiddles<N, E>(tw, tab, w, l);
}

// t[r] = twiddle power r of pass p (p >= 1)
template <int p, int R, int N, int E, typename Real>
__device__ __forceinline__ void pass_twiddles(cx<Real> (&t)[R], const LeanTw<N, E, Real> &tw) {
  pow_fill<R>(t, tw.sub[LeanPlan<N, E>::powoff(p)]);
}
template <int p, int R, int N, int E, typename Real>
__device__ __forceinline__ void pass_twiddles(cx<Real> (&t)[R], const FullTw<N, E, Real> &tw) {
  sfor<1, R>([&](auto ri) { t[decltype(ri)::value] = tw.sub[p][decltype(ri)::value]; });
}
template <int p, int R, int N, int E, bool XG, typename Real>
__device__ __forceinline__ void pass_twiddles(cx<Real> (&t)[R], const FmaTw<N, E, Real, XG> &tw) {
  sfor<1, R>([&](auto ri) { t[decltype(ri)::value] = tw.sub[p][decltype(ri)::value]; });
}
// t[i][r] = cross-wave twiddle power r for group i: the same base powers for
// every group (the group's rotation is applied on use), or with FmaTw the
// group's own twiddles
template <int Q, int WV, int N, int E, typename Real>
__device__ __forceinline__ void cross_twiddles(cx<Real> (&t)[Q][WV], const LeanTw<N, E, Real> &tw) {
  pow_fill<WV>(t[0], tw.x[0]);
  sfor<1, Q>([&](auto ii) { sfor<1, WV>([&](auto ri) {
    t[decltype(ii)::value][decltype(ri)::value] = t[0][decltype(ri)::value]; }); });
}
template <int Q, int WV, int N, int E, typename Real>
__device__ __forceinline__ void cross_twiddles(cx<Real> (&t)[Q][WV], const FullTw<N, E, Real> &tw) {
  sfor<0, Q>([&](auto ii) { sfor<1, WV>([&](auto ri) {
    t[decltype(ii)::value][decltype(ri)::value] = tw.x[decltype(ri)::value]; }); });
}
template <int Q, int WV, int N, int E, bool XG, typename Real>
__device__ __forceinline__ void cross_twiddles(cx<Real> (&t)[Q][WV],
                                               const FmaTw<N, E, Real, XG> &tw) {
  sfor<0, Q>([&](auto ii) { sfor<1, WV>([&](auto ri) {
    t[decltype(ii)::value][decltype(ri)::value] =
        tw.x[XG ? decltype(ii)::value : 0][decltype(ri)::value];
  }); });
}

// v_permlane32_swap: the upper 32 lanes of a trade places with the lower 32
// lanes of b; v_permlane16_swap: the odd rows (16 lanes) of a with the even
// rows of b
__device__ __forceinline__ void lane_swap32(double &a, double &b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32));
  b = __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
}
__device__ __forceinline__ void lane_swap16(double &a, double &b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32));
  b = __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
}
__device__ __forceinline__ void lane_swap32(float &a, float &b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a),
                                                  __builtin_bit_cast(unsigned, b), false, false);
  a = __builtin_bit_cast(float, (unsigned)r[0]);
  b = __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ void lane_swap16(float &a, float &b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a),
                                                  __builtin_bit_cast(unsigned, b), false, false);
  a = __builtin_bit_cast(float, (unsigned)r[0]);
  b = __builtin_bit_cast(float, (unsigned)r[1]);
}

// The last exchange of a 256-point sub-transform at four modes per thread
// (radix-4 passes, 64 lanes): after the third pass element r of lane t
// belongs at position 64 (t >> 4) + 16 r + (t & 15), and the last pass needs
// position t' + 64 m in slot m, so register bits 0-1 trade places with lane
// bits 4-5 and nothing else moves: two swap stages, no renaming.
// sizes whose last sub-transform exchange lane_exchange4 does
template <int N, int E> constexpr bool lx_ok() {
  using PL = typename LeanPlan<N, E>::Sub;
  return E == 4 && PL::P >= 2 && PL::radix(PL::P - 2) == 4 && PL::ns(PL::P - 2) == 16;
}
template <int E, typename Real> __device__ __forceinline__ void lane_exchange4(cx<Real> (&v)[E]) {
  static_assert(E == 4, "four modes per thread");
  sfor<0, 2>([&](auto ri) {
    constexpr int r = decltype(ri)::value;  // 0 1
    lane_swap32(v[r].re, v[r + 2].re);
    lane_swap32(v[r].im, v[r + 2].im);
  });
  sfor<0, 2>([&](auto ri) {
    constexpr int r = 2 * decltype(ri)::value;  // 0 2
    lane_swap16(v[r].re, v[r + 1].re);
    lane_swap16(v[r].im, v[r + 1].im);
  });
}

// The passes of two independent wave-local transforms of sign S, a in region
// ra and b in region rb, software-pipelined.  On entry a has had its first
// pass's butterflies (lean_compute<0>) and b holds its input; on exit a is
// transformed and b still needs its last pass's butterflies.  In between, a's
// scatter and next gather interleave with b's butterflies of the same pass,
// and b's with a's butterflies of the next pass.
// LX: the last exchange in registers (lane_exchange4; 256-point
// sub-transforms at four modes per thread, see lx_ok)
template <int N, int E, int S, int PS, int NV, bool LX = false, typename Real, typename TW>
__device__ __forceinline__ void pair_passes(cx<Real> (&va)[E], cx<Real> (&vb)[E], cx<Real> *ra,
                                            cx<Real> *rb, const TW &tw, int l) {
  using LP = LeanPlan<N, E>;
  using PL = typename LP::Sub;
  constexpr bool FMA = IsFmaTw<TW>::value;
  sfor<0, PL::P - 1>([&](auto pi) {
    constexpr int p = decltype(pi)::value;
    constexpr int R = PL::radix(p), R1 = PL::radix(p + 1);
    cx<Real> t[R], t1[R1];
    if constexpr (PL::ns(p) > 1) pass_twiddles<p>(t, tw);
    if constexpr (LX && p == PL::P - 2) {
      static_assert(E == 4 && R == 4 && PL::ns(p) == 16, "lane exchange: 256-point, radix 4");
      lane_exchange4(va);
      lean_compute<N, E, S, p, FMA>(vb, t);
      pass_twiddles<p + 1>(t1, tw);
      lane_exchange4(vb);
      lean_compute<N, E, S, p + 1, FMA>(va, t1);
    } else {
      lean_scatter<N, E, PS, p>(va, ra, l);
      wave_fence();  // scatter before gather (other lanes' values)
      lean_gather<PS>(va, ra, l);
      lean_compute<N, E, S, p, FMA>(vb, t);
      // a pass without twiddles has about half the VALU work
      interleave_ds_valu<2 * E, (PL::ns(p) > 1 ? NV : NV / 2)>();
      pass_twiddles<p + 1>(t1, tw);
      lean_scatter<N, E, PS, p>(vb, rb, l);
      wave_fence();
      lean_gather<PS>(vb, rb, l);
      lean_compute<N, E, S, p + 1, FMA>(va, t1);
      interleave_ds_valu<2 * E, NV>();
    }
  });
}

template <int N, int E, int S, typename Real, typename TW>
__device__ __forceinline__ void lean_compute_last(cx<Real> (&v)[E], const TW &tw) {
  using LP = LeanPlan<N, E>;
  using PL = typename LP::Sub;
  constexpr int PL1 = PL::P - 1, RL = PL::radix(PL1);
  cx<Real> tl[RL];
  pass_twiddles<PL1>(tl, tw);
  lean_compute<N, E, S, PL1, IsFmaTw<TW>::value>(v, tl);
}

// Cross-wave compute of the forward path (WV-point DFTs over n2 and
// twiddles) for one sequence, in place in v.
// COMB: t[i] already holds group i's rotation.
template <int N, int E, int S, bool COMB, int I, typename Real>
__device__ __forceinline__ void lean_cross_tw(cx<Real> (&z)[(LeanPlan<N, E>::WV)],
                                              const cx<Real> (&t)[(LeanPlan<N, E>::WV)]) {
  if constexpr (COMB) {
    sfor<1, LeanPlan<N, E>::WV>([&](auto ri) {
      constexpr int r = decltype(ri)::value;
      z[r] = ctw<S>(z[r], t[r]);
    });
  } else {
    cross_twiddle<N, E, S, I>(z, t);
  }
}

template <int N, int E, int S, bool COMB, typename Real>
__device__ __forceinline__ void lean_cross_dft(
    cx<Real> (&v)[E], const cx<Real> (&t)[(LeanPlan<N, E>::Q)][(LeanPlan<N, E>::WV)]) {
  using LP = LeanPlan<N, E>;
  constexpr int WV = LP::WV, Q = LP::Q;
  sfor<0, Q>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    cx<Real> z[WV];
    sfor<0, WV>([&](auto ri) { z[decltype(ri)::value] = v[i + Q * decltype(ri)::value]; });
    dft_reg<WV, S>(z);
    lean_cross_tw<N, E, S, COMB, i>(z, t[i]);
    sfor<0, WV>([&](auto ri) { v[i + Q * decltype(ri)::value] = z[decltype(ri)::value]; });
  });
}

// Scatter of the forward path's cross-wave result to the WV regions of X.
template <int N, int E, int PS, typename Real>
__device__ __forceinline__ void lean_cross_scatter(const cx<Real> (&v)[E], cx<Real> *X, int c0) {
  using LP = LeanPlan<N, E>;
  constexpr int LB1 = LdsLen<LP::N1, PS>::value;
  constexpr int WV = LP::WV, Q = LP::Q;
  sfor<0, Q>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    const int n1 = lpad_off<PS, 64 * i, false>(c0);
    sfor<0, WV>([&](auto ri) {
      constexpr int r = decltype(ri)::value;
      X[r * LB1 + n1] = v[i + Q * r];
    });
  });
}

// Gather of the back path's cross-wave input from the WV regions of X.
template <int N, int E, int PS, typename Real>
__device__ __forceinline__ void lean_cross_gather(cx<Real> (&v)[E], const cx<Real> *X, int c0) {
  using LP = LeanPlan<N, E>;
  constexpr int LB1 = LdsLen<LP::N1, PS>::value;
  constexpr int WV = LP::WV, Q = LP::Q;
  sfor<0, Q>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    const int n1 = lpad_off<PS, 64 * i, false>(c0);
    sfor<0, WV>([&](auto ri) {
      constexpr int r = decltype(ri)::value;
      v[i + Q * r] = X[r * LB1 + n1];
    });
  });
}

// Cross-wave compute of the back path (twiddles, WV-point DFTs over k2).
template <int N, int E, int S, bool COMB, typename Real>
__device__ __forceinline__ void lean_cross_idft(
    cx<Real> (&v)[E], const cx<Real> (&t)[(LeanPlan<N, E>::Q)][(LeanPlan<N, E>::WV)]) {
  using LP = LeanPlan<N, E>;
  constexpr int WV = LP::WV, Q = LP::Q;
  sfor<0, Q>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    cx<Real> z[WV];
    sfor<0, WV>([&](auto ri) { z[decltype(ri)::value] = v[i + Q * decltype(ri)::value]; });
    lean_cross_tw<N, E, S, COMB, i>(z, t[i]);
    dft_reg<WV, S>(z);
    sfor<0, WV>([&](auto ri) { v[i + Q * decltype(ri)::value] = z[decltype(ri)::value]; });
  });
}

// Two forward paths (mode order in, scrambled order out) in contexts XA, XB,
// every LDS exchange of one sequence interleaved with arithmetic of the other.
// PRE: barrier first (single buffer set).
template <int N, int E, int S, int PS, bool PRE, int NV, bool LX = false, typename Real,
          typename TW>
__device__ __forceinline__ void lean_fwd2(cx<Real> (&va)[E], cx<Real> (&vb)[E], cx<Real> *XA,
                                          cx<Real> *XB, const TW &tw, int w, int l) {
  using LP = LeanPlan<N, E>;
  constexpr int LB1 = LdsLen<LP::N1, PS>::value;
  constexpr int WV = LP::WV;
  static_assert(WV > 1, "paired kernels need the cross-wave exchange");
  if constexpr (PRE) __syncthreads();
  constexpr bool COMB = CombTw<TW>::value;
  cx<Real> t[LP::Q][WV];
  cross_twiddles(t, tw);
  const int c0 = lpad<PS>(l + 64 * w * LP::Q);
  __builtin_amdgcn_sched_barrier(0);
  lean_cross_dft<N, E, S, COMB>(va, t);
  __builtin_amdgcn_sched_barrier(0);
  lean_cross_scatter<N, E, PS>(va, XA, c0);
  lean_cross_dft<N, E, S, COMB>(vb, t);
  interleave_ds_valu<E, NV>();
  lean_cross_scatter<N, E, PS>(vb, XB, c0);
  __syncthreads();
  const int r0 = w * LB1;
  lean_gather<PS>(va, XA + r0, l);
  __builtin_amdgcn_sched_barrier(0);
  lean_gather<PS>(vb, XB + r0, l);
  lean_compute<N, E, S, 0>(va, (const cx<Real> *)nullptr);
  interleave_ds_valu<E, NV / 2>();
  pair_passes<N, E, S, PS, NV, LX>(va, vb, XA + r0, XB + r0, tw, l);
  lean_compute_last<N, E, S>(vb, tw);
}

// Two back paths (scrambled order in, mode order out) in contexts XA, XB.
template <int N, int E, int S, int PS, bool PRE, int NV, bool LX = false, typename Real,
          typename TW>
__device__ __forceinline__ void lean_back2(cx<Real> (&va)[E], cx<Real> (&vb)[E], cx<Real> *XA,
                                           cx<Real> *XB, const TW &tw, int w, int l) {
  using LP = LeanPlan<N, E>;
  constexpr int LB1 = LdsLen<LP::N1, PS>::value;
  constexpr int WV = LP::WV;
  if constexpr (PRE) __syncthreads();
  const int r0 = w * LB1;
  __builtin_amdgcn_sched_barrier(0);
  lean_compute<N, E, S, 0>(va, (const cx<Real> *)nullptr);
  __builtin_amdgcn_sched_barrier(0);
  pair_passes<N, E, S, PS, NV, LX>(va, vb, XA + r0, XB + r0, tw, l);
  // own regions: the transform's last gathers come before these scatters
  wave_fence();
  const int g0 = r0 + lpad<PS>(l);
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    XA[lpad_off<PS, 64 * m, false>(g0)] = va[m];
  });
  lean_compute_last<N, E, S>(vb, tw);
  interleave_ds_valu<E, NV>();
  wave_fence();
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    XB[lpad_off<PS, 64 * m, false>(g0)] = vb[m];
  });
  __syncthreads();
  constexpr bool COMB = CombTw<TW>::value;
  cx<Real> t[LP::Q][WV];
  cross_twiddles(t, tw);
  const int c0 = lpad<PS>(l + 64 * w * LP::Q);
  lean_cross_gather<N, E, PS>(va, XA, c0);
  __builtin_amdgcn_sched_barrier(0);
  lean_cross_gather<N, E, PS>(vb, XB, c0);
  lean_cross_idft<N, E, S, COMB>(va, t);
  interleave_ds_valu<E, NV>();
  lean_cross_idft<N, E, S, COMB>(vb, t);
}

// ---------------------------------------------------------------------------
// N = 2048 as 8 x 256 (LY = 1).  Thread c = 64 w + l holds modes c + 256 m.
// The inverse path takes the 8-point DFT over its own slots (the three top
// index bits), twiddles w^(c k1), and writes region k1 at position c; after
// the barrier the 8 regions are two 256-point sub-transforms per wave, on
// alternate lanes (lane = 2 t + s, region k1 = 2 w + s, thread t holds
// positions t + 32 m).  A sub-transform is three Stockham passes, radix 8, 8
// and 4: one exchange through the wave's own regions, and one, after the
// second pass, that moves data only between lanes whose index differs in
// bits 4 and 5, done with v_permlane16_swap / v_permlane32_swap in
// registers.  Against the two-level layout (a 4-point cross step, one
// 512-point sub-transform per wave with two LDS exchanges) a transform takes
// two LDS exchanges instead of three.  The forward path runs the same
// sub-transform, writes its own regions, and after the barrier the thread
// gathers position c of every region, twiddles and takes the 8-point DFT,
// which leaves mode c + 256 m in slot m.
struct D8 {
  static constexpr int N = 2048, E = 8, N1 = 256;
  __device__ static int mode(int w, int l, int m) { return 64 * w + l + 256 * m; }
};
// Region length in elements: 256 positions with one pad element every 8
// (288), plus an offset that starts the regions of alternate lanes 64 bytes
// apart modulo 128 (FP64 +12, FP32 +8).  Measured at 256 x N=2048 (FP64, us
// per step): +0 9.50, +4 9.20, +8 9.45, +12 9.12, +16 9.46: 128-byte offsets
// land on the same LDS banks.
template <typename Real> struct D8L {
  static constexpr int RL = 288 + (sizeof(Real) == 8 ? 12 : 8);
  static constexpr int CTX = 8 * RL;
};

// cross twiddles x[k1] = exp(-2 pi i c k1 / N) (XP; else x[1] only, the
// powers formed where they are applied, for kernels short of registers);
// the multiply-add level twiddles of pass 1 (radix 8, base
// exp(-2 pi i (t mod 8) / 64)) and of the two radix-4 butterflies of pass 2
// (bases exp(-2 pi i (t + 32 q) / 256))
template <typename Real, bool XP = true> struct D8Tw {
  cx<Real> x[XP ? 8 : 2];
  cx<Real> p1[8];
  cx<Real> p2[2][4];
};
template <typename Real, bool XP>
__device__ __forceinline__ void d8_cross_twiddles(cx<Real> (&t)[8], const D8Tw<Real, XP> &tw) {
  if constexpr (XP) sfor<1, 8>([&](auto ki) { t[decltype(ki)::value] = tw.x[decltype(ki)::value]; });
  else pow_fill<8>(t, tw.x[1]);
}

// tab[i] = exp(-2 pi i i / 2048)
template <typename Real, bool XP>
__device__ __forceinline__ void load_d8_twiddles(D8Tw<Real, XP> &tw,
                                                 const cx<Real> *__restrict__ tab, int w, int l) {
  const int c = 64 * w + l, t = l >> 1;
  sfor<1, (XP ? 8 : 2)>([&](auto ki) {
    constexpr int k1 = decltype(ki)::value;
    tw.x[k1] = tab[(c * k1) & (D8::N - 1)];
  });
  // level of length len, butterfly kk: b^(R / len) exp(-2 pi i kk / len)
  auto level = [&](cx<Real> *dst, int R, int bidx) {
    for (int len = 2, half = 1; len <= R; len *= 2, half *= 2)
      for (int kk = 0; kk < half; ++kk)
        dst[half + kk] = fma_form(tab[((R / len) * bidx + kk * (D8::N / len)) & (D8::N - 1)]);
  };
  level(tw.p1, 8, 32 * (t & 7));
  level(tw.p2[0], 4, 8 * t);
  level(tw.p2[1], 4, 8 * (t + 32));
}
template <typename Real, bool XP>
__device__ __forceinline__ void load_twiddle_source(D8Tw<Real, XP> &tw, const cx<Real> *tab, int w,
                                                    int l) {
  load_d8_twiddles(tw, tab, w, l);
}

// The second exchange of a sub-transform.  After pass 1 element r of thread
// t belongs at position 64 (t >> 3) + 8 r + (t & 7); pass 2 needs positions
// t' + 32 m in slot m.  Source and destination agree in t & 7; the swap over
// lane bit 5 trades register bit 1 for t bit 4, the swap over lane bit 4
// register bit 0 for t bit 3, and slot m is then register 4 (m & 1) +
// 2 (m >> 2) + ((m >> 1) & 1).
template <typename Real> __device__ __forceinline__ void d8_lane_exchange(cx<Real> (&v)[8]) {
  sfor<0, 4>([&](auto ji) {
    constexpr int r = (decltype(ji)::value & 1) + 4 * (decltype(ji)::value >> 1);  // 0 1 4 5
    lane_swap32(v[r].re, v[r ^ 2].re);
    lane_swap32(v[r].im, v[r ^ 2].im);
  });
  sfor<0, 4>([&](auto ji) {
    constexpr int r = 2 * decltype(ji)::value;  // 0 2 4 6
    lane_swap16(v[r].re, v[r ^ 1].re);
    lane_swap16(v[r].im, v[r ^ 1].im);
  });
  cx<Real> u[8];
  sfor<0, 8>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    u[m] = v[4 * (m & 1) + 2 * (m >> 2) + ((m >> 1) & 1)];
  });
  sfor<0, 8>([&](auto mi) { v[decltype(mi)::value] = u[decltype(mi)::value]; });
}

// passes 1 and 2 of a sub-transform (pass 2: radix-4 butterflies q = 0, 1 on
// slots q + 2 s, positions t + 32 q + 64 s), natural order out
template <int S, typename Real, typename TW>
__device__ __forceinline__ void d8_pass1(cx<Real> (&v)[8], const TW &tw) {
  dft_reg_fma<8, S>(v, tw.p1);
}
template <int S, typename Real, typename TW>
__device__ __forceinline__ void d8_pass2(cx<Real> (&v)[8], const TW &tw) {
  sfor<0, 2>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    cx<Real> z[4];
    sfor<0, 4>([&](auto si) { z[decltype(si)::value] = v[q + 2 * decltype(si)::value]; });
    dft_reg_fma<4, S>(z, tw.p2[q]);
    sfor<0, 4>([&](auto si) { v[q + 2 * decltype(si)::value] = z[decltype(si)::value]; });
  });
}
// the first exchange: pass 0 leaves element r at position 8 t + r
template <typename Real>
__device__ __forceinline__ void d8_scatter0(const cx<Real> (&v)[8], cx<Real> *R, int t) {
  const int b = lpad<3>(8 * t);
  sfor<0, 8>([&](auto ri) { R[b + decltype(ri)::value] = v[decltype(ri)::value]; });
}
template <typename Real>
__device__ __forceinline__ void d8_gather(cx<Real> (&v)[8], const cx<Real> *R, int t) {
  sfor<0, 8>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    v[m] = R[lpad<3>(t + 32 * m)];
  });
}
template <typename Real>
__device__ __forceinline__ void d8_put(const cx<Real> (&v)[8], cx<Real> *R, int t) {
  sfor<0, 8>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    R[lpad<3>(t + 32 * m)] = v[m];
  });
}
// region k1 at position c, for k1 = 0..7
template <typename Real>
__device__ __forceinline__ void d8_cross_put(const cx<Real> (&v)[8], cx<Real> *X, int c) {
  const int o = lpad<3>(c);
  sfor<0, 8>([&](auto ki) { X[decltype(ki)::value * D8L<Real>::RL + o] = v[decltype(ki)::value]; });
}
template <typename Real>
__device__ __forceinline__ void d8_cross_get(cx<Real> (&v)[8], const cx<Real> *X, int c) {
  const int o = lpad<3>(c);
  sfor<0, 8>([&](auto ki) { v[decltype(ki)::value] = X[decltype(ki)::value * D8L<Real>::RL + o]; });
}
template <int S, typename Real, typename TW>
__device__ __forceinline__ void d8_cross_inv(cx<Real> (&v)[8], const TW &tw) {
  dft_reg<8, S>(v);
  cx<Real> t[8];
  d8_cross_twiddles(t, tw);
  sfor<1, 8>([&](auto ki) { v[decltype(ki)::value] = ctw<S>(v[decltype(ki)::value], t[decltype(ki)::value]); });
}
template <int S, typename Real, typename TW>
__device__ __forceinline__ void d8_cross_fwd(cx<Real> (&v)[8], const TW &tw) {
  cx<Real> t[8];
  d8_cross_twiddles(t, tw);
  sfor<1, 8>([&](auto ki) { v[decltype(ki)::value] = ctw<S>(v[decltype(ki)::value], t[decltype(ki)::value]); });
  dft_reg<8, S>(v);
}

// Two inverse paths (mode order in, sub-transform order out) in contexts XA,
// XB, the LDS traffic of one sequence interleaved with the other's
// arithmetic.  PRE: barrier first (single buffer set).
template <int S, bool PRE, int NV, typename Real, typename TW>
__device__ __forceinline__ void d8_inv2(cx<Real> (&va)[8], cx<Real> (&vb)[8], cx<Real> *XA,
                                        cx<Real> *XB, const TW &tw, int w, int l) {
  if constexpr (PRE) __syncthreads();
  const int c = 64 * w + l, t = l >> 1, reg = (2 * w + (l & 1)) * D8L<Real>::RL;
  __builtin_amdgcn_sched_barrier(0);
  d8_cross_inv<S>(va, tw);
  __builtin_amdgcn_sched_barrier(0);
  d8_cross_put(va, XA, c);
  d8_cross_inv<S>(vb, tw);
  interleave_ds_valu<8, NV>();
  d8_cross_put(vb, XB, c);
  __syncthreads();
  d8_gather(va, XA + reg, t);
  __builtin_amdgcn_sched_barrier(0);
  d8_gather(vb, XB + reg, t);
  dft_reg<8, S>(va);
  interleave_ds_valu<8, NV / 2>();
  d8_scatter0(va, XA + reg, t);
  wave_fence();  // scatter before gather (other lanes' values)
  d8_gather(va, XA + reg, t);
  dft_reg<8, S>(vb);
  interleave_ds_valu<16, NV / 2>();
  d8_scatter0(vb, XB + reg, t);
  wave_fence();
  d8_gather(vb, XB + reg, t);
  d8_pass1<S>(va, tw);
  interleave_ds_valu<16, NV>();
  d8_lane_exchange(va);
  d8_pass2<S>(va, tw);
  d8_pass1<S>(vb, tw);
  d8_lane_exchange(vb);
  d8_pass2<S>(vb, tw);
}

// Two forward paths (sub-transform order in, mode order out).
template <int S, bool PRE, int NV, typename Real, typename TW>
__device__ __forceinline__ void d8_fwd2(cx<Real> (&va)[8], cx<Real> (&vb)[8], cx<Real> *XA,
                                        cx<Real> *XB, const TW &tw, int w, int l) {
  if constexpr (PRE) __syncthreads();
  const int c = 64 * w + l, t = l >> 1, reg = (2 * w + (l & 1)) * D8L<Real>::RL;
  __builtin_amdgcn_sched_barrier(0);
  dft_reg<8, S>(va);
  __builtin_amdgcn_sched_barrier(0);
  d8_scatter0(va, XA + reg, t);
  wave_fence();
  d8_gather(va, XA + reg, t);
  dft_reg<8, S>(vb);
  interleave_ds_valu<16, NV / 2>();
  d8_scatter0(vb, XB + reg, t);
  wave_fence();
  d8_gather(vb, XB + reg, t);
  d8_pass1<S>(va, tw);
  interleave_ds_valu<16, NV>();
  d8_lane_exchange(va);
  d8_pass2<S>(va, tw);
  // own regions: the sub-transform's gathers come before these writes
  wave_fence();
  d8_put(va, XA + reg, t);
  d8_pass1<S>(vb, tw);
  interleave_ds_valu<8, NV>();
  d8_lane_exchange(vb);
  d8_pass2<S>(vb, tw);
  wave_fence();
  d8_put(vb, XB + reg, t);
  __syncthreads();
  d8_cross_get(va, XA, c);
  __builtin_amdgcn_sched_barrier(0);
  d8_cross_get(vb, XB, c);
  d8_cross_fwd<S>(va, tw);
  interleave_ds_valu<8, NV>();
  d8_cross_fwd<S>(vb, tw);
}

// LY: the two-level layout (0), N = 2048 as 8 x 256 (1), or the two-level
// layout with the last sub-transform exchange in registers (2, four modes per
// thread; the slot order is that of 0, so stage records and the reverse
// sweep are shared)
template <typename Real, int N, int E, int PS, int LY = 0> struct DuoShape {
  using LP = LeanPlan<N, E>;
  static constexpr int W = LP::W;
  static constexpr int LB1 = LdsLen<LP::N1, PS>::value;
  static constexpr int CTX = LY == 1 ? D8L<Real>::CTX : LP::WV * LB1;  // one transform's exchange context
  static constexpr int LIMIT = 160 * 1024;
  static constexpr int NSET = 4 * CTX * (int)sizeof(cx<Real>) <= LIMIT ? 2 : 1;
  static constexpr int PER_INST = NSET * 2 * CTX;
  static constexpr int LDS_BYTES = PER_INST * (int)sizeof(cx<Real>);
  static constexpr int THREADS = 64 * W;
  static_assert(W > 1, "one instance spans several wavefronts");
  static_assert(LDS_BYTES <= LIMIT, "LDS over the gfx950 per-workgroup limit");
  static_assert(LY != 1 || (N == D8::N && E == D8::E && PS == 3), "the 8 x 256 layout is N = 2048, E = 8");
};

// mode of slot m of thread (w, l)
template <int LY, int N, int E> __device__ __forceinline__ int duo_mode(int w, int l, int m) {
  if constexpr (LY == 1) return D8::mode(w, l, m);
  else return WavePlan<N, E, 1, 0>::mode(w, l, m);
}
// storage position of slot m on the transformed side (the stage records of
// the inverse transforms): a bijection onto [0, N) with lanes contiguous,
// the same in the forward recompute and the reverse sweep of a layout
template <int LY, int N, int E> __device__ __forceinline__ int duo_tslot(int w, int l, int m) {
  if constexpr (LY == 1) return l + 64 * (w + 4 * m);
  else return WavePlan<N, E, 1, 0>::tslot(w, l, m);
}

// REC: record the stage inputs (mode order) and inverse transforms (slot
// order duo_tslot of the layout, which its reverse sweep reads)
template <typename Real, int N, int E, int PS, int NV, int FT, bool REC, int LY = 0>
__global__ void __launch_bounds__((DuoShape<Real, N, E, PS, LY>::THREADS)) rk4_duo(RunArgs a) {
  using SH = DuoShape<Real, N, E, PS, LY>;
  using WP = WavePlan<N, E, 1, 0>;
  constexpr bool ONESET = SH::NSET == 1;
  __shared__ cx<Real> lds[SH::PER_INST];

  const int lane = (int)threadIdx.x & 63;
  const int w = (int)threadIdx.x >> 6;
  const int id = a.order[blockIdx.x];
  const DevInst d = a.inst[id];
  // round parity 0 (inverse transforms) and 1 (forward transforms)
  cx<Real> *XA0 = lds, *XB0 = lds + SH::CTX;
  cx<Real> *XA1 = ONESET ? XA0 : lds + 2 * SH::CTX, *XB1 = ONESET ? XB0 : lds + 3 * SH::CTX;
  cx<Real> *A = reinterpret_cast<cx<Real> *>(a.A) + d.offset;
  const double *kap = a.kappa + d.offset;
  const double *omg = a.omega + d.offset;

  std::conditional_t<
      LY == 1, D8Tw<Real>,
      std::conditional_t<FT >= 2, FmaTw<N, E, Real, FT == 2>,
                         std::conditional_t<FT == 1, FullTw<N, E, Real>, LeanTw<N, E, Real>>>>
      tw;
  if constexpr (LY == 1)
    load_twiddle_source(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);
  else
    load_twiddle_source<N, E>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  // KU: kappa the same for every mode of the instance, -kappa/2 one
  // wave-uniform value instead of E registers per thread.  Taken in the
  // 8 x 256 layout only; measured (256 instances, us per RK4 step): N = 2048
  // FP64 8.98 -> 8.80, FP32 6.95 either way; the two-level layout at
  // N = 1024 5.88 -> 5.94, so it keeps the per-mode registers.
  bool bad = false;
  auto run = [&](auto ku) {
    constexpr bool KU = decltype(ku)::value;
    const Real lr0 = (Real)(-0.5 * d.kappa0);
    cx<Real> y[E], yw[E], va[E], vb[E];
    Real lr[E];
    double om[E];
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const int i = duo_mode<LY, N, E>(w, lane, m);
      y[m] = A[i];
      if constexpr (!KU) lr[m] = (Real)(-0.5 * kap[i]);
      om[m] = omg[i];
    });
    const bool pump_owner = (w == 0 && lane == 0);
    const Real gn = (Real)d.g0n;                // g0 / N, mode side
    const Real gt = (Real)(d.g0n * (double)N);  // g0, transformed side
    const cx<Real> pump = {(Real)d.pump_re, (Real)d.pump_im};
    const double h = a.h;
    const Real hh = (Real)(0.5 * h), hf = (Real)h, h6 = (Real)(h / 6.0);
    cx<Real> *ckpt = reinterpret_cast<cx<Real> *>(a.ckpt);
    cx<Real> *stages = reinterpret_cast<cx<Real> *>(a.stages);
    int32_t to_ckpt = a.ckpt_every;
    int64_t ckpt_slot = 0;

    // W = L(sig) u + p in slot m
    auto lin = [&](const cx<Real> &u, auto mi, double sig) {
      constexpr int m = decltype(mi)::value;
      const Real det = (Real)(om[m] - sig);
      const Real lm = KU ? lr0 : lr[m];
      cx<Real> q = {lm * u.re - det * u.im, lm * u.im + det * u.re};
      if constexpr (m == E / 2) {
        if (pump_owner) q = cadd(q, pump);
      }
      return q;
    };
    auto cube = [](const cx<Real> &x) {
      const Real p = x.re * x.re + x.im * x.im;
      return cx<Real>{p * x.re, p * x.im};
    };
    auto rec_u = [&](int64_t n, int s, auto mi, const cx<Real> &u) {
      if constexpr (REC) {
        constexpr int m = decltype(mi)::value;
        stages[stage_offset(n, s, a.total) + d.offset + duo_mode<LY, N, E>(w, lane, m)] = u;
      }
    };
    auto rec_a = [&](int64_t n, int s, auto mi, const cx<Real> &x) {
      if constexpr (REC) {
        constexpr int m = decltype(mi)::value;
        stages[stage_offset(n, s, a.total) + a.total + d.offset + duo_tslot<LY, N, E>(w, lane, m)] = x;
      }
    };

    for (int64_t n = 0; n < a.n_steps; ++n) {
      const double t0 = (double)(a.step0 + n) * h;
      const double s1 = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0);
      const double s2 = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + 0.5 * h);
      const double s4 = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + h);
      // ---- R0: a_1 = IDFT(y), IDFT(y + h/2 W_1)
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        rec_u(n, 0, mi, y[m]);
        va[m] = y[m];
        const cx<Real> w1 = lin(y[m], mi, s1);
        vb[m] = {y[m].re + hh * w1.re, y[m].im + hh * w1.im};
      });
      if constexpr (LY == 1) d8_inv2<+1, ONESET, NV>(va, vb, XA0, XB0, tw, w, lane);
      else lean_fwd2<N, E, +1, PS, ONESET, NV, LY == 2>(va, vb, XA0, XB0, tw, w, lane);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        rec_a(n, 0, mi, va[m]);
        const cx<Real> b1 = cube(va[m]);
        // a_2 = IDFT(y + h/2 (W_1 + i (g0/N) DFT b_1)) = IDFT(y + h/2 W_1) + h/2 i g0 b_1
        const cx<Real> a2 = {vb[m].re - hh * gt * b1.im, vb[m].im + hh * gt * b1.re};
        rec_a(n, 1, mi, a2);
        va[m] = b1;
        vb[m] = cube(a2);
      });
      // ---- R1: K'_1, K'_2
      if constexpr (LY == 1) d8_fwd2<-1, ONESET, NV>(va, vb, XA1, XB1, tw, w, lane);
      else lean_back2<N, E, -1, PS, ONESET, NV, LY == 2>(va, vb, XA1, XB1, tw, w, lane);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const cx<Real> w1 = lin(y[m], mi, s1);
        const cx<Real> k1 = {w1.re - gn * va[m].im, w1.im + gn * va[m].re};
        const cx<Real> u2 = {y[m].re + hh * k1.re, y[m].im + hh * k1.im};
        rec_u(n, 1, mi, u2);
        const cx<Real> w2 = lin(u2, mi, s2);
        const cx<Real> k2 = {w2.re - gn * vb[m].im, w2.im + gn * vb[m].re};
        const cx<Real> u3 = {y[m].re + hh * k2.re, y[m].im + hh * k2.im};
        rec_u(n, 2, mi, u3);
        const cx<Real> w3 = lin(u3, mi, s2);
        // from here on y + h W_3 and y + h/6 (k_1 + 2 k_2 + 2 W_3) stand for y,
        // the accumulator and W_3: u_4 = yw + h i (g0/N) K'_3 and
        // y' = y + h/6 (k_1 + 2 k_2 + 2 W_3) + h/6 (2 i (g0/N) K'_3 + k_4)
        yw[m] = {y[m].re + hf * w3.re, y[m].im + hf * w3.im};
        y[m] = {y[m].re + h6 * (k1.re + (Real)2 * (k2.re + w3.re)),
                y[m].im + h6 * (k1.im + (Real)2 * (k2.im + w3.im))};
        va[m] = u3;
        vb[m] = yw[m];
      });
      // ---- R2: a_3 = IDFT(u_3), IDFT(y + h W_3)
      if constexpr (LY == 1) d8_inv2<+1, ONESET, NV>(va, vb, XA0, XB0, tw, w, lane);
      else lean_fwd2<N, E, +1, PS, ONESET, NV, LY == 2>(va, vb, XA0, XB0, tw, w, lane);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        rec_a(n, 2, mi, va[m]);
        const cx<Real> b3 = cube(va[m]);
        // a_4 = IDFT(y + h (W_3 + i (g0/N) DFT b_3)) = IDFT(y + h W_3) + h i g0 b_3
        const cx<Real> a4 = {vb[m].re - hf * gt * b3.im, vb[m].im + hf * gt * b3.re};
        rec_a(n, 3, mi, a4);
        va[m] = b3;
        vb[m] = cube(a4);
      });
      // ---- R3: K'_3, K'_4
      if constexpr (LY == 1) d8_fwd2<-1, ONESET, NV>(va, vb, XA1, XB1, tw, w, lane);
      else lean_back2<N, E, -1, PS, ONESET, NV, LY == 2>(va, vb, XA1, XB1, tw, w, lane);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        // i (g0/N) K'_3
        const cx<Real> q3 = {-gn * va[m].im, gn * va[m].re};
        const cx<Real> u4 = {yw[m].re + hf * q3.re, yw[m].im + hf * q3.im};
        rec_u(n, 3, mi, u4);
        const cx<Real> w4 = lin(u4, mi, s4);
        const cx<Real> k4 = {w4.re - gn * vb[m].im, w4.im + gn * vb[m].re};
        y[m] = {y[m].re + h6 * ((Real)2 * q3.re + k4.re), y[m].im + h6 * ((Real)2 * q3.im + k4.im)};
      });
      if (ckpt != nullptr && --to_ckpt == 0) {
        to_ckpt = a.ckpt_every;
        cx<Real> *dst = ckpt + ckpt_slot * a.total + d.offset;
        sfor<0, E>([&](auto mi) {
          constexpr int m = decltype(mi)::value;
          dst[duo_mode<LY, N, E>(w, lane, m)] = y[m];
        });
        ++ckpt_slot;
      }
    }
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      A[duo_mode<LY, N, E>(w, lane, m)] = y[m];
      bad |= !(isfinite(y[m].re) && isfinite(y[m].im));
    });
  };
  if constexpr (LY == 1) {
    if (d.kappa_uniform) run(std::true_type{});
    else run(std::false_type{});
  } else {
    run(std::false_type{});
  }
  if (bad) atomicOr(&a.flags[id], 1);
}

// Reverse sweep over one checkpoint segment, paired like the forward step.
// With ybar' the cotangent of the step's output, kbar_s = w_s h ybar' +
// c_{s+1} h ubar_{s+1}, and ubar_s = conj(L_s) kbar_s + DFT(q_s), where
// q_s = 2 |a_s|^2 z_s + a_s^2 conj(z_s), z_s = IDFT(-i (g0/N) kbar_s) (the
// transpose of the Kerr term's derivative at a_s = IDFT(u_s)).  By
// linearity, IDFT(ubar_s) = IDFT(conj(L_s) kbar_s) + N q_s, so with
// Ybar = IDFT(ybar') and P_s = IDFT(conj(L_s) kbar_s):
//   z_{s-1} = -i (g0/N) (w_{s-1} h Ybar + c_s h (P_s + N q_s)),
// and a step takes four rounds of two transforms:
//   A: Ybar, P_4             -> z_4, q_4, z_3, q_3
//   B: DFT q_4, q_3          -> ubar_4, kbar_3, ubar_3, kbar_2
//   C: IDFT(kbar_2), IDFT(h/6 ybar' + h/2 conj(L_2) kbar_2)
//                            -> z_2, q_2, z_1, q_1
//   D: DFT q_2, q_1          -> ubar_2, kbar_1, ubar_1;  ybar = ybar' + sum ubar_s
// (round C transforms the combinations themselves, known after round B:
// IDFT(kbar_2) = h/3 Ybar + h/2 IDFT(ubar_3), so Ybar need not be kept from
// round A to round C).
// Parameter cotangents per stage: gbar_omega += Re(conj(kbar) i u),
// gbar_kappa -= Re(conj(kbar) u) / 2, gbar_Ain += sqrt(kappa_ext) kbar at
// mu = 0.  This kernel only stores kbar_s (a.kbar); adj_params forms the
// sums from it and the stage inputs u_s afterwards, so neither the
// accumulators nor u_s occupy registers here.  The time-domain records a_s
// are loaded a round before they are needed.
template <typename Real, int N, int E, int PS, int NV, int FT, int LY = 0>
__global__ void __launch_bounds__((DuoShape<Real, N, E, PS, LY>::THREADS)) rk4_duo_reverse(AdjArgs a) {
  using SH = DuoShape<Real, N, E, PS, LY>;
  constexpr bool ONESET = SH::NSET == 1;
  __shared__ cx<Real> lds[SH::PER_INST];

  const int lane = (int)threadIdx.x & 63;
  const int w = (int)threadIdx.x >> 6;
  const int id = a.order[blockIdx.x];
  const DevInst d = a.inst[id];
  cx<Real> *XA0 = lds, *XB0 = lds + SH::CTX;
  cx<Real> *XA1 = ONESET ? XA0 : lds + 2 * SH::CTX, *XB1 = ONESET ? XB0 : lds + 3 * SH::CTX;
  const double *kap = a.kappa + d.offset;
  const double *omg = a.omega + d.offset;
  cx<Real> *gA = reinterpret_cast<cx<Real> *>(a.gA) + d.offset;
  const cx<Real> *stages = reinterpret_cast<const cx<Real> *>(a.stages);

  std::conditional_t<
      LY == 1, D8Tw<Real, false>,
      std::conditional_t<FT >= 2, FmaTw<N, E, Real, FT == 2>,
                         std::conditional_t<FT == 1, FullTw<N, E, Real>, LeanTw<N, E, Real>>>>
      tw;
  if constexpr (LY == 1)
    load_twiddle_source(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);
  else
    load_twiddle_source<N, E>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  cx<Real> yb1[E], yb[E], k2[E], va[E], vb[E], ra[E], rb[E];
  Real lr[E];
  double om[E];
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = duo_mode<LY, N, E>(w, lane, m);
    yb1[m] = gA[i];
    lr[m] = (Real)(-0.5 * kap[i]);
    om[m] = omg[i];
  });
  cx<Real> *kbar = reinterpret_cast<cx<Real> *>(a.kbar);
  const Real gn = (Real)d.g0n, nn_r = (Real)N;
  const double h = a.h;
  const Real hw1 = (Real)(h / 6.0), hw2 = (Real)(h / 3.0), hh = (Real)(0.5 * h), hf = (Real)h;

  // conj(L(sig)) k in slot m
  auto clin = [&](const cx<Real> &k, auto mi, double sig) {
    constexpr int m = decltype(mi)::value;
    const Real det = (Real)(om[m] - sig);
    return cx<Real>{lr[m] * k.re + det * k.im, lr[m] * k.im - det * k.re};
  };
  // -i (g0/N) x
  auto mig = [&](const cx<Real> &x) { return cx<Real>{gn * x.im, -gn * x.re}; };
  // 2 |a|^2 z + a^2 conj(z)
  auto kerr_t = [](const cx<Real> &z, const cx<Real> &av) {
    const Real p2 = (Real)2 * (av.re * av.re + av.im * av.im);
    const cx<Real> a2 = {av.re * av.re - av.im * av.im, (Real)2 * av.re * av.im};
    return cx<Real>{p2 * z.re + a2.re * z.re + a2.im * z.im,
                    p2 * z.im + a2.im * z.re - a2.re * z.im};
  };
  // kbar_s of step n, for the parameter cotangents (launch_adj_params)
  auto store_kbar = [&](int64_t n, int s, auto mi, const cx<Real> &kv) {
    constexpr int m = decltype(mi)::value;
    kbar[(n * 4 + s) * a.total + d.offset + duo_mode<LY, N, E>(w, lane, m)] = kv;
  };
  // record addresses are rebuilt at each use (an opaque base) rather than
  // kept in registers for the whole run
  auto load_a = [&](cx<Real> (&dst)[E], int64_t n, int s) {
    const cx<Real> *rec = stages + stage_offset(n, s, a.total) + a.total + d.offset;
    int base = duo_tslot<LY, N, E>(w, lane, 0);
    asm volatile("" : "+v"(base));
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      dst[m] = rec[base + (duo_tslot<LY, N, E>(w, lane, m) - duo_tslot<LY, N, E>(w, lane, 0))];
    });
  };

  for (int nn = a.n_seg - 1; nn >= 0; --nn) {
    const double t0 = (double)(a.step_first + nn) * h;
    const double s1 = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0);
    const double s2 = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + 0.5 * h);
    const double s4 = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + h);
    // ---- A: Ybar = IDFT(ybar'), P_4 = IDFT(conj(L_4) kbar_4), kbar_4 = h/6 ybar'
    load_a(ra, nn, 3);
    load_a(rb, nn, 2);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      va[m] = yb1[m];
      vb[m] = clin(cx<Real>{hw1 * yb1[m].re, hw1 * yb1[m].im}, mi, s4);
    });
    if constexpr (LY == 1) d8_inv2<+1, ONESET, NV>(va, vb, XA0, XB0, tw, w, lane);
    else lean_fwd2<N, E, +1, PS, ONESET, NV, lx_ok<N, E>()>(va, vb, XA0, XB0, tw, w, lane);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const cx<Real> q4 = kerr_t(mig(cx<Real>{hw1 * va[m].re, hw1 * va[m].im}), ra[m]);
      const cx<Real> x3 = {hw2 * va[m].re + hf * (vb[m].re + nn_r * q4.re),
                           hw2 * va[m].im + hf * (vb[m].im + nn_r * q4.im)};
      va[m] = q4;
      vb[m] = kerr_t(mig(x3), rb[m]);
    });
    // ---- B: DFT(q_4), DFT(q_3)
    if constexpr (LY == 1) d8_fwd2<-1, ONESET, NV>(va, vb, XA1, XB1, tw, w, lane);
    else lean_back2<N, E, -1, PS, ONESET, NV, lx_ok<N, E>()>(va, vb, XA1, XB1, tw, w, lane);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const cx<Real> k4 = {hw1 * yb1[m].re, hw1 * yb1[m].im};
      const cx<Real> c4 = clin(k4, mi, s4);
      const cx<Real> ub4 = {c4.re + va[m].re, c4.im + va[m].im};
      store_kbar(nn, 3, mi, k4);
      const cx<Real> k3 = {hw2 * yb1[m].re + hf * ub4.re, hw2 * yb1[m].im + hf * ub4.im};
      const cx<Real> c3 = clin(k3, mi, s2);
      const cx<Real> ub3 = {c3.re + vb[m].re, c3.im + vb[m].im};
      store_kbar(nn, 2, mi, k3);
      yb[m] = {yb1[m].re + ub4.re + ub3.re, yb1[m].im + ub4.im + ub3.im};
      k2[m] = {hw2 * yb1[m].re + hh * ub3.re, hw2 * yb1[m].im + hh * ub3.im};
      const cx<Real> c2 = clin(k2[m], mi, s2);
      va[m] = k2[m];
      vb[m] = {hw1 * yb1[m].re + hh * c2.re, hw1 * yb1[m].im + hh * c2.im};
    });
    // ---- C: IDFT(kbar_2) = h/3 Ybar + h/2 IDFT(ubar_3),
    //         IDFT(h/6 ybar' + h/2 conj(L_2) kbar_2) = h/6 Ybar + h/2 P_2
    load_a(ra, nn, 1);
    load_a(rb, nn, 0);
    if constexpr (LY == 1) d8_inv2<+1, ONESET, NV>(va, vb, XA0, XB0, tw, w, lane);
    else lean_fwd2<N, E, +1, PS, ONESET, NV, lx_ok<N, E>()>(va, vb, XA0, XB0, tw, w, lane);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const cx<Real> q2 = kerr_t(mig(va[m]), ra[m]);
      const cx<Real> x1 = {vb[m].re + hh * nn_r * q2.re, vb[m].im + hh * nn_r * q2.im};
      va[m] = q2;
      vb[m] = kerr_t(mig(x1), rb[m]);
    });
    // ---- D: DFT(q_2), DFT(q_1)
    if constexpr (LY == 1) d8_fwd2<-1, ONESET, NV>(va, vb, XA1, XB1, tw, w, lane);
    else lean_back2<N, E, -1, PS, ONESET, NV, lx_ok<N, E>()>(va, vb, XA1, XB1, tw, w, lane);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const cx<Real> c2 = clin(k2[m], mi, s2);
      const cx<Real> ub2 = {c2.re + va[m].re, c2.im + va[m].im};
      store_kbar(nn, 1, mi, k2[m]);
      const cx<Real> k1 = {hw1 * yb1[m].re + hh * ub2.re, hw1 * yb1[m].im + hh * ub2.im};
      const cx<Real> c1 = clin(k1, mi, s1);
      const cx<Real> ub1 = {c1.re + vb[m].re, c1.im + vb[m].im};
      store_kbar(nn, 0, mi, k1);
      yb1[m] = {yb[m].re + ub2.re + ub1.re, yb[m].im + ub2.im + ub1.im};
    });
  }
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = duo_mode<LY, N, E>(w, lane, m);
    gA[i] = yb1[m];
  });
}

// Parameter cotangents of one segment from the stage inputs u_s and the
// kbar_s the paired reverse sweep stored: one thread per mode, summing over
// the segment's steps and stages (FP64).
__global__ void __launch_bounds__(256) adj_params(AdjArgs a, int n) {
  const int nb = (n + 255) / 256;
  const int slot = (int)blockIdx.x / nb, i = ((int)blockIdx.x % nb) * 256 + (int)threadIdx.x;
  if (slot >= a.count || i >= n) return;
  const int id = a.order[slot];
  const DevInst d = a.inst[id];
  const cx<double> *st = reinterpret_cast<const cx<double> *>(a.stages);
  const cx<double> *kb = reinterpret_cast<const cx<double> *>(a.kbar);
  double go = 0.0, gk = 0.0;
  cx<double> gain = {0.0, 0.0};
  for (int nn = 0; nn < a.n_seg; ++nn) {
    for (int s = 0; s < 4; ++s) {
      const cx<double> u = st[stage_offset(nn, s, a.total) + d.offset + i];
      const cx<double> kv = kb[((int64_t)nn * 4 + s) * a.total + d.offset + i];
      go += kv.im * u.re - kv.re * u.im;
      gk -= 0.5 * (kv.re * u.re + kv.im * u.im);
      if (i == n / 2) gain = cadd(gain, kv);
    }
  }
  if (a.g_omega) a.g_omega[d.offset + i] += go;
  if (a.g_kappa) a.g_kappa[d.offset + i] += gk;
  if (i == n / 2 && a.g_ain) {
    a.g_ain[2 * id] += d.sqrt_kext * gain.re;
    a.g_ain[2 * id + 1] += d.sqrt_kext * gain.im;
  }
}

hipError_t launch_adj_params(int n, const AdjArgs &a, hipStream_t st) {
  const int nb = (n + 255) / 256;
  hipLaunchKernelGGL(adj_params, dim3(a.count * nb), dim3(256), 0, st, a, n);
  return hipGetLastError();
}

template <typename Real, int N, int E, int PS, int NV, int FT>
hipError_t launch_duo_adj(const AdjArgs &a, hipStream_t st) {
  using SH = DuoShape<Real, N, E, PS>;
  hipLaunchKernelGGL((rk4_duo_reverse<Real, N, E, PS, NV, FT>), dim3(a.count), dim3(SH::THREADS),
                     0, st, a);
  return hipGetLastError();
}

// the 8 x 256 layout, forward (with stage records for its reverse sweep) and
// reverse
template <typename Real, int NV>
hipError_t launch_duo8_fwd(const RunArgs &a, hipStream_t st) {
  using SH = DuoShape<Real, D8::N, D8::E, 3, 1>;
  if (a.stages)
    hipLaunchKernelGGL((rk4_duo<Real, D8::N, D8::E, 3, NV, 2, true, 1>), dim3(a.count),
                       dim3(SH::THREADS), 0, st, a);
  else
    hipLaunchKernelGGL((rk4_duo<Real, D8::N, D8::E, 3, NV, 2, false, 1>), dim3(a.count),
                       dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}
template <typename Real, int NV>
hipError_t launch_duo8_adj(const AdjArgs &a, hipStream_t st) {
  using SH = DuoShape<Real, D8::N, D8::E, 3, 1>;
  hipLaunchKernelGGL((rk4_duo_reverse<Real, D8::N, D8::E, 3, NV, 2, 1>), dim3(a.count),
                     dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

template <typename Real, int N, int E, int PS, int NV, int FT, int LY = 0>
hipError_t launch_duo_fwd(const RunArgs &a, hipStream_t st) {
  using SH = DuoShape<Real, N, E, PS, LY>;
  if (a.stages)
    hipLaunchKernelGGL((rk4_duo<Real, N, E, PS, NV, FT, true, LY>), dim3(a.count),
                       dim3(SH::THREADS), 0, st, a);
  else
    hipLaunchKernelGGL((rk4_duo<Real, N, E, PS, NV, FT, false, LY>), dim3(a.count),
                       dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

// defined in cme_lean.hip: the reverse sweep over the stage records (u_s in
// mode order, a_s in the time-domain slot order this kernel also uses)
template <typename Real, int N, int E, int PS>
hipError_t launch_lean_adj(const AdjArgs &a, hipStream_t st);

// NV: VALU instructions scheduled after each LDS instruction of the other
// sequence (reported as the variant's exchange field)
// FT: twiddles formed from one base per pass (0), all powers held in
// registers (1), or the level twiddles of the multiply-add form and the
// cross-wave twiddles of each element group held in registers (2); reported
// as exchange = NV + 16 FT.  The reverse sweep holds all powers in registers
// (FT = 1), or for an FT = 2 kernel the multiply-add level twiddles with one
// set of cross-wave powers (3: the per-group ones would spill it); it reads
// the stage records in the same slot order whatever the forward kernel's
// twiddle source.
// Reverse sweep of a paired forward kernel: the paired reverse, except at
// eight wavefronts per instance (N = 4096), where its registers do not fit
// two waves per SIMD and the lean reverse, which reads the same stage
// records, is used.
template <typename Real, int N, int E, int PS, int NV, int FT> constexpr AdjLaunch duo_adj_ptr() {
  if constexpr (N / (64 * E) >= 8) return &launch_lean_adj<Real, N, E, PS>;
  else return &launch_duo_adj<Real, N, E, PS, NV, FT == 2 ? 3 : 1>;
}

// LX: the last sub-transform exchange in registers (layout 2), reported as
// + 64 in the tuning field
template <typename Real, int N, int E, int PS, int NV, int FT, bool LX = false>
constexpr Variant duo_variant() {
  constexpr int LY = LX ? 2 : 0;
  using SH = DuoShape<Real, N, E, PS, LY>;
  if constexpr (std::is_same<Real, double>::value)
    return Variant{0, N, E, 1, PS, NV + 16 * FT + 64 * LX, 2, 1, SH::THREADS, SH::LDS_BYTES,
                   &launch_duo_fwd<Real, N, E, PS, NV, FT, LY>, duo_adj_ptr<Real, N, E, PS, NV, FT>(), 0,
                   N / (64 * E) < 8 ? 1 : 0};
  else  // FP32 plans have no adjoint
    return Variant{1, N, E, 1, PS, NV + 16 * FT + 64 * LX, 2, 1, SH::THREADS, SH::LDS_BYTES,
                   &launch_duo_fwd<Real, N, E, PS, NV, FT, LY>, nullptr};
}

// 8 x 256 layout: reported with two sub-transforms per wave (v = 2)
template <typename Real, int NV> constexpr Variant duo8_variant() {
  using SH = DuoShape<Real, D8::N, D8::E, 3, 1>;
  if constexpr (std::is_same<Real, double>::value)
    return Variant{0, D8::N, D8::E, 2, 3, NV + 32, 2, 1, SH::THREADS, SH::LDS_BYTES,
                   &launch_duo8_fwd<Real, NV>, &launch_duo8_adj<Real, NV>, 0, 1};
  else  // FP32 plans have no adjoint
    return Variant{1, D8::N, D8::E, 2, 3, NV + 32, 2, 1, SH::THREADS, SH::LDS_BYTES,
                   &launch_duo8_fwd<Real, NV>, nullptr};
}

// The first entry of a size is its default.  N = 512 and 1024 run four
// elements per thread (two and four wavefronts per instance: 39% and 21%
// faster than the previous defaults at 256 instances); N = 4096 runs eight
// wavefronts per instance, two per SIMD, with the twiddles rebuilt on use
// (the register-held tables do not fit), 5% faster than the lean kernel.
// N = 2048: the 8 x 256 layout with the multiply-add butterflies (FP64),
// else the two-level layout with them (FT = 2).  Round-robin timings of
// 256 x N=2048 (sweep workload, us per step): 8 x 256 NV = 5 / 6 / 7 / 8:
// 9.12 / 9.08 / 9.04 / 9.04; two-level FT = 2 NV = 5: 9.38 (2747 VALU
// instructions per wave and step in place of 2967 with every power held:
// 9.55); FP32 8 x 256 NV = 5 / 7 / 8 / 12 / 16: 7.07 / 7.03 / 6.97 / 6.99 /
// 7.00, two-level FT = 2 7.09 (7.52 with every power held); FP64 NV = 10 and
// 12: 8.99 and 9.28.  At N = 1024 (radix-4 passes) the multiply-add form saves 7% of the
// instructions and no time, so it is not built there.  The 8 x 256
// layout's adjoint runs in the same layout (reverse sweep with the
// cross-wave powers formed on use): 61.9 against 64.6 ms on the two-level
// variant for the N = 2048 gradient workload.
// N = 512 and 1024 take the last sub-transform exchange in registers
// (lane_exchange4): 256 x N=1024 6.78 -> 6.07 us per step (FP32 4.56 ->
// 4.29), 256 x N=512 4.93 -> 4.86 (FP32 3.91 -> 3.81).
static const Variant kDuoVariants[] = {
    duo_variant<double, 512, 4, 2, 4, 1, true>(), duo_variant<double, 1024, 4, 2, 5, 1, true>(),
    duo_variant<double, 512, 4, 2, 4, 1>(),  duo_variant<double, 1024, 4, 2, 5, 1>(),
    duo_variant<double, 1024, 4, 2, 4, 1>(), duo_variant<double, 1024, 8, 3, 4, 1>(),
    duo8_variant<double, 7>(),               duo8_variant<double, 5>(),
    duo_variant<double, 2048, 8, 3, 5, 2>(), duo_variant<double, 2048, 8, 3, 4, 2>(),
    duo_variant<double, 2048, 8, 3, 5, 1>(), duo_variant<double, 2048, 8, 3, 4, 1>(),
    duo_variant<double, 2048, 8, 3, 4, 0>(), duo_variant<double, 4096, 8, 3, 4, 0>(),
    duo_variant<double, 4096, 8, 3, 5, 0>(),
};

// FP32: the same kernels with FP32 state and transforms (time and detuning
// bookkeeping in FP64, rounded once per stage); the defaults for FP32
// N = 512, 1024 (four modes per thread) and 2048: 36%, 38% and 17% faster
// than the one-transform wave kernel at 256 instances.
static const Variant kDuoVariantsF32[] = {
    duo_variant<float, 512, 4, 2, 4, 1, true>(), duo_variant<float, 1024, 4, 2, 5, 1, true>(),
    duo_variant<float, 512, 4, 2, 4, 1>(),  duo_variant<float, 1024, 4, 2, 5, 1>(),
    duo_variant<float, 1024, 4, 2, 4, 1>(), duo_variant<float, 1024, 8, 3, 5, 1>(),
    duo8_variant<float, 8>(),
    duo_variant<float, 2048, 8, 3, 5, 2>(), duo_variant<float, 2048, 8, 3, 4, 2>(),
    duo_variant<float, 2048, 8, 3, 5, 1>(), duo_variant<float, 2048, 8, 3, 4, 1>(),
};

const Variant *variants_duo_f32(int *count) {
  *count = (int)(sizeof(kDuoVariantsF32) / sizeof(kDuoVariantsF32[0]));
  return kDuoVariantsF32;
}

const Variant *variants_duo(int *count) {
  *count = (int)(sizeof(kDuoVariants) / sizeof(kDuoVariants[0]));
  return kDuoVariants;
}

}  // namespace cme
