// cme_stream.hip -- classic RK4 on the two-level transform of cme_fft.hpp with
// the RK4 vectors kept in global memory instead of registers.
//
// For the largest LDS-resident transforms (N = 8192: 128 KiB of FP64 field,
// one instance per CU) a thread owns 16 modes, and holding the state y, the
// RK4 partial update and the stage input in registers beside the transform
// and its twiddles does not fit the 256 registers a lane has at two
// wavefronts per SIMD.  Here only the stage input u_s lives in registers
// across the two transforms of a stage; y is read from and written back to
// the caller's state in place, and the stage derivatives, the partial update
// and u_4 sit in the class workspace (two complex values per mode).
// Every access is coalesced (lanes own consecutive modes) and the
// per-instance vectors stay in L2 / MALL, so the traffic they add is on-chip.
//
// Per RK4 stage s (Sec. 2; stage times t, t+h/2, t+h/2, t+h): a = IDFT(u_s),
// b = |a|^2 a, NK = DFT(b) (Eq. (4), the 1/N folded into g0/N), then
//   k_s = (-kappa/2 + i(omega' - sigma(t_s))) u_s + i (g0/N) NK + [mu = 0] pump,
// and the next stage input u_{s+1} = y + c_{s+1} h k_s.  Two workspace
// vectors carry the step: stages 1 and 2 store k_1 and k_2 alone (the stage
// inputs u_2 = y + h/2 k_1 and u_3 = y + h/2 k_2 are formed again from them
// and y where needed), stage 3 stores the partial update
// P = y + h/6 k_1 + h/3 k_2 + h/3 k_3 and u_4, and stage 4 writes the new state
// y = P + h/6 k_4 without reading y.  Per mode and step that is 208 bytes of
// global traffic in FP64 with omega' held in registers (plus 32 for kappa
// where it varies over the modes; where it is the same for every mode of an
// instance it is not read), and in FP32, with y and -kappa/2 in registers
// too, 72 bytes whatever kappa.
#include <type_traits>

#include "cme_lean.hpp"
#include "cme_wave.hpp"

namespace cme {

// The two-level transform of cme_fft.hpp (fft_fwdpath / fft_backpath, one
// element of the cross-wave DFT per lane and slot: Q = 1) with only the
// sub-transform twiddles held in registers, all their powers or (PB) one
// base per pass.  The cross-wave twiddles are formed where they are applied:
//   forward path  w^{n1 r}, r < WV, as powers of w^{n1} (n1 = l + 64 w);
//   back path     w^{(l + 64 j)(w V + v)} = w^{l (w V + v)} (w^{64 (w V + v)})^j
// (w = e^{-2 pi i / N}, conjugated for the inverse sign by ctw), from five
// table entries per thread.
// PB: one base per pass, its powers formed in the pass (as in cme_lean.hpp):
// 48 fewer registers for the FP64 kernel, which then does not spill.
template <int N, int E, int V, bool PB, typename Real> struct StreamTw {
  using WP = WavePlan<N, E, V, 0>;
  cx<Real> sub[PB ? WP::Sub::P : WP::Sub::NTW];
  cx<Real> bx;     // w^{n1}
  cx<Real> cy[V];  // w^{l (w V + v)}
  cx<Real> dy[V];  // w^{64 (w V + v)}
};

template <int N, int E, int V, bool PB, typename Real>
__device__ __forceinline__ void load_stream_twiddles(StreamTw<N, E, V, PB, Real> &tw,
                                                     const cx<Real> *__restrict__ tab, int w,
                                                     int l) {
  using WP = WavePlan<N, E, V, 0>;
  using PL = typename WP::Sub;
  static_assert(WP::Q == 1, "one cross-wave element per slot");
  if constexpr (PB) {
    // base of pass p: w_N1^{k STRIDE}, k = l mod NS_p (the sub-transform
    // table is every WV-th entry of the length-N one)
    sfor<1, PL::P>([&](auto pi) {
      constexpr int p = decltype(pi)::value;
      constexpr int R = PL::radix(p), NSp = PL::ns(p);
      static_assert(PL::qd(p) == 1, "one twiddle set per pass");
      constexpr int STRIDE = WP::N1 / (NSp * R);
      tw.sub[p] = tab[(l & (NSp - 1)) * STRIDE * WP::WV];
    });
  } else {
    load_twiddles<WP::N1, WP::ES, WP::WV>(tw.sub, tab, l);
  }
  tw.bx = tab[l + 64 * w];
  sfor<0, V>([&](auto vi) {
    constexpr int vv = decltype(vi)::value;
    tw.cy[vv] = tab[(l * (w * V + vv)) & (N - 1)];
    tw.dy[vv] = tab[(64 * (w * V + vv)) & (N - 1)];
  });
}

// fft_wave_multi (cme_fft.hpp) with the twiddles of each pass formed from
// its base: V independent wave-local transforms of length N1 = 64 ES in the
// regions reg + v LB1.
template <int N1, int ES, int V, int S, int PS, typename Real>
__device__ __forceinline__ void stream_wave_multi(cx<Real> (&v)[V * ES], cx<Real> *reg,
                                                  const cx<Real> (&tb)[(FftPlan<N1, ES>::P)],
                                                  int l) {
  using PL = FftPlan<N1, ES>;
  constexpr int T = 64;
  constexpr int LB1 = LdsLen<N1, PS>::value;
  sfor<0, PL::P>([&](auto pi) {
    constexpr int p = decltype(pi)::value;
    constexpr int R = PL::radix(p), NSp = PL::ns(p);
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
    cx<Real> t[R];
    if constexpr (NSp > 1) pow_fill<R>(t, tb[p]);
    sfor<0, V>([&](auto vi) {
      constexpr int vv = decltype(vi)::value;
      sfor<0, Qb>([&](auto qi) {
        constexpr int q = decltype(qi)::value;
        cx<Real> z[R];
        sfor<0, R>([&](auto ri) {
          z[decltype(ri)::value] = v[vv * ES + q + decltype(ri)::value * Qb];
        });
        if constexpr (NSp > 1) {
          sfor<1, R>([&](auto ri) {
            constexpr int r = decltype(ri)::value;
            z[r] = ctw<S>(z[r], t[r]);
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

template <int N1, int ES, int V, int S, int PS, int NT, typename Real>
__device__ __forceinline__ void stream_sub(cx<Real> (&v)[V * ES], cx<Real> *reg,
                                           const cx<Real> (&tw)[NT], int l) {
  if constexpr (NT == FftPlan<N1, ES>::P && NT != FftPlan<N1, ES>::NTW)
    stream_wave_multi<N1, ES, V, S, PS>(v, reg, tw, l);
  else
    fft_wave_multi<N1, ES, V, S, PS>(v, reg, tw, l);
}

template <int N, int E, int V, int S, int PS, bool PRE, bool PB, typename Real>
__device__ __forceinline__ void stream_fwdpath(cx<Real> (&v)[E], cx<Real> *X,
                                               const StreamTw<N, E, V, PB, Real> &tw, int w,
                                               int l) {
  using WP = WavePlan<N, E, V, 0>;
  constexpr int LB1 = LdsLen<WP::N1, PS>::value;
  constexpr int WV = WP::WV, ES = WP::ES;
  if constexpr (PRE) cross_sync<WP::W>();
  {
    cx<Real> z[WV];
    sfor<0, WV>([&](auto ri) { z[decltype(ri)::value] = v[decltype(ri)::value]; });
    dft_reg<WV, S>(z);
    cx<Real> t[WV];
    pow_fill<WV>(t, tw.bx);
    const int n1 = l + 64 * w;
    sfor<0, WV>([&](auto ri) {
      constexpr int r = decltype(ri)::value;
      X[r * LB1 + lpad<PS>(n1)] = r == 0 ? z[0] : ctw<S>(z[r], t[r]);
    });
  }
  cross_sync<WP::W>();
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    constexpr int vv = m / ES, j = m % ES;
    v[m] = X[(w * V + vv) * LB1 + lpad<PS>(l + 64 * j)];
  });
  stream_sub<WP::N1, ES, V, S, PS>(v, X + w * V * LB1, tw.sub, l);
}

template <int N, int E, int V, int S, int PS, bool PB, typename Real>
__device__ __forceinline__ void stream_backpath(cx<Real> (&v)[E], cx<Real> *X, cx<Real> *Y,
                                                const StreamTw<N, E, V, PB, Real> &tw, int w,
                                                int l) {
  using WP = WavePlan<N, E, V, 0>;
  constexpr int LB1 = LdsLen<WP::N1, PS>::value;
  constexpr int WV = WP::WV, ES = WP::ES;
  stream_sub<WP::N1, ES, V, S, PS>(v, X + w * V * LB1, tw.sub, l);
  if (Y == X) wave_sync();  // own regions: the transform's last reads come first
  sfor<0, V>([&](auto vi) {
    constexpr int vv = decltype(vi)::value;
    cx<Real> dp[ES];
    pow_fill<ES>(dp, tw.dy[vv]);
    sfor<0, ES>([&](auto ji) {
      constexpr int j = decltype(ji)::value;
      constexpr int m = vv * ES + j;
      const cx<Real> t = j == 0 ? tw.cy[vv] : cmul(tw.cy[vv], dp[j]);
      Y[(w * V + vv) * LB1 + lpad<PS>(l + 64 * j)] = ctw<S>(v[m], t);
    });
  });
  cross_sync<WP::W>();
  const int n1 = l + 64 * w;
  cx<Real> z[WV];
  sfor<0, WV>([&](auto ri) {
    constexpr int r = decltype(ri)::value;
    z[r] = Y[r * LB1 + lpad<PS>(n1)];
  });
  dft_reg<WV, S>(z);
  sfor<0, WV>([&](auto ri) { v[decltype(ri)::value] = z[decltype(ri)::value]; });
}

// N = 8192 as 16 x 512 on alternate lanes (IL).  Thread c = 64 w + l holds
// modes c + 512 m, as in the two-level layout, so the stage arithmetic is
// unchanged.  The inverse path takes the 16-point DFT over the thread's
// slots, twiddles w^(c k1), and writes region k1 at position c; after the
// barrier wave w runs the 512-point sub-transforms of regions 2 w and
// 2 w + 1 on alternate lanes (lane = 2 t + s), thread t holding positions
// t + 32 m of one of them: radix 16, one exchange through its region, radix
// 16, then an exchange that only trades register bit 0 for t bit 4 (lane
// bit 5: one v_permlane32_swap stage and a renaming of slots), radix 2.
// Against the two-level layout (two 512-point sub-transforms per wave at
// eight modes per thread, two exchanges through LDS each) a transform makes
// one LDS exchange fewer.  The forward path is the mirror image.
template <typename Real> struct S16 {
  static constexpr int N = 8192, E = 16;
  // region length: 512 positions with one pad element every 16 (544), plus
  // an offset that starts the regions of alternate lanes 64 bytes apart
  // modulo 128 (regions 128 bytes apart share the LDS banks)
  static constexpr int RL = 544 + (sizeof(Real) == 8 ? 4 : 8);
};

// w^c for the cross twiddles (powers formed on use), the pass-1 base
// exp(-2 pi i (t mod 16) / 256) and the pass-2 base exp(-2 pi i t / 512)
template <typename Real> struct S16Tw {
  cx<Real> bx, b1, b2;
};
template <typename Real>
__device__ __forceinline__ void load_s16_twiddles(S16Tw<Real> &tw, const cx<Real> *__restrict__ tab,
                                                  int w, int l) {
  const int t = l >> 1;
  tw.bx = tab[l + 64 * w];
  tw.b1 = tab[32 * (t & 15)];
  tw.b2 = tab[16 * t];
}

template <typename Real>
__device__ __forceinline__ void s16_swap32(double &a, double &b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32));
  b = __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
}
template <typename Real>
__device__ __forceinline__ void s16_swap32(float &a, float &b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a),
                                                  __builtin_bit_cast(unsigned, b), false, false);
  a = __builtin_bit_cast(float, (unsigned)r[0]);
  b = __builtin_bit_cast(float, (unsigned)r[1]);
}

// One 512-point sub-transform of sign S in place in v (slot m: position
// t + 32 m, natural order in and out), its one LDS exchange through the
// region R.
template <int S, typename Real>
__device__ __forceinline__ void s16_sub(cx<Real> (&v)[16], cx<Real> *R, const S16Tw<Real> &tw,
                                        int t) {
  // pass 0: element r goes to position 16 t + r
  dft_reg<16, S>(v);
  wave_sync();  // the region's earlier reads come before these writes
  const int b = lpad<4>(16 * t);
  sfor<0, 16>([&](auto ri) { R[b + decltype(ri)::value] = v[decltype(ri)::value]; });
  wave_sync();
  sfor<0, 16>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    v[m] = R[lpad<4>(t + 32 * m)];
  });
  // pass 1 (NS = 16): element r goes to position 256 (t >> 4) + 16 r + (t & 15)
  {
    cx<Real> tp[16];
    pow_fill<16>(tp, tw.b1);
    sfor<1, 16>([&](auto ri) {
      constexpr int r = decltype(ri)::value;
      v[r] = ctw<S>(v[r], tp[r]);
    });
  }
  dft_reg<16, S>(v);
  // pass 2 needs position t' + 32 m in slot m: the source thread agrees with
  // t' in bits 0-3 and has bit 4 = m >> 3; the element is r = 2 (m & 7) +
  // (t' >> 4).  Swapping the odd registers of the lower half-wave with the
  // even ones of the upper half trades register bit 0 for t bit 4; slot m is
  // then register 2 (m & 7) + (m >> 3).
  sfor<0, 8>([&](auto ki) {
    constexpr int k = 2 * decltype(ki)::value;
    s16_swap32<Real>(v[k].re, v[k + 1].re);
    s16_swap32<Real>(v[k].im, v[k + 1].im);
  });
  {
    cx<Real> u[16];
    sfor<0, 16>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      u[m] = v[2 * (m & 7) + (m >> 3)];
    });
    sfor<0, 16>([&](auto mi) { v[decltype(mi)::value] = u[decltype(mi)::value]; });
  }
  // pass 2 (NS = 256): butterfly q on slots q and q + 8, twiddle
  // exp(-2 pi i (t + 32 q) / 512) = b2 exp(-2 pi i q / 16)
  sfor<0, 8>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    cx<Real> x = ctw<S>(v[q + 8], tw.b2);
    if constexpr (q > 0) x = twc<S, q, 16>(x);
    const cx<Real> a = v[q];
    v[q] = cadd(a, x);
    v[q + 8] = csub(a, x);
  });
}

// Inverse path (mode order in, sub-transform order out).  PRE: barrier first
// (one exchange buffer: the previous forward path's gathers).
template <int S, bool PRE, typename Real>
__device__ __forceinline__ void s16_inv(cx<Real> (&v)[16], cx<Real> *X, const S16Tw<Real> &tw,
                                        int w, int l) {
  constexpr int RL = S16<Real>::RL;
  if constexpr (PRE) cross_sync<8>();
  dft_reg<16, S>(v);
  {
    cx<Real> tp[16];
    pow_fill<16>(tp, tw.bx);
    const int o = lpad<4>(l + 64 * w);
    sfor<0, 16>([&](auto ki) {
      constexpr int k1 = decltype(ki)::value;
      X[k1 * RL + o] = k1 == 0 ? v[0] : ctw<S>(v[k1], tp[k1]);
    });
  }
  cross_sync<8>();
  const int t = l >> 1;
  cx<Real> *R = X + (2 * w + (l & 1)) * RL;
  sfor<0, 16>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    v[m] = R[lpad<4>(t + 32 * m)];
  });
  s16_sub<S>(v, R, tw, t);
}

// Forward path (sub-transform order in, mode order out); the sub-transform
// runs in X (own region), the exchange goes through Y.
template <int S, typename Real>
__device__ __forceinline__ void s16_fwd(cx<Real> (&v)[16], cx<Real> *X, cx<Real> *Y,
                                        const S16Tw<Real> &tw, int w, int l) {
  constexpr int RL = S16<Real>::RL;
  const int t = l >> 1, reg = (2 * w + (l & 1)) * RL;
  s16_sub<S>(v, X + reg, tw, t);
  if (Y == X) wave_sync();  // own region: the sub-transform's last reads come first
  sfor<0, 16>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    Y[reg + lpad<4>(t + 32 * m)] = v[m];
  });
  cross_sync<8>();
  cx<Real> tp[16];
  pow_fill<16>(tp, tw.bx);
  const int o = lpad<4>(l + 64 * w);
  sfor<0, 16>([&](auto ki) {
    constexpr int k1 = decltype(ki)::value;
    v[k1] = k1 == 0 ? Y[o] : ctw<S>(Y[k1 * RL + o], tp[k1]);
  });
  dft_reg<16, S>(v);
}

// Raw buffer accesses: one 32-bit per-lane offset register plus a constant
// per-slot offset in a scalar register, so that the addresses of the E slots
// a thread owns cost no 64-bit registers (hoisted out of the time loop, 64-bit
// pointers for every slot and array would crowd out the transform).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int vo, int so) {
  if constexpr (sizeof(T) == 16)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
  else if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store(T x, __amdgpu_buffer_rsrc_t r, int vo, int so) {
  if constexpr (sizeof(T) == 16) {
    using V4 = __attribute__((ext_vector_type(4))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, x), r, vo, so, 0);
  } else {
    using V2 = __attribute__((ext_vector_type(2))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, vo, so, 0);
  }
}

// D: prefetch distance of the stage arithmetic (slots whose operands are in
// flight while one slot is computed).
// YR: the state y held in registers for the whole launch (FP32, whose
// registers have the room) instead of read from the caller's array at every
// stage; it is written back after the last step.  OR: omega' held in
// registers for the launch (16 values per thread) instead of read at every
// stage, and in FP32 -kappa/2 as well.
// IL: the 16 x 512 layout on alternate lanes (S16)
template <typename Real, int N, int E, int V, int PS, int D, bool PB, bool YR, bool OR,
          bool IL = false>
__global__ void __launch_bounds__((WaveShape<Real, N, E, V, PS, 0>::THREADS))
    rk4_stream(RunArgs a) {
  constexpr int TP = 0;
  static_assert(D >= 1, "prefetch distance");
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  using WP = WavePlan<N, E, V, TP>;
  static_assert(WP::W > 1 && SH::IPB == 1, "one instance per workgroup");
  static_assert(!IL || (N == S16<Real>::N && E == S16<Real>::E && V == 2 && WP::W == 8),
                "the 16 x 512 layout is N = 8192 at 16 modes per thread");
  static_assert(!IL || 16 * S16<Real>::RL <= SH::WV * SH::LB1, "16 x 512 regions in one buffer");
  __shared__ cx<Real> lds[SH::PER_INST];

  const int lane = (int)threadIdx.x & 63;
  const int w = (int)threadIdx.x >> 6;
  const int slot = (int)blockIdx.x;
  const int id = a.order[slot];
  const DevInst d = a.inst[id];
  cx<Real> *X = lds;
  cx<Real> *Y = SH::TWO ? X + SH::WV * SH::LB1 : X;  // FP32: a second exchange buffer fits
  cx<Real> *A = reinterpret_cast<cx<Real> *>(a.A) + d.offset;
  constexpr int CB = (int)sizeof(cx<Real>);
  const __amdgpu_buffer_rsrc_t rA = buf_rsrc(A, N * CB);
  cx<Real> *work = reinterpret_cast<cx<Real> *>(a.work) + (int64_t)slot * 2 * N;
  const __amdgpu_buffer_rsrc_t rW1 = buf_rsrc(work, N * CB);
  const __amdgpu_buffer_rsrc_t rW2 = buf_rsrc(work + N, N * CB);
  const __amdgpu_buffer_rsrc_t rK = buf_rsrc(a.kappa + d.offset, N * 8);
  const __amdgpu_buffer_rsrc_t rW = buf_rsrc(a.omega + d.offset, N * 8);
  // slot m of this thread holds mode i0 + N1 m (Q = 1)
  static_assert(WP::Q == 1, "one cross-wave element per slot");
  const int i0 = lane + 64 * w;

  std::conditional_t<IL, S16Tw<Real>, StreamTw<N, E, V, PB, Real>> tw;
  if constexpr (IL)
    load_s16_twiddles(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);
  else
    load_stream_twiddles<N, E, V>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  cx<Real> v[E];
  cx<Real> yr[YR ? E : 1];
  double omr[OR ? E : 1];
  // FP32 with OR: -kappa/2 too, already rounded to the stage arithmetic's precision
  constexpr bool LRR = OR && sizeof(Real) == 4;
  Real lrr[LRR ? E : 1];
  const bool pump_owner = (w == 0 && lane == 0);  // mode N/2 sits in slot E/2 there
  const Real gn = (Real)d.g0n;
  const cx<Real> pump = {(Real)d.pump_re, (Real)d.pump_im};
  const double h = a.h;
  const Real h2 = (Real)(0.5 * h), h1 = (Real)h, h3 = (Real)(h / 3.0), h6 = (Real)(h / 6.0);
  cx<Real> *ckpt = reinterpret_cast<cx<Real> *>(a.ckpt);
  int32_t to_ckpt = a.ckpt_every;
  int64_t ckpt_slot = 0;
  bool bad = false;

  // KU: kappa the same for every mode of the instance (not read per stage)
  auto run = [&](auto ku) {
    constexpr bool KU = decltype(ku)::value;
    const Real lr0 = (Real)(-0.5 * d.kappa0);
    // the first stage input: the state
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      v[m] = buf_load<cx<Real>>(rA, CB * i0, CB * WP::N1 * m);
      if constexpr (YR) yr[m] = v[m];
      if constexpr (OR) omr[m] = buf_load<double>(rW, 8 * i0, 8 * WP::N1 * m);
      if constexpr (LRR) lrr[m] = (Real)(-0.5 * buf_load<double>(rK, 8 * i0, 8 * WP::N1 * m));
    });
    for (int64_t n = 0; n < a.n_steps; ++n) {
      const double t0 = (double)(a.step0 + n) * h;
      sfor<0, 4>([&](auto si) {
        constexpr int s = decltype(si)::value;
        // the stage input u_s is in v (the transform overwrites it; the stage
        // arithmetic reads it back from the state, k_1 or U)
          const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, t0 + kCw[s] * h);
        // with one buffer the forward path fences the previous back path's reads
        if constexpr (IL) s16_inv<+1, !SH::TWO>(v, X, tw, w, lane);
        else stream_fwdpath<N, E, V, +1, PS, !SH::TWO, PB>(v, X, tw, w, lane);
        sfor<0, E>([&](auto mi) {
          constexpr int m = decltype(mi)::value;
          const Real p = v[m].re * v[m].re + v[m].im * v[m].im;
          v[m] = {p * v[m].re, p * v[m].im};
        });
        if constexpr (IL) s16_fwd<-1>(v, X, Y, tw, w, lane);
        else stream_backpath<N, E, V, -1, PS, PB>(v, X, Y, tw, w, lane);
        // Stage arithmetic, slot by slot, with the loads of slot m + D issued
        // before slot m is computed (a ring of D slots of operands), so that
        // the global-memory latency is paid about once per stage.  v[m] is
        // consumed (N K) and refilled with the next stage input.
        struct Ops {
          cx<Real> y, w1, w2;
          double kap, om;
        };
        Ops ring[D];
        __builtin_amdgcn_sched_barrier(0);  // no operand load above the transforms
        auto fetch = [&](auto mi) {
          constexpr int m = decltype(mi)::value;
          constexpr int off = CB * WP::N1 * m;  // slot m: mode i0 + N1 m
          Ops &o = ring[m % D];
          // slot contents: W1 = k_1 (after s = 0) or P (after s = 2), W2 = k_2
          // (after s = 1) or u_4 (after s = 2); y is the caller's state
          if constexpr (s < 3 && !YR) o.y = buf_load<cx<Real>>(rA, CB * i0, off);
          if constexpr (!KU && !LRR) o.kap = buf_load<double>(rK, 8 * i0, 8 * WP::N1 * m);
          if constexpr (!OR) o.om = buf_load<double>(rW, 8 * i0, 8 * WP::N1 * m);
          if constexpr (s > 0) o.w1 = buf_load<cx<Real>>(rW1, CB * i0, off);
          if constexpr (s > 1) o.w2 = buf_load<cx<Real>>(rW2, CB * i0, off);
        };
        sfor<0, (D < E ? D : E)>(fetch);
        sfor<0, E>([&](auto mi) {
          constexpr int m = decltype(mi)::value;
          __builtin_amdgcn_sched_barrier(0);
          Ops o = ring[m % D];
          if constexpr (YR) o.y = yr[m];
          if constexpr (OR) o.om = omr[m];
          if constexpr (m + D < E) fetch(ic<m + D>{});
          constexpr int off = CB * WP::N1 * m;
          Real lr = lr0;
          if constexpr (!KU && LRR) lr = lrr[m];
          if constexpr (!KU && !LRR) lr = (Real)(-0.5 * o.kap);
          const Real det = (Real)(o.om - sig);
          // the stage input: y, y + h/2 k_1, y + h/2 k_2, u_4
          cx<Real> u = o.y;
          if constexpr (s == 1) u = {o.y.re + h2 * o.w1.re, o.y.im + h2 * o.w1.im};
          if constexpr (s == 2) u = {o.y.re + h2 * o.w2.re, o.y.im + h2 * o.w2.im};
          if constexpr (s == 3) u = o.w2;
          cx<Real> k = {lr * u.re - det * u.im - gn * v[m].im, lr * u.im + det * u.re + gn * v[m].re};
          if constexpr (m == E / 2) {
            if (pump_owner) k = cadd(k, pump);
          }
          if constexpr (s == 0) {  // W1 = k_1
            buf_store(k, rW1, CB * i0, off);
            v[m] = {u.re + h2 * k.re, u.im + h2 * k.im};
          } else if constexpr (s == 1) {  // W2 = k_2
            buf_store(k, rW2, CB * i0, off);
            v[m] = {o.y.re + h2 * k.re, o.y.im + h2 * k.im};
          } else if constexpr (s == 2) {  // W1 = P = y + h/6 k_1 + h/3 k_2 + h/3 k_3, W2 = u_4
            const cx<Real> p1 = {o.y.re + h6 * o.w1.re, o.y.im + h6 * o.w1.im};
            const cx<Real> p2 = {p1.re + h3 * o.w2.re, p1.im + h3 * o.w2.im};
            buf_store(cx<Real>{p2.re + h3 * k.re, p2.im + h3 * k.im}, rW1, CB * i0, off);
            v[m] = {o.y.re + h1 * k.re, o.y.im + h1 * k.im};
            buf_store(v[m], rW2, CB * i0, off);
          } else {
            v[m] = {o.w1.re + h6 * k.re, o.w1.im + h6 * k.im};
            if constexpr (YR) {
              yr[m] = v[m];
              if (n + 1 == a.n_steps) buf_store(v[m], rA, CB * i0, off);
            } else {
              buf_store(v[m], rA, CB * i0, off);
            }
            if (ckpt != nullptr && to_ckpt == 1)
              ckpt[ckpt_slot * a.total + d.offset + i0 + WP::N1 * m] = v[m];
            if (n + 1 == a.n_steps) bad |= !(isfinite(v[m].re) && isfinite(v[m].im));
          }
        });
        __builtin_amdgcn_sched_barrier(0);
      });
      if (ckpt != nullptr && --to_ckpt == 0) {
        to_ckpt = a.ckpt_every;
        ++ckpt_slot;
      }
    }
  };
  if (d.kappa_uniform) run(std::true_type{});
  else run(std::false_type{});
  if (bad) atomicOr(&a.flags[id], 1);
}

template <typename Real, int N, int E, int V, int PS, int D, bool PB, bool YR, bool OR, bool IL>
hipError_t launch_stream_fwd(const RunArgs &a, hipStream_t st) {
  using SH = WaveShape<Real, N, E, V, PS, 0>;
  if (a.stages != nullptr || a.work == nullptr) return hipErrorInvalidValue;
  if (a.count <= 0 || a.n_steps <= 0) return hipSuccess;
  hipLaunchKernelGGL((rk4_stream<Real, N, E, V, PS, D, PB, YR, OR, IL>), dim3(a.count),
                     dim3(SH::THREADS), 0, st, a);
  return hipGetLastError();
}

// kind 13; two complex values of class workspace per mode (k_1, then the
// partial update; k_2, then u_4); no reverse sweep (the adjoint uses another
// variant of the size).  The tuning field holds D, plus 16 with PB, 32 with YR,
// 64 with OR and 128 with IL.
template <typename Real, int N, int E, int V, int PS, int D, bool PB, bool YR = false,
          bool OR = false, bool IL = false>
constexpr Variant stream_variant() {
  using SH = WaveShape<Real, N, E, V, PS, 0>;
  return Variant{std::is_same<Real, double>::value ? 0 : 1, N, E, V, PS,
                 D + 16 * PB + 32 * YR + 64 * OR + 128 * IL, 13, SH::IPB, SH::THREADS,
                 SH::LDS_BYTES, &launch_stream_fwd<Real, N, E, V, PS, D, PB, YR, OR, IL>, nullptr,
                 2};
}

// The interaction-picture RK4 of cme_rk4ip.hip (its step is written out
// there) on the same transforms and layout.  The per-mode factor
// D = exp((-kappa/2 + i omega') h/2) is formed once per launch (FP64, then
// rounded) into the third workspace vector; the detuning phase is one scalar
// per half step.  Per stage, from the stage's N(u) = q:
//   stage 1: yI = P1 y, k1 = P1 q   -> the state array holds yI, W1 = k1
//   stage 2: k2 = q                 -> W2 = k2
//   stage 3: k3 = q                 -> W1 = Q = yI + h/6 (k1 + 2 k2 + 2 k3),
//                                      next input P2 (yI + h k3)
//   stage 4: y' = P2 Q + h/6 q      -> the state array
// (P1 = D exp(-i int_t0^tm sigma), P2 = D exp(-i int_tm^t1 sigma)): 224 bytes
// of global traffic per mode and step in FP64.
template <typename Real, int N, int E, int V, int PS, int D, bool IL = false>
__global__ void __launch_bounds__((WaveShape<Real, N, E, V, PS, 0>::THREADS))
    rk4ip_stream(RunArgs a) {
  constexpr int TP = 0;
  static_assert(D >= 1, "prefetch distance");
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  using WP = WavePlan<N, E, V, TP>;
  static_assert(WP::W > 1 && SH::IPB == 1, "one instance per workgroup");
  static_assert(WP::Q == 1, "one cross-wave element per slot");
  __shared__ cx<Real> lds[SH::PER_INST];

  const int lane = (int)threadIdx.x & 63;
  const int w = (int)threadIdx.x >> 6;
  const int slot = (int)blockIdx.x;
  const int id = a.order[slot];
  const DevInst d = a.inst[id];
  cx<Real> *X = lds;
  cx<Real> *Y = SH::TWO ? X + SH::WV * SH::LB1 : X;
  cx<Real> *A = reinterpret_cast<cx<Real> *>(a.A) + d.offset;
  constexpr int CB = (int)sizeof(cx<Real>);
  const __amdgpu_buffer_rsrc_t rA = buf_rsrc(A, N * CB);
  cx<Real> *work = reinterpret_cast<cx<Real> *>(a.work) + (int64_t)slot * 3 * N;
  const __amdgpu_buffer_rsrc_t rW1 = buf_rsrc(work, N * CB);
  const __amdgpu_buffer_rsrc_t rW2 = buf_rsrc(work + N, N * CB);
  const __amdgpu_buffer_rsrc_t rD = buf_rsrc(work + 2 * N, N * CB);
  const int i0 = lane + 64 * w;  // slot m: mode i0 + N1 m

  static_assert(!IL || (N == S16<Real>::N && E == S16<Real>::E && V == 2 && WP::W == 8),
                "the 16 x 512 layout is N = 8192 at 16 modes per thread");
  std::conditional_t<IL, S16Tw<Real>, StreamTw<N, E, V, true, Real>> tw;
  if constexpr (IL)
    load_s16_twiddles(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);
  else
    load_stream_twiddles<N, E, V>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);

  const double h = a.h;
  cx<Real> v[E];
  {
    const __amdgpu_buffer_rsrc_t rK = buf_rsrc(a.kappa + d.offset, N * 8);
    const __amdgpu_buffer_rsrc_t rO = buf_rsrc(a.omega + d.offset, N * 8);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const double mag = exp(-0.25 * h * buf_load<double>(rK, 8 * i0, 8 * WP::N1 * m));
      double sn, cs;
      sincos(0.5 * h * buf_load<double>(rO, 8 * i0, 8 * WP::N1 * m), &sn, &cs);
      buf_store(cx<Real>{(Real)(mag * cs), (Real)(mag * sn)}, rD, CB * i0, CB * WP::N1 * m);
      v[m] = buf_load<cx<Real>>(rA, CB * i0, CB * WP::N1 * m);
    });
  }
  const bool pump_owner = (w == 0 && lane == 0);  // mode N/2 sits in slot E/2 there
  const Real gn = (Real)d.g0n;
  const cx<Real> pump = {(Real)d.pump_re, (Real)d.pump_im};
  const Real hh = (Real)(0.5 * h), hf = (Real)h, h6 = (Real)(h / 6.0), two = (Real)2;
  cx<Real> *ckpt = reinterpret_cast<cx<Real> *>(a.ckpt);
  int32_t to_ckpt = a.ckpt_every;
  int64_t ckpt_slot = 0;
  bool bad = false;

  for (int64_t n = 0; n < a.n_steps; ++n) {
    const double t0 = (double)(a.step0 + n) * h, tm = t0 + 0.5 * h, t1 = t0 + h;
    double sn, cs;
    sincos(-sigma_integral(d.sigma0, d.sigma1, d.tau_ramp, t0, tm), &sn, &cs);
    const cx<Real> c1 = {(Real)cs, (Real)sn};
    sincos(-sigma_integral(d.sigma0, d.sigma1, d.tau_ramp, tm, t1), &sn, &cs);
    const cx<Real> c2 = {(Real)cs, (Real)sn};
    sfor<0, 4>([&](auto si) {
      constexpr int s = decltype(si)::value;
      if constexpr (IL) s16_inv<+1, !SH::TWO>(v, X, tw, w, lane);
      else stream_fwdpath<N, E, V, +1, PS, !SH::TWO, true>(v, X, tw, w, lane);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const Real p = v[m].re * v[m].re + v[m].im * v[m].im;
        v[m] = {p * v[m].re, p * v[m].im};
      });
      if constexpr (IL) s16_fwd<-1>(v, X, Y, tw, w, lane);
      else stream_backpath<N, E, V, -1, PS, true>(v, X, Y, tw, w, lane);
      struct Ops {
        cx<Real> y, w1, w2, dm;
      };
      Ops ring[D];
      __builtin_amdgcn_sched_barrier(0);  // no operand load above the transforms
      auto fetch = [&](auto mi) {
        constexpr int m = decltype(mi)::value;
        constexpr int off = CB * WP::N1 * m;
        Ops &o = ring[m % D];
        if constexpr (s < 3) o.y = buf_load<cx<Real>>(rA, CB * i0, off);  // y, then yI
        if constexpr (s != 1) o.dm = buf_load<cx<Real>>(rD, CB * i0, off);
        if constexpr (s >= 2) o.w1 = buf_load<cx<Real>>(rW1, CB * i0, off);
        if constexpr (s == 2) o.w2 = buf_load<cx<Real>>(rW2, CB * i0, off);
      };
      sfor<0, (D < E ? D : E)>(fetch);
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        __builtin_amdgcn_sched_barrier(0);
        const Ops o = ring[m % D];
        if constexpr (m + D < E) fetch(ic<m + D>{});
        constexpr int off = CB * WP::N1 * m;
        cx<Real> q = {-gn * v[m].im, gn * v[m].re};  // N(u) = i (g0/N) N K + pump
        if constexpr (m == E / 2) {
          if (pump_owner) q = cadd(q, pump);
        }
        if constexpr (s == 0) {
          const cx<Real> p1 = cmul(o.dm, c1);
          const cx<Real> k1 = cmul(p1, q), yi = cmul(p1, o.y);
          buf_store(yi, rA, CB * i0, off);
          buf_store(k1, rW1, CB * i0, off);
          v[m] = {yi.re + hh * k1.re, yi.im + hh * k1.im};
        } else if constexpr (s == 1) {
          buf_store(q, rW2, CB * i0, off);
          v[m] = {o.y.re + hh * q.re, o.y.im + hh * q.im};
        } else if constexpr (s == 2) {
          cx<Real> acc = {o.w1.re + two * o.w2.re, o.w1.im + two * o.w2.im};
          acc = {acc.re + two * q.re, acc.im + two * q.im};
          buf_store(cx<Real>{o.y.re + h6 * acc.re, o.y.im + h6 * acc.im}, rW1, CB * i0, off);
          v[m] = cmul(cmul(o.dm, c2), cx<Real>{o.y.re + hf * q.re, o.y.im + hf * q.im});
        } else {
          const cx<Real> z = cmul(cmul(o.dm, c2), o.w1);
          v[m] = {z.re + h6 * q.re, z.im + h6 * q.im};
          buf_store(v[m], rA, CB * i0, off);
          if (ckpt != nullptr && to_ckpt == 1)
            ckpt[ckpt_slot * a.total + d.offset + i0 + WP::N1 * m] = v[m];
          if (n + 1 == a.n_steps) bad |= !(isfinite(v[m].re) && isfinite(v[m].im));
        }
      });
      __builtin_amdgcn_sched_barrier(0);
    });
    if (ckpt != nullptr && --to_ckpt == 0) {
      to_ckpt = a.ckpt_every;
      ++ckpt_slot;
    }
  }
  if (bad) atomicOr(&a.flags[id], 1);
}

template <typename Real, int N, int E, int V, int PS, int D, bool IL = false>
hipError_t launch_stream_ip_fwd(const RunArgs &a, hipStream_t st) {
  using SH = WaveShape<Real, N, E, V, PS, 0>;
  if (a.stages != nullptr || a.work == nullptr) return hipErrorInvalidValue;
  if (a.count <= 0 || a.n_steps <= 0) return hipSuccess;
  hipLaunchKernelGGL((rk4ip_stream<Real, N, E, V, PS, D, IL>), dim3(a.count), dim3(SH::THREADS), 0,
                     st, a);
  return hipGetLastError();
}

// kind 14; three complex values of class workspace per mode (W1, W2 and the
// per-mode factor D); no reverse sweep.  The tuning field holds D, plus 128
// with IL.
template <typename Real, int N, int E, int V, int PS, int D, bool IL = false>
constexpr Variant stream_ip_variant() {
  using SH = WaveShape<Real, N, E, V, PS, 0>;
  return Variant{std::is_same<Real, double>::value ? 0 : 1, N, E, V, PS, D + 128 * IL, 14,
                 SH::IPB, SH::THREADS, SH::LDS_BYTES,
                 &launch_stream_ip_fwd<Real, N, E, V, PS, D, IL>, nullptr, 3};
}

// The first of each precision is the default: the 16 x 512 layout (IL).
// Measured, us per step for 1 / 16 / 128 instances (per-mode kappa): FP64 IL
// D = 2 47.2 / 47.1 / 54.0, IL D = 1 47.6 / 47.5 / 55.0, against the
// two-level OR PB D = 1 52.3 / 52.7 / 57.6; FP32 IL 27.3 / 27.5 (100) / 27.4
// against 31.3 / 31.4 / 31.5; interaction picture FP64 IL 44.3 / 48.6 (64) /
// 52.6 against 50.0 / 53.5 / 55.8, FP32 IL 32.0 (16) / 32.9 (100) / 33.2.
// FP64 IL D = 3 ran 1-2% faster than D = 2 (48.4 against 49.3 at 128
// instances, uniform kappa) but spills 12 bytes per lane (D = 4: 32), and
// FP32 IL D = 2 or 8 changed nothing; none of them is built.
// The two-level figures, us per step for 1,
// 100 and 128 instances with per-mode kappa (kappa the same for every mode):
// FP64 OR PB D = 1 52.1 / 56.7 / 57.8 (49.0 / 53.6 / 55.7; 255 VGPRs, no
// spills), OR PB D = 2 52.1 / 56.3 / 57.1 (48.9 / 53.2 / 54.8; spills 36
// bytes per lane), PB D = 2 55.3 / 59.7 / 61.2 (51.5 / 56.2 / 58.0), PB D = 1
// 54.8 / 60.0 / 61.1 (52.0 / 56.1 / 58.3); with every twiddle power held the
// kernel spills at any D, and the FP64 state does not fit beside the
// transform.  FP32 YR OR PB D = 4 31.3 / 31.8 / 32.9 (31.1 / 32.2 / 32.3),
// YR OR PB D = 2 31.4 / 32.1 / 32.4 (31.3 / 31.9 / 32.7), YR PB D = 4 38.5 /
// 39.2 / 39.9 (34.7 / 35.5 / 36.3), D = 4 41.8 / 42.8 / 43.6 (38.2 / 39.2 /
// 39.7).  The stage arithmetic's global-memory traffic is streamed by one CU
// at about 57 bytes per clock; the transforms alone take about 40 us (FP64).
// Interaction picture (kind 14), us per step for 1 / 16 / 64 / 128
// instances, per-mode kappa: FP64 D = 2 49.9 / 50.4 / 51.6 / 56.4, D = 1
// 50.4 / 50.8 / 53.8 / 58.6 (the staged interaction-picture kernels: 58.5 /
// 63.5 / 78.9 / 96.8; repeated runs move each figure by up to 2 us); FP32
// D = 4 35.9 / 35.9 / 36.1 / 36.4, D = 2 35.9 / 35.9 / 36.1 / 36.9.
static const Variant kStreamVariants[] = {
    stream_variant<double, 8192, 16, 2, 3, 2, true, false, true, true>(),
    stream_variant<double, 8192, 16, 2, 3, 1, true, false, true, true>(),
    stream_variant<float, 8192, 16, 2, 3, 4, true, true, true, true>(),
    stream_variant<double, 8192, 16, 2, 3, 1, true, false, true>(),
    stream_variant<double, 8192, 16, 2, 3, 2, true, false, true>(),
    stream_variant<double, 8192, 16, 2, 3, 2, true>(),
    stream_variant<double, 8192, 16, 2, 3, 1, true>(),
    stream_variant<float, 8192, 16, 2, 3, 4, true, true, true>(),
    stream_variant<float, 8192, 16, 2, 3, 2, true, true, true>(),
    stream_variant<float, 8192, 16, 2, 3, 4, true, true>(),
    stream_variant<float, 8192, 16, 2, 3, 4, false>(),
    stream_ip_variant<double, 8192, 16, 2, 3, 2, true>(),
    stream_ip_variant<double, 8192, 16, 2, 3, 2>(),
    stream_ip_variant<double, 8192, 16, 2, 3, 1>(),
    stream_ip_variant<float, 8192, 16, 2, 3, 4, true>(),
    stream_ip_variant<float, 8192, 16, 2, 3, 4>(),
    stream_ip_variant<float, 8192, 16, 2, 3, 2>(),
};

const Variant *variants_stream(int *count) {
  *count = (int)(sizeof(kStreamVariants) / sizeof(kStreamVariants[0]));
  return kStreamVariants;
}

}  // namespace cme
