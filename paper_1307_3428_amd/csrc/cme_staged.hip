// cme_staged.hip -- the solver for transforms that do not fit one workgroup
// well (N = 8192 ... 65536): four-step transforms whose transpose goes
// through global memory (L2 / MALL / HBM) instead of LDS.  Classic RK4 (FP64
// and FP32, cyclic or padded sum), the interaction-picture RK4, the
// split-step map and the four-wave-mixing sum alone (cme_fwm) run on them;
// the classic RK4 is described here, the others where they are defined.
//
// N = N1 N2; mode index m = m1 + N1 m2 (m1 < N1, m2 < N2); transformed index
// j = j2 + N2 j1.  With w_L = e^{2 pi i / L} and w = w_N, the inverse
// transform of Eq. (4) factors as
//   a_{j2 + N2 j1} = sum_m1 w_N1^{j1 m1} [ w^{j2 m1} sum_m2 u_{m1 + N1 m2} w_N2^{j2 m2} ]
// and the forward transform of b = |a|^2 a as its mirror image
//   N K_{m1 + N1 m2} = sum_j2 w_N2^{-j2 m2} [ w^{-j2 m1} sum_j1 b_{j2 + N2 j1} w_N1^{-j1 m1} ].
// Both bracketed half-transforms are kept in one scratch array S[j2][m1] per
// instance, and a step of the RK4 solver alternates two kernels:
//   column kernel (a team of N2/E threads per m1): finish the forward
//     transform (outer sum over j2) -> N K for the team's N2 modes; form the
//     stage derivative k_s = L_s u_s + i (g0/N) N K + [m = N/2] pump, the RK4
//     combination, the next stage input, and start its inverse transform
//     (inner sum over m2, times w^{j2 m1}) into S;
//   row kernel (a team of N1/E threads per j2): finish the inverse transform
//     (outer sum over m1), cube pointwise, start the forward transform (inner
//     sum over j1, times w^{-j2 m1}) into S.
// A step is 4 x (row, column) launches; a run starts with one column launch
// that only starts the inverse transform of the state.  Two RK4 vectors live
// in a plan-owned workspace next to S (classic RK4: k_1, then the partial
// update; k_2, then u_4; the interaction picture: the accumulated derivative
// and the stage input); the state is read and written in the caller's array.
// Every launch moves each of these arrays at most once, so the path is bound
// by memory traffic.
//
// Each team transforms its column or row with the radix-E Stockham passes of
// cme_fft.hpp in registers, exchanging through a private LDS buffer inside
// one wavefront (no workgroup barrier).
#include <type_traits>

#include "cme_fft.hpp"
#include "cme_internal.hpp"

namespace cme {

namespace {

// Real: the precision of the state, the transforms, the stored arrays and
// the stage arithmetic (FP64, or FP32 for classic RK4 and RK4IP).
template <typename Real> struct StagedArgsT {
  const DevInst *inst;
  const int32_t *order;
  int32_t count;
  int32_t tail;            // column kernel, last stage of the run: no next transform
  cx<Real> *A;             // caller's packed state
  const double *kappa;
  const double *omega;
  const cx<Real> *tab;     // exp(-2 pi i k / N), k < N
  cx<Real> *work;          // per class slot: S and the two RK4 vectors (3 N each)
  double h;
  double t0;               // time at the start of the step
  cx<Real> *ckpt;          // checkpoint row for this step (packed like A) or null
  int32_t *flags;
};
using StagedArgs = StagedArgsT<double>;

template <typename Real> __device__ __forceinline__ cx<Real> dn(cx<double> z) {
  return {(Real)z.re, (Real)z.im};
}

constexpr int kPS = 3;  // one LDS pad element every 8

// Cross twiddles tw[m] = w_N^{-a (b + m T)} (tab[k] = w_N^{-k}) for the E
// elements of a thread, as w^{-a b} w^{-a T m}: the second factor is the same
// for every lane of a team, so a wavefront gathers a few distinct table
// entries instead of one per lane and element; one complex product each.
template <int N, int E, int T, typename Real>
__device__ __forceinline__ void cross_tw(cx<Real> (&tw)[E], const cx<Real> *tab, int a, int b) {
  const cx<Real> base = tab[(a * b) & (N - 1)];
  tw[0] = base;
  sfor<1, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    tw[m] = cmul(base, tab[(a * T * m) & (N - 1)]);
  });
}

// RK4 stage nodes
__device__ __forceinline__ constexpr double stage_c(int s) { return s == 0 ? 0.0 : (s == 3 ? 1.0 : 0.5); }

template <int N, int N1, int E, int WPB> struct ColShape {
  static constexpr int N2 = N / N1;
  static constexpr int T = N2 / E;       // threads per column
  static constexpr int CW = 64 / T;      // columns per wavefront
  static constexpr int C = CW * WPB;     // columns per workgroup
  static constexpr int NB = N1 / C;      // workgroups per instance
  static constexpr int LB = LdsLen<N2, kPS>::value + 1;
  static constexpr int LDS_BYTES = WPB * CW * LB * 16;
  static_assert(T >= 1 && T <= 64 && N1 % C == 0, "column shape");
};

template <int N, int N1, int E, int WPB> struct RowShape {
  static constexpr int N2 = N / N1;
  static constexpr int T = N1 / E;       // threads per row
  static constexpr int RW = 64 / T;      // rows per wavefront
  static constexpr int R = RW * WPB;     // rows per workgroup
  static constexpr int NB = N2 / R;      // workgroups per instance
  static constexpr int LB = LdsLen<N1, kPS>::value + 1;
  static constexpr int LDS_BYTES = WPB * RW * LB * 16;
  static_assert(T >= 1 && T <= 64 && N2 % R == 0, "row shape");
};

// IP: the interaction-picture RK4 instead (the linear part exact): per step
// from t0, with P1, P2 = exp((-kappa/2 + i omega') h/2 - i int sigma) over the
// two half steps and N(u) = i (g0/N) N K + pump,
//   stage 1: yI = P1 y -> U, k1 = P1 N(y) -> ACC, next yI + h/2 k1;
//   stage 2: k2 = N(u2), ACC += 2 k2, next yI + h/2 k2;
//   stage 3: k3 = N(u3), ACC += 2 k3, next P2 (yI + h k3);
//   stage 4: k4 = N(u4), y' = P2 (yI + h/6 ACC) + h/6 k4.
// PAD: the alias-free truncated sum (CME_FWM_PADDED): the instance's N/2
// modes sit at transform indices [N/4, 3N/4) (index i <-> mode i - N/4 of
// the caller's state); the derivative is zero outside that band, so the
// other half stays zero and the cyclic sum over the band is the literal one.
// STAGE < 0: start the inverse transform of the state (first launch of a run);
// STAGE = s in 0..3: RK4 stage s + 1 as described above; STAGE = 4: finish
// the forward transform and write the four-wave-mixing sum K = (N K) / N
// (cme_fwm), packed like the state, to a.ckpt.
template <int N, int N1, int E, int WPB, int STAGE, bool IP = false, typename Real = double,
          bool PAD = false>
__global__ void __launch_bounds__(64 * WPB) staged_col(StagedArgsT<Real> a) {
  using SH = ColShape<N, N1, E, WPB>;
  constexpr int N2 = SH::N2, T = SH::T;
  static_assert(!PAD || !IP, "the padded sum steps classic RK4");
  constexpr int Q4 = N / 4;
  auto in_band = [](int i) { return !PAD || (i >= Q4 && i < 3 * Q4); };
  auto phys = [](int i) { return PAD ? i - Q4 : i; };  // index in the caller's state
  __shared__ cx<Real> lds[WPB * SH::CW * SH::LB];
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  const int slot = (int)blockIdx.x / SH::NB, cb = (int)blockIdx.x % SH::NB;
  const int cl = lane % SH::CW, t = lane / SH::CW;
  const int m1 = cb * SH::C + wv * SH::CW + cl;
  const int id = a.order[slot];
  const DevInst d = a.inst[id];
  cx<Real> *A = a.A + d.a_offset;
  cx<Real> *S = a.work + (int64_t)slot * 3 * N;
  cx<Real> *ACC = S + N, *U = S + 2 * N;
  cx<Real> *buf = lds + (wv * SH::CW + cl) * SH::LB;

  cx<Real> tw[FftPlan<N2, E>::NTW];
  load_twiddles<N2, E, N1>(tw, a.tab, t);
  cx<Real> v[E];

  if constexpr (STAGE < 0) {
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const int i = m1 + N1 * (t + m * T);
      v[m] = in_band(i) ? A[phys(i)] : cx<Real>{(Real)0, (Real)0};
    });
  } else {
    // outer sum of the forward transform: v[m] = N K at mode m1 + N1 (t + m T)
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      v[m] = S[(t + m * T) * N1 + m1];
    });
    fft_team<N2, E, -1, kPS, false, 0, SYNC_WAVE>(v, buf, buf, tw, t);
    if constexpr (STAGE == 4) {
      const double inv_n = 1.0 / (double)N;
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const int i = m1 + N1 * (t + m * T);
        if (in_band(i)) a.ckpt[d.a_offset + phys(i)] = dn<Real>({v[m].re * inv_n, v[m].im * inv_n});
      });
      return;
    }
    // The stage arithmetic runs in Real; only the time-dependent coefficients
    // (sigma(t), omega' - sigma, the propagators' phase with the integral of
    // sigma) are formed in FP64 and rounded to Real once per stage.
    const double h = a.h;
    const double *kap = a.kappa + d.offset, *omg = a.omega + d.offset;
    const Real gn = (Real)d.g0n;
    const cx<Real> pump = {(Real)d.pump_re, (Real)d.pump_im};
    bool bad = false;
    if constexpr (IP) {
      // detuning phase of the half step whose propagator this stage applies
      const double tm = a.t0 + 0.5 * h;
      const double sg = STAGE == 0 ? sigma_integral(d.sigma0, d.sigma1, d.tau_ramp, a.t0, tm)
                                   : sigma_integral(d.sigma0, d.sigma1, d.tau_ramp, tm, a.t0 + h);
      auto prop = [&](int i) {  // P = exp(-kappa h/4) exp(i (omega' h/2 - int sigma))
        const double mag = exp(-0.25 * h * kap[i]);
        double sn, cs;
        sincos(0.5 * h * omg[i] - sg, &sn, &cs);
        return cx<Real>{(Real)(mag * cs), (Real)(mag * sn)};
      };
      const Real h2 = (Real)(0.5 * h), h1 = (Real)h, h6 = (Real)(h / 6.0), two = (Real)2;
      sfor<0, E>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        const int i = m1 + N1 * (t + m * T);
        const cx<Real> nk = v[m];
        cx<Real> k = {-gn * nk.im, gn * nk.re};
        if (i == N / 2) k = cadd(k, pump);
        cx<Real> nxt;
        if constexpr (STAGE == 0) {
          const cx<Real> p1 = prop(i);
          const cx<Real> yi = cmul(p1, A[i]);
          const cx<Real> k1 = cmul(p1, k);
          ACC[i] = k1;
          U[i] = yi;
          nxt = {yi.re + h2 * k1.re, yi.im + h2 * k1.im};
        } else if constexpr (STAGE == 1) {
          const cx<Real> yi = U[i], acc = ACC[i];
          ACC[i] = {acc.re + two * k.re, acc.im + two * k.im};
          nxt = {yi.re + h2 * k.re, yi.im + h2 * k.im};
        } else if constexpr (STAGE == 2) {
          const cx<Real> yi = U[i], acc = ACC[i];
          ACC[i] = {acc.re + two * k.re, acc.im + two * k.im};
          nxt = cmul(prop(i), cx<Real>{yi.re + h1 * k.re, yi.im + h1 * k.im});
        } else {
          const cx<Real> yi = U[i], acc = ACC[i];
          const cx<Real> z = cmul(prop(i), cx<Real>{yi.re + h6 * acc.re, yi.im + h6 * acc.im});
          nxt = {z.re + h6 * k.re, z.im + h6 * k.im};
          A[i] = nxt;
          if (a.ckpt) a.ckpt[d.a_offset + i] = nxt;
          bad |= !(isfinite(nxt.re) && isfinite(nxt.im));
        }
        v[m] = nxt;
      });
    } else {
    // Two workspace vectors carry the step (as in cme_stream.hip): W1 holds
    // k_1 after stage 1 and P = y + h/6 k_1 + h/3 k_2 + h/3 k_3 after stage 3,
    // W2 holds k_2 after stage 2 and u_4 after stage 3; u_2 and u_3 are formed
    // again from y and k_1, k_2, and stage 4 does not read y.  kappa is not
    // read where it is the same for every mode of the instance.
    const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, a.t0 + stage_c(STAGE) * h);
    const Real h2 = (Real)(0.5 * h), h1 = (Real)h, h3 = (Real)(h / 3.0), h6 = (Real)(h / 6.0);
    const bool ku = d.kappa_uniform != 0;
    const Real lr0 = (Real)(-0.5 * d.kappa0);
    cx<Real> *W1 = ACC, *W2 = U;
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const int i = m1 + N1 * (t + m * T);
      const bool band = in_band(i);
      const cx<Real> zero = {(Real)0, (Real)0};
      cx<Real> y = zero, w1 = zero, w2 = zero, u;
      if constexpr (STAGE < 3) {
        if (band) y = A[phys(i)];
      }
      if constexpr (STAGE == 1 || STAGE == 2) w1 = W1[i];
      if constexpr (STAGE >= 2) w2 = W2[i];
      if constexpr (STAGE == 0) u = y;
      if constexpr (STAGE == 1) u = {y.re + h2 * w1.re, y.im + h2 * w1.im};
      if constexpr (STAGE == 2) u = {y.re + h2 * w2.re, y.im + h2 * w2.im};
      if constexpr (STAGE == 3) u = w2;
      const cx<Real> nk = v[m];
      const Real lr = ku ? lr0 : (Real)(-0.5 * kap[i]), li = (Real)(omg[i] - sig);
      // k = L u + i (g0/N) N K
      cx<Real> k = {lr * u.re - li * u.im - gn * nk.im, lr * u.im + li * u.re + gn * nk.re};
      if (i == N / 2) k = cadd(k, pump);
      if (!band) k = zero;
      cx<Real> nxt;
      if constexpr (STAGE == 0) {
        W1[i] = k;
        nxt = {y.re + h2 * k.re, y.im + h2 * k.im};
      } else if constexpr (STAGE == 1) {
        W2[i] = k;
        nxt = {y.re + h2 * k.re, y.im + h2 * k.im};
      } else if constexpr (STAGE == 2) {
        const cx<Real> p1 = {y.re + h6 * w1.re, y.im + h6 * w1.im};
        const cx<Real> p2 = {p1.re + h3 * w2.re, p1.im + h3 * w2.im};
        W1[i] = {p2.re + h3 * k.re, p2.im + h3 * k.im};
        nxt = {y.re + h1 * k.re, y.im + h1 * k.im};
        W2[i] = nxt;
      } else {
        const cx<Real> p = W1[i];
        nxt = {p.re + h6 * k.re, p.im + h6 * k.im};
        if (band) {
          A[phys(i)] = nxt;
          if (a.ckpt) a.ckpt[d.a_offset + phys(i)] = nxt;
        }
        bad |= !(isfinite(nxt.re) && isfinite(nxt.im));
      }
      v[m] = nxt;
    });
    }
    if constexpr (STAGE == 3) {
      if (bad) atomicOr(&a.flags[id], 1);
      if (a.tail) return;
    }
  }
  // inner sum of the inverse transform over m2, times w^{+j2 m1}
  fft_team<N2, E, +1, kPS, false, 0, SYNC_WAVE>(v, buf, buf, tw, t);
  cx<Real> xw[E];
  cross_tw<N, E, T>(xw, a.tab, m1, t);
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    S[(t + m * T) * N1 + m1] = cmulc(v[m], xw[m]);
  });
}

template <int N, int N1, int E, int WPB, typename Real = double>
__global__ void __launch_bounds__(64 * WPB) staged_row(StagedArgsT<Real> a) {
  using SH = RowShape<N, N1, E, WPB>;
  constexpr int T = SH::T;
  __shared__ cx<Real> lds[WPB * SH::RW * SH::LB];
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  const int slot = (int)blockIdx.x / SH::NB, rb = (int)blockIdx.x % SH::NB;
  const int team = lane / T, t = lane % T;
  const int j2 = rb * SH::R + wv * SH::RW + team;
  cx<Real> *S = a.work + (int64_t)slot * 3 * N + (int64_t)j2 * N1;
  cx<Real> *buf = lds + (wv * SH::RW + team) * SH::LB;

  cx<Real> tw[FftPlan<N1, E>::NTW];
  load_twiddles<N1, E, N / N1>(tw, a.tab, t);
  cx<Real> v[E];
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    v[m] = S[t + m * T];
  });
  // outer sum of the inverse transform over m1: a_{j2 + N2 j1}, j1 = t + m T
  fft_team<N1, E, +1, kPS, false, 0, SYNC_WAVE>(v, buf, buf, tw, t);
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const Real p = v[m].re * v[m].re + v[m].im * v[m].im;
    v[m] = {p * v[m].re, p * v[m].im};
  });
  // inner sum of the forward transform over j1, times w^{-j2 m1}
  fft_team<N1, E, -1, kPS, false, 0, SYNC_WAVE>(v, buf, buf, tw, t);
  cx<Real> xw[E];
  cross_tw<N, E, T>(xw, a.tab, j2, t);
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    S[t + m * T] = cmul(v[m], xw[m]);
  });
}

template <int N, int N1, int E, int WPB, bool IP = false, typename Real = double, bool PAD = false>
hipError_t launch_staged(const RunArgs &r, hipStream_t st) {
  using CS = ColShape<N, N1, E, WPB>;
  using RS = RowShape<N, N1, E, WPB>;
  if (r.stages != nullptr || r.work == nullptr) return hipErrorInvalidValue;
  if (r.count <= 0 || r.n_steps <= 0) return hipSuccess;
  StagedArgsT<Real> a{};
  a.inst = r.inst;
  a.order = r.order;
  a.count = r.count;
  a.A = reinterpret_cast<cx<Real> *>(r.A);
  a.kappa = r.kappa;
  a.omega = r.omega;
  a.tab = reinterpret_cast<const cx<Real> *>(r.twiddle);
  a.work = reinterpret_cast<cx<Real> *>(r.work);
  a.h = r.h;
  a.flags = r.flags;
  const dim3 cgrid(r.count * CS::NB), rgrid(r.count * RS::NB), blk(64 * WPB);
  cx<Real> *ck = reinterpret_cast<cx<Real> *>(r.ckpt);
  a.t0 = (double)r.step0 * r.h;
  hipLaunchKernelGGL((staged_col<N, N1, E, WPB, -1, IP, Real, PAD>), cgrid, blk, 0, st, a);
  int64_t slot = 0;
  for (int64_t n = 0; n < r.n_steps; ++n) {
    a.t0 = (double)(r.step0 + n) * r.h;
    a.ckpt = nullptr;
    if (ck && r.ckpt_every > 0 && (n + 1) % r.ckpt_every == 0) a.ckpt = ck + (slot++) * r.total;
    a.tail = n + 1 == r.n_steps;
    hipLaunchKernelGGL((staged_row<N, N1, E, WPB, Real>), rgrid, blk, 0, st, a);
    hipLaunchKernelGGL((staged_col<N, N1, E, WPB, 0, IP, Real, PAD>), cgrid, blk, 0, st, a);
    hipLaunchKernelGGL((staged_row<N, N1, E, WPB, Real>), rgrid, blk, 0, st, a);
    hipLaunchKernelGGL((staged_col<N, N1, E, WPB, 1, IP, Real, PAD>), cgrid, blk, 0, st, a);
    hipLaunchKernelGGL((staged_row<N, N1, E, WPB, Real>), rgrid, blk, 0, st, a);
    hipLaunchKernelGGL((staged_col<N, N1, E, WPB, 2, IP, Real, PAD>), cgrid, blk, 0, st, a);
    hipLaunchKernelGGL((staged_row<N, N1, E, WPB, Real>), rgrid, blk, 0, st, a);
    hipLaunchKernelGGL((staged_col<N, N1, E, WPB, 3, IP, Real, PAD>), cgrid, blk, 0, st, a);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The split-step map (Sec. 2, the second method) on the same transforms.  A
// step from t0: exact linear half step with sigma frozen at t0 + h/4, a =
// IDFT(y), the exact Kerr rotation a e^{i g0 h |a|^2}, y = DFT(a) / N, exact
// linear half step with sigma at t0 + 3h/4.  Two launches per step:
//   row kernel: finish the inverse transform, rotate, start the forward one;
//   column kernel: finish the forward transform, the step's second half step
//   (and its checkpoint), the next step's first half step, start the next
//   inverse transform.
// MODE 0: first launch of a run (first half step of the first step);
// MODE 1: between steps; MODE 2: last step of the run (result to the state).
// ---------------------------------------------------------------------------

// y e^{L dt} + [pump mode] s (e^{L dt} - 1) / L with L = -kappa/2 + i(omega' - sigma)
__device__ __forceinline__ cx<double> linear_exact(cx<double> y, double kap, double om, double sig,
                                                   double dt, bool pump_mode, cx<double> s) {
  const double lre = -0.5 * kap, lim = om - sig;
  const double mag = exp(lre * dt);
  double sn, cs;
  sincos(lim * dt, &sn, &cs);
  const cx<double> e = {mag * cs, mag * sn};
  cx<double> out = cmul(y, e);
  if (pump_mode) {
    cx<double> phi;  // (e - 1) / L, or its small-|L dt| limit
    if (sqrt(lre * lre + lim * lim) * dt > 1e-8) {
      const double den = lre * lre + lim * lim;
      phi = {((e.re - 1.0) * lre + e.im * lim) / den, (e.im * lre - (e.re - 1.0) * lim) / den};
    } else {
      phi = {dt * (1.0 + 0.5 * lre * dt), dt * (0.5 * lim * dt)};
    }
    out = cadd(out, cmul(s, phi));
  }
  return out;
}

template <int N, int N1, int E, int WPB, int MODE>
__global__ void __launch_bounds__(64 * WPB) split_col(StagedArgs a) {
  using SH = ColShape<N, N1, E, WPB>;
  constexpr int N2 = SH::N2, T = SH::T;
  __shared__ cx<double> lds[WPB * SH::CW * SH::LB];
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  const int slot = (int)blockIdx.x / SH::NB, cb = (int)blockIdx.x % SH::NB;
  const int cl = lane % SH::CW, t = lane / SH::CW;
  const int m1 = cb * SH::C + wv * SH::CW + cl;
  const int id = a.order[slot];
  const DevInst d = a.inst[id];
  cx<double> *A = a.A + d.a_offset;
  cx<double> *S = a.work + (int64_t)slot * 3 * N;
  cx<double> *buf = lds + (wv * SH::CW + cl) * SH::LB;
  const double *kap = a.kappa + d.offset, *omg = a.omega + d.offset;
  const cx<double> s = {d.pump_re, d.pump_im};
  const double h = a.h, hh = 0.5 * a.h;

  cx<double> tw[FftPlan<N2, E>::NTW];
  load_twiddles<N2, E, N1>(tw, a.tab, t);
  cx<double> v[E];
  if constexpr (MODE == 0) {
    const double sig = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, a.t0 + 0.25 * h);
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const int i = m1 + N1 * (t + m * T);
      v[m] = linear_exact(A[i], kap[i], omg[i], sig, hh, i == N / 2, s);
    });
  } else {
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      v[m] = S[(t + m * T) * N1 + m1];
    });
    fft_team<N2, E, -1, kPS, false, 0, SYNC_WAVE>(v, buf, buf, tw, t);
    const double inv_n = 1.0 / (double)N;
    const double sig2 = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, a.t0 + 0.75 * h);
    const double sig1 = sigma_at(d.sigma0, d.sigma1, d.tau_ramp, a.t0 + 1.25 * h);
    bool bad = false;
    sfor<0, E>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      const int i = m1 + N1 * (t + m * T);
      const cx<double> y2 = {v[m].re * inv_n, v[m].im * inv_n};
      const cx<double> yn = linear_exact(y2, kap[i], omg[i], sig2, hh, i == N / 2, s);
      if (a.ckpt) a.ckpt[d.a_offset + i] = yn;
      if constexpr (MODE == 2) {
        A[i] = yn;
        bad |= !(isfinite(yn.re) && isfinite(yn.im));
      } else {
        v[m] = linear_exact(yn, kap[i], omg[i], sig1, hh, i == N / 2, s);
      }
    });
    if constexpr (MODE == 2) {
      if (bad) atomicOr(&a.flags[id], 1);
      return;
    }
  }
  fft_team<N2, E, +1, kPS, false, 0, SYNC_WAVE>(v, buf, buf, tw, t);
  cx<double> xw[E];
  cross_tw<N, E, T>(xw, a.tab, m1, t);
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    S[(t + m * T) * N1 + m1] = cmulc(v[m], xw[m]);
  });
}

template <int N, int N1, int E, int WPB>
__global__ void __launch_bounds__(64 * WPB) split_row(StagedArgs a) {
  using SH = RowShape<N, N1, E, WPB>;
  constexpr int T = SH::T;
  __shared__ cx<double> lds[WPB * SH::RW * SH::LB];
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  const int slot = (int)blockIdx.x / SH::NB, rb = (int)blockIdx.x % SH::NB;
  const int team = lane / T, t = lane % T;
  const int j2 = rb * SH::R + wv * SH::RW + team;
  const DevInst d = a.inst[a.order[slot]];
  cx<double> *S = a.work + (int64_t)slot * 3 * N + (int64_t)j2 * N1;
  cx<double> *buf = lds + (wv * SH::RW + team) * SH::LB;
  const double gh = d.g0n * (double)N * a.h;  // g0 h

  cx<double> tw[FftPlan<N1, E>::NTW];
  load_twiddles<N1, E, N / N1>(tw, a.tab, t);
  cx<double> v[E];
  sfor<0, E>([&](auto mi) { v[decltype(mi)::value] = S[t + decltype(mi)::value * T]; });
  fft_team<N1, E, +1, kPS, false, 0, SYNC_WAVE>(v, buf, buf, tw, t);
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    double sn, cs;
    sincos(gh * (v[m].re * v[m].re + v[m].im * v[m].im), &sn, &cs);
    v[m] = cmul(v[m], cx<double>{cs, sn});
  });
  fft_team<N1, E, -1, kPS, false, 0, SYNC_WAVE>(v, buf, buf, tw, t);
  cx<double> xw[E];
  cross_tw<N, E, T>(xw, a.tab, j2, t);
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    S[t + m * T] = cmul(v[m], xw[m]);
  });
}

template <int N, int N1, int E, int WPB>
hipError_t launch_split_staged(const RunArgs &r, hipStream_t st) {
  using CS = ColShape<N, N1, E, WPB>;
  using RS = RowShape<N, N1, E, WPB>;
  if (r.stages != nullptr || r.work == nullptr) return hipErrorInvalidValue;
  if (r.count <= 0 || r.n_steps <= 0) return hipSuccess;
  StagedArgs a{};
  a.inst = r.inst;
  a.order = r.order;
  a.count = r.count;
  a.A = reinterpret_cast<cx<double> *>(r.A);
  a.kappa = r.kappa;
  a.omega = r.omega;
  a.tab = reinterpret_cast<const cx<double> *>(r.twiddle);
  a.work = reinterpret_cast<cx<double> *>(r.work);
  a.h = r.h;
  a.flags = r.flags;
  const dim3 cgrid(r.count * CS::NB), rgrid(r.count * RS::NB), blk(64 * WPB);
  cx<double> *ck = reinterpret_cast<cx<double> *>(r.ckpt);
  a.t0 = (double)r.step0 * r.h;
  hipLaunchKernelGGL((split_col<N, N1, E, WPB, 0>), cgrid, blk, 0, st, a);
  int64_t slot = 0;
  for (int64_t n = 0; n < r.n_steps; ++n) {
    a.t0 = (double)(r.step0 + n) * r.h;
    a.ckpt = nullptr;
    if (ck && r.ckpt_every > 0 && (n + 1) % r.ckpt_every == 0) a.ckpt = ck + (slot++) * r.total;
    hipLaunchKernelGGL((split_row<N, N1, E, WPB>), rgrid, blk, 0, st, a);
    if (n + 1 == r.n_steps)
      hipLaunchKernelGGL((split_col<N, N1, E, WPB, 2>), cgrid, blk, 0, st, a);
    else
      hipLaunchKernelGGL((split_col<N, N1, E, WPB, 1>), cgrid, blk, 0, st, a);
  }
  return hipGetLastError();
}

template <int N, int N1, int E, int WPB> constexpr Variant split_staged_variant() {
  using CS = ColShape<N, N1, E, WPB>;
  using RS = RowShape<N, N1, E, WPB>;
  return Variant{0, N, E, N1, kPS, WPB, 9, 1, 64 * WPB,
                 CS::LDS_BYTES > RS::LDS_BYTES ? CS::LDS_BYTES : RS::LDS_BYTES,
                 &launch_split_staged<N, N1, E, WPB>, nullptr, 3};
}

// The four-wave-mixing sum alone (cme_fwm): r.A in, r.ckpt out, through the
// class workspace.
template <int N, int N1, int E, int WPB, bool PAD>
hipError_t fwm_staged(const RunArgs &r, hipStream_t st) {
  using CS = ColShape<N, N1, E, WPB>;
  using RS = RowShape<N, N1, E, WPB>;
  if (r.work == nullptr || r.ckpt == nullptr) return hipErrorInvalidValue;
  if (r.count <= 0) return hipSuccess;
  StagedArgs a{};
  a.inst = r.inst;
  a.order = r.order;
  a.count = r.count;
  a.A = reinterpret_cast<cx<double> *>(r.A);
  a.kappa = r.kappa;
  a.omega = r.omega;
  a.tab = reinterpret_cast<const cx<double> *>(r.twiddle);
  a.work = reinterpret_cast<cx<double> *>(r.work);
  a.ckpt = reinterpret_cast<cx<double> *>(r.ckpt);
  a.flags = r.flags;
  const dim3 cgrid(r.count * CS::NB), rgrid(r.count * RS::NB), blk(64 * WPB);
  hipLaunchKernelGGL((staged_col<N, N1, E, WPB, -1, false, double, PAD>), cgrid, blk, 0, st, a);
  hipLaunchKernelGGL((staged_row<N, N1, E, WPB>), rgrid, blk, 0, st, a);
  hipLaunchKernelGGL((staged_col<N, N1, E, WPB, 4, false, double, PAD>), cgrid, blk, 0, st, a);
  return hipGetLastError();
}

template <int N, int N1, int E, int WPB, bool IP = false, typename Real = double>
constexpr Variant staged_variant() {
  using CS = ColShape<N, N1, E, WPB>;
  using RS = RowShape<N, N1, E, WPB>;
  constexpr int scale = 16 / (int)sizeof(cx<Real>);  // the shapes count 16-byte elements
  return Variant{std::is_same<Real, double>::value ? 0 : 1, N, E, N1, kPS, WPB, IP ? 8 : 6, 1,
                 64 * WPB, (CS::LDS_BYTES > RS::LDS_BYTES ? CS::LDS_BYTES : RS::LDS_BYTES) / scale,
                 &launch_staged<N, N1, E, WPB, IP, Real>, nullptr, 3};
}

// (N, N1, E, waves per workgroup); the field `v` of a variant holds N1 and
// `tp` the waves per workgroup.  The
// first of a size is its default: eight waves per workgroup measured 1-7%
// faster than four.
const Variant kStagedVariants[] = {
    staged_variant<8192, 128, 8, 8>(),  staged_variant<8192, 64, 8, 8>(),
    staged_variant<8192, 128, 8, 4>(),  staged_variant<16384, 128, 8, 8>(),
    staged_variant<16384, 128, 8, 4>(), staged_variant<32768, 256, 8, 8>(),
    staged_variant<32768, 256, 8, 4>(), staged_variant<65536, 256, 8, 8>(),
    staged_variant<65536, 256, 8, 4>(),
    // FP32 state, transforms and stage arithmetic (FP64 only in the time-dependent coefficients)
    staged_variant<8192, 128, 8, 8, false, float>(),  staged_variant<16384, 128, 8, 8, false, float>(),
    staged_variant<32768, 256, 8, 8, false, float>(), staged_variant<65536, 256, 8, 8, false, float>(),
};

// split-step map on the same transforms (kind 9)
const Variant kStagedSplitVariants[] = {
    split_staged_variant<8192, 128, 8, 8>(),  split_staged_variant<16384, 128, 8, 8>(),
    split_staged_variant<32768, 256, 8, 8>(), split_staged_variant<65536, 256, 8, 8>(),
};

// alias-free truncated sum on the same transforms (kind 10): transform
// length N for instances of N/2 = 8192 ... 32768 modes
template <int N, int N1, int E, int WPB> constexpr Variant staged_pad_variant() {
  using CS = ColShape<N, N1, E, WPB>;
  using RS = RowShape<N, N1, E, WPB>;
  return Variant{0, N, E, N1, kPS, WPB, 10, 1, 64 * WPB,
                 CS::LDS_BYTES > RS::LDS_BYTES ? CS::LDS_BYTES : RS::LDS_BYTES,
                 &launch_staged<N, N1, E, WPB, false, double, true>, nullptr, 3};
}
const Variant kStagedPadVariants[] = {
    staged_pad_variant<16384, 128, 8, 8>(), staged_pad_variant<32768, 256, 8, 8>(),
    staged_pad_variant<65536, 256, 8, 8>(),
};

// interaction-picture RK4 on the same transforms (kind 8)
const Variant kStagedIpVariants[] = {
    staged_variant<8192, 128, 8, 8, true>(),  staged_variant<16384, 128, 8, 8, true>(),
    staged_variant<32768, 256, 8, 8, true>(), staged_variant<65536, 256, 8, 8, true>(),
    // FP32 above 8192: state, transforms and stage arithmetic (FP64 only in the propagator's phase)
    staged_variant<16384, 128, 8, 8, true, float>(), staged_variant<32768, 256, 8, 8, true, float>(),
    staged_variant<65536, 256, 8, 8, true, float>(),
};

}  // namespace

template <int N, int N1> hipError_t fwm_staged_any(bool pad, const RunArgs &r, hipStream_t st) {
  return pad ? fwm_staged<N, N1, 8, 8, true>(r, st) : fwm_staged<N, N1, 8, 8, false>(r, st);
}

hipError_t launch_staged_fwm(int n, bool pad, const RunArgs &r, hipStream_t st) {
  switch (n) {
    case 16384: return fwm_staged_any<16384, 128>(pad, r, st);
    case 32768: return fwm_staged_any<32768, 256>(pad, r, st);
    case 65536: return fwm_staged_any<65536, 256>(pad, r, st);
    default: return hipErrorInvalidValue;
  }
}

const Variant *variants_staged_pad(int *count) {
  *count = (int)(sizeof(kStagedPadVariants) / sizeof(kStagedPadVariants[0]));
  return kStagedPadVariants;
}

const Variant *variants_staged_split(int *count) {
  *count = (int)(sizeof(kStagedSplitVariants) / sizeof(kStagedSplitVariants[0]));
  return kStagedSplitVariants;
}

const Variant *variants_staged_ip(int *count) {
  *count = (int)(sizeof(kStagedIpVariants) / sizeof(kStagedIpVariants[0]));
  return kStagedIpVariants;
}

const Variant *variants_staged(int *count) {
  *count = (int)(sizeof(kStagedVariants) / sizeof(kStagedVariants[0]));
  return kStagedVariants;
}

}  // namespace cme
