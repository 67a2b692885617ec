// cme_fwm.hip -- the four-wave-mixing sum alone: for every instance of a plan,
//   K_mu = sum over alpha - beta + gamma = mu (mod N) of A_alpha conj(A_beta) A_gamma
// (Eq. (1), cyclic), evaluated as in Eq. (4): a = IDFT(A), b = |a|^2 a,
// K = DFT(b) / N.  The transforms are the library's own: the one-level team
// transform of cme_fft.hpp below 128 modes, the two-level wave transform of
// the wave kernels up to 8192, and the staged four-step transform above
// (cme_staged.hip).  Input A and output K are packed like the state.
#include <type_traits>

#include "cme_wave.hpp"

namespace cme {

namespace {

// PAD: a padded plan's instance of N/2 modes sits at transform indices
// [N/4, 3N/4) (mode i - N/4 of the caller's arrays), the rest of the input is
// zero, and only the band is written: the cyclic sum over the zero-padded
// transform restricted to the band is the truncated sum.
template <typename Real, int N, int E, int V, int PS, int TP, bool PAD = false>
__global__ void __launch_bounds__((WaveShape<Real, N, E, V, PS, TP>::THREADS)) fwm_wave(RunArgs a) {
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
  const DevInst d = a.inst[a.order[slot]];
  cx<Real> *X = lds + sub * SH::PER_INST;
  cx<Real> *Y = SH::TWO ? X + SH::WV * SH::LB1 : X;
  constexpr int Q4 = N / 4;
  auto in_band = [](int i) { return !PAD || (i >= Q4 && i < 3 * Q4); };
  auto phys = [](int i) { return PAD ? i - Q4 : i; };
  const int64_t off = PAD ? d.a_offset : d.offset;
  const cx<Real> *A = reinterpret_cast<const cx<Real> *>(a.A) + off;
  cx<Real> *K = reinterpret_cast<cx<Real> *>(a.ckpt) + off;
  WaveTwiddles<N, E, V, TP, Real> tw;
  load_wave_twiddles<N, E, V>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), w, lane);
  cx<Real> v[E];
  sfor<0, E>([&](auto mi) {
    const int i = WP::mode(w, lane, decltype(mi)::value);
    v[decltype(mi)::value] = in_band(i) ? A[phys(i)] : cx<Real>{(Real)0, (Real)0};
  });
  fft_fwdpath<N, E, V, TP, +1, PS, !SH::TWO>(v, X, tw, w, lane);
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const Real p = v[m].re * v[m].re + v[m].im * v[m].im;
    v[m] = {p * v[m].re, p * v[m].im};
  });
  fft_backpath<N, E, V, TP, -1, PS>(v, X, Y, tw, w, lane);
  const Real inv_n = (Real)1 / (Real)N;
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const int i = WP::mode(w, lane, m);
    if (in_band(i)) K[phys(i)] = {v[m].re * inv_n, v[m].im * inv_n};
  });
}

// below one wavefront per instance: one instance per workgroup of N / E
// threads, thread t holding modes t + m T
template <typename Real, int N, int E>
__global__ void __launch_bounds__(N / E) fwm_team(RunArgs a) {
  constexpr int T = N / E, PS = 2;
  __shared__ cx<Real> buf[LdsLen<N, PS>::value];
  const int t = (int)threadIdx.x;
  const DevInst d = a.inst[a.order[blockIdx.x]];
  const cx<Real> *A = reinterpret_cast<const cx<Real> *>(a.A) + d.offset;
  cx<Real> *K = reinterpret_cast<cx<Real> *>(a.ckpt) + d.offset;
  cx<Real> tw[FftPlan<N, E>::NTW];
  load_twiddles<N, E>(tw, reinterpret_cast<const cx<Real> *>(a.twiddle), t);
  cx<Real> v[E];
  sfor<0, E>([&](auto mi) { v[decltype(mi)::value] = A[t + decltype(mi)::value * T]; });
  fft_team<N, E, +1, PS, false, 0, SYNC_BLOCK>(v, buf, buf, tw, t);
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    const Real p = v[m].re * v[m].re + v[m].im * v[m].im;
    v[m] = {p * v[m].re, p * v[m].im};
  });
  fft_team<N, E, -1, PS, false, 0, SYNC_BLOCK>(v, buf, buf, tw, t);
  const Real inv_n = (Real)1 / (Real)N;
  sfor<0, E>([&](auto mi) {
    constexpr int m = decltype(mi)::value;
    K[t + m * T] = {v[m].re * inv_n, v[m].im * inv_n};
  });
}

template <typename Real, int N, int E, int V, int PS, int TP = 0, bool PAD = false>
hipError_t launch_wave_fwm(const RunArgs &a, hipStream_t st) {
  using SH = WaveShape<Real, N, E, V, PS, TP>;
  const int grid = (a.count + SH::IPB - 1) / SH::IPB;
  hipLaunchKernelGGL((fwm_wave<Real, N, E, V, PS, TP, PAD>), dim3(grid), dim3(SH::THREADS), 0, st,
                     a);
  return hipGetLastError();
}

template <typename Real, int N, int E> hipError_t launch_team_fwm(const RunArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((fwm_team<Real, N, E>), dim3(a.count), dim3(N / E), 0, st, a);
  return hipGetLastError();
}

template <typename Real> hipError_t launch_fwm_real(int n, const RunArgs &a, hipStream_t st) {
  switch (n) {
    case 16: return launch_team_fwm<Real, 16, 4>(a, st);
    case 32: return launch_team_fwm<Real, 32, 4>(a, st);
    case 64: return launch_team_fwm<Real, 64, 4>(a, st);
    case 128: return launch_wave_fwm<Real, 128, 2, 1, 1>(a, st);
    case 256: return launch_wave_fwm<Real, 256, 4, 1, 2>(a, st);
    case 512: return launch_wave_fwm<Real, 512, 8, 1, 3>(a, st);
    case 1024: return launch_wave_fwm<Real, 1024, 8, 1, 3>(a, st);
    case 2048: return launch_wave_fwm<Real, 2048, 8, 1, 3>(a, st);
    case 4096: return launch_wave_fwm<Real, 4096, 8, 1, 3>(a, st);
    case 8192: return launch_wave_fwm<Real, 8192, 16, 2, 3>(a, st);
    default: return hipErrorInvalidValue;
  }
}

// padded plans (FP64): transform length n for instances of n/2 modes
hipError_t launch_fwm_pad(int n, const RunArgs &a, hipStream_t st) {
  switch (n) {
    case 256: return launch_wave_fwm<double, 256, 4, 1, 2, 0, true>(a, st);
    case 512: return launch_wave_fwm<double, 512, 8, 1, 3, 0, true>(a, st);
    case 1024: return launch_wave_fwm<double, 1024, 8, 1, 3, 0, true>(a, st);
    case 2048: return launch_wave_fwm<double, 2048, 8, 1, 3, 0, true>(a, st);
    case 4096: return launch_wave_fwm<double, 4096, 8, 1, 3, 0, true>(a, st);
    case 8192: return launch_wave_fwm<double, 8192, 16, 2, 3, 0, true>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// a.A: input, a.ckpt: output; sizes above 8192 go to the staged transform
hipError_t launch_staged_fwm(int n, bool pad, const RunArgs &a, hipStream_t st);  // cme_staged.hip

hipError_t launch_fwm(int precision, int n, bool pad, const RunArgs &a, hipStream_t st) {
  if (a.count <= 0) return hipSuccess;
  if (n > 8192) return precision == 0 ? launch_staged_fwm(n, pad, a, st) : hipErrorInvalidValue;
  if (pad) return precision == 0 ? launch_fwm_pad(n, a, st) : hipErrorInvalidValue;
  return precision == 0 ? launch_fwm_real<double>(n, a, st) : launch_fwm_real<float>(n, a, st);
}

}  // namespace cme
