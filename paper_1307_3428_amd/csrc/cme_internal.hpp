// cme_internal.hpp -- structures shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cme {

// Per-instance constants on the device (built by cme_init from cme_instance).
struct DevInst {
  int64_t offset;      // first element in the packed per-mode arrays
  double pump_re;      // sqrt(kappa_ext) * A_in: the drive term of Eq. (1)
  double pump_im;
  double g0n;          // g0 / N: the forward transform carries the 1/N of Eq. (4)
  double sqrt_kext;    // sqrt(kappa_ext), for the pump gradient
  double sigma0, sigma1, tau_ramp;
  int32_t n;
  int32_t kappa_uniform;  // 1: kappa_mu is the same for every mode (kappa0), and the
                          // kernels that stream kappa from global memory may skip it
  int64_t a_offset;    // first element in the caller's packed state (padded plans:
                       // the state has n/2 modes per instance, kappa/omega' n)
  double kappa0;       // kappa_mu of mode 0 (every mode when kappa_uniform)
};

// Arguments of one persistent forward launch over one size class.
struct RunArgs {
  const DevInst *inst;     // [batch]
  const int32_t *order;    // instance ids of this class, in launch order
  int32_t count;           // instances in this class
  int32_t ckpt_every;      // 0: no checkpoints
  void *A;                 // packed state, complex Real [total]
  const double *kappa;     // packed kappa_mu [total]
  const double *omega;     // packed omega'_mu [total]
  const void *twiddle;     // exp(-2 pi i k / N), k < N, complex Real
  double h;
  int64_t step0;
  int64_t n_steps;
  void *ckpt;              // complex Real [n_steps / ckpt_every][total] or null
  int64_t total;
  int32_t *flags;          // [batch] non-finite flags
  void *stages;            // adjoint recompute: per step and stage, the stage input u_s
                           // and its inverse transform a_s, [K][4][2][total], or null
  void *work;              // class workspace of variants with work > 0: `work` complex
                           // values per mode for each instance of the class, in class order
};

// Arguments of one reverse (adjoint) launch over one segment of one class.
struct AdjArgs {
  const DevInst *inst;
  const int32_t *order;
  int32_t count;
  int32_t n_seg;           // steps in this segment
  const void *stages;      // u_s and a_s of every step of the segment [K][4][2][total]
  void *gA;                // in: cotangent of the state after the segment; out: before
  const double *kappa;
  const double *omega;
  const void *twiddle;
  double h;
  int64_t step_first;      // step index of the first step of the segment
  int64_t total;
  double *g_omega;         // [total] or null (accumulated)
  double *g_kappa;         // [total] or null (accumulated)
  double *g_ain;           // [2 batch] or null (accumulated)
  void *kbar;              // variants with adj_kbar: the reverse sweep stores kbar_s of every
                           // step and stage here, [K][4][total] complex, in place of
                           // accumulating the parameter cotangents (launch_adj_params does)
};

// Offset of the stage-s record of step n in the adjoint stage buffer: the
// stage input u_s (mode order, packed like A) at this offset, the inverse
// transform a_s = IDFT(u_s) (in the kernel's time-domain slot order) total
// elements further.
__host__ __device__ inline int64_t stage_offset(int64_t n, int s, int64_t total) {
  return (n * 4 + s) * 2 * total;
}

__host__ __device__ inline double sigma_at(double sigma0, double sigma1, double tau_ramp,
                                           double t) {
  if (!(tau_ramp > 0.0)) return sigma0;
  const double s = t < 0.0 ? 0.0 : (t > tau_ramp ? tau_ramp : t);
  return sigma0 + (sigma1 - sigma0) * (s / tau_ramp);
}

// integral of sigma(t) over [a, b], 0 <= a <= b, for the ramp of sigma_at
// (the interaction-picture kernels' exact linear propagators)
__host__ __device__ inline double sigma_integral(double s0, double s1, double tau, double a,
                                                 double b) {
  if (!(tau > 0.0)) return s0 * (b - a);
  double ramp;  // integral of min(t, tau)
  if (b <= tau) ramp = 0.5 * (b - a) * (b + a);
  else if (a >= tau) ramp = tau * (b - a);
  else ramp = 0.5 * (tau - a) * (tau + a) + tau * (b - tau);
  return s0 * (b - a) + (s1 - s0) / tau * ramp;
}

using FwdLaunch = hipError_t (*)(const RunArgs &, hipStream_t);
using AdjLaunch = hipError_t (*)(const AdjArgs &, hipStream_t);

// One compiled kernel variant.
struct Variant {
  int precision;   // 0 FP64, 1 FP32
  int n;           // modes
  int e;           // elements per thread
  int v;           // wave-local sub-transforms per wave (1 for team kernels)
  int ps;          // LDS padding: one element every 2^ps (0: none)
  int tp;          // wave kernels: sub-transform kind (0 Stockham, 1 registers + LDS, 2 registers)
  int kind;        // 0: team kernel (cme_kernels.hip), 1: two-level wave kernel
                   // (cme_wave.hpp), 2: four rounds of two interleaved transforms
                   // per RK4 step (cme_duo.hip), 3: two-level kernel sized for two
                   // waves per SIMD (cme_lean.hip), 4: split-step map (cme_split.hip),
                   // 5: RK4 with the padded (alias-free truncated) sum (cme_wave.hip),
                   // 6: RK4 with four-step transforms staged through global memory
                   // (cme_staged.hip; `v` holds the row length N1), 7: interaction-
                   // picture RK4 (cme_rk4ip.hip), 8: interaction-picture RK4 on the
                   // staged transforms (cme_staged.hip), 9: split-step map on the
                   // staged transforms (cme_staged.hip), 10: RK4 with the padded sum
                   // on the staged transforms (cme_staged.hip), 11: RK4 with the
                   // padded sum on the lean kernel (cme_lean.hip), 12: interaction-
                   // picture RK4 on the lean kernel (cme_lean.hip), 13: RK4 on the
                   // two-level transform with the RK4 vectors in global memory
                   // (cme_stream.hip), 14: interaction-picture RK4 on that
                   // layout (cme_stream.hip)
  int ipb;         // instances per workgroup
  int threads;     // workgroup size
  int lds_bytes;   // static LDS per workgroup
  FwdLaunch fwd;
  AdjLaunch adj;   // null if no adjoint kernel for this variant (FP32)
  int work = 0;    // complex values of class workspace per mode (RunArgs::work)
  int adj_kbar = 0;  // the reverse sweep stores kbar_s (AdjArgs::kbar) for launch_adj_params
};

const Variant *variants_team(int *count);  // cme_kernels.hip
const Variant *variants_wave(int *count);      // cme_wave.hip (FP64)
const Variant *variants_pad(int *count);       // cme_wave.hip (padded sum)
const Variant *variants_wave_f32(int *count);  // cme_wave_f32.hip
const Variant *variants_lean(int *count);  // cme_lean.hip
const Variant *variants_duo(int *count);   // cme_duo.hip
const Variant *variants_duo_f32(int *count);  // cme_duo.hip (FP32)
const Variant *variants_split(int *count); // cme_split.hip
const Variant *variants_staged(int *count);  // cme_staged.hip
const Variant *variants_rk4ip(int *count);   // cme_rk4ip.hip
const Variant *variants_staged_ip(int *count);  // cme_staged.hip (interaction picture)
const Variant *variants_staged_split(int *count);  // cme_staged.hip (split-step)
const Variant *variants_staged_pad(int *count);    // cme_staged.hip (padded sum)
const Variant *variants_stream(int *count);   // cme_stream.hip
const Variant *variants(int *count);       // all of them (cme_api.hip)

// The four-wave-mixing sum alone for one size class (cme_fwm.hip): reads the
// packed amplitudes at a.A and writes K at a.ckpt (same packing); sizes above
// 8192 use the staged transform and the class workspace a.work.  pad: a
// padded plan's class (transform length n, instances of n/2 modes, the
// truncated sum).
hipError_t launch_fwm(int precision, int n, bool pad, const RunArgs &a, hipStream_t st);

// Parameter cotangents of one segment from the stage inputs u_s (a.stages)
// and the stored kbar_s (a.kbar) of a class of n-mode instances (FP64,
// cme_duo.hip): g_omega += Re(conj(kbar) i u), g_kappa -= Re(conj(kbar) u) / 2,
// g_ain += sqrt(kappa_ext) kbar at mu = 0, summed over the segment's steps and
// stages.
hipError_t launch_adj_params(int n, const AdjArgs &a, hipStream_t st);

}  // namespace cme
