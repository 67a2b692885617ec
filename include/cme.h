/*
 * cme.h -- C ABI of the MI355X (gfx950) solver for the Kerr-comb coupled mode
 * equations (CME) of Hansson, Modotto & Wabnitz, "On the numerical simulation
 * of Kerr frequency combs using coupled mode equations", arXiv:1307.3428.
 *
 * The solver time-steps Eq. (1) of the paper in the frame rotating with the
 * pump and the FSR grid (the frame of Eq. (2), without its rescaling):
 *
 *   dA_mu/dtau = (-kappa_mu/2 + i(omega'_mu - sigma(tau))) A_mu
 *                + [mu == 0] sqrt(kappa_ext) A_in + i g0 K_mu(A),
 *
 *   K_mu = sum over alpha - beta + gamma = mu (mod N) of A_alpha conj(A_beta) A_gamma,
 *
 * where omega'_mu = omega_mu - omega_0 - mu D1 (the FSR offset of Eq. (2) read
 * as mu times the FSR) and sigma = omega_in - omega_0 (Eq. (1)).  The
 * four-wave-mixing sum K is evaluated as in Eq. (4): an inverse transform of
 * the mode amplitudes, the pointwise cube |a|^2 a, and a forward transform
 * carrying the single 1/N; both transforms run as FFTs inside the GPU kernels.
 * Time stepping is the classic fourth-order Runge-Kutta scheme named in
 * Sec. 2 (stage times t, t+h/2, t+h/2, t+h; weights 1/6, 1/3, 1/3, 1/6);
 * cme_init also offers the paper's frequency-domain split-step method and
 * an interaction-picture RK4, and cme_fwm evaluates K alone.
 *
 * Conventions shared by every entry point
 *   - An instance is one resonator.  Its N mode amplitudes are stored
 *     contiguously in centred order: element i holds mode mu = i - N/2, so the
 *     pump mode mu = 0 is element N/2.  N must be a power of two,
 *     16 <= N <= 65536 (N <= 32768 with the padded sum); above 8192
 *     transform points FP64 with any integrator (classic RK4 for the padded
 *     sum) or FP32 with classic RK4 or RK4IP (CME_EUNSUPPORTED otherwise).
 *   - A batch packs instances back to back; instance b starts at element
 *     inst[b].mode_offset of every per-mode array (state, kappa, omega').
 *     Ranges of different instances must not overlap.  "total" below is the
 *     number of packed elements: max over b of mode_offset + n_modes.
 *   - Complex arrays are interleaved (re, im) pairs: 16 bytes per element in
 *     FP64 plans, 8 bytes in FP32 plans.
 *   - Time enters only through the integer step index: step n of a call with
 *     first step step0 is at tau = (step0 + n) * h.  Splitting a run into
 *     several calls therefore gives bit-identical results.
 *   - Device pointers are HIP device addresses on the device that was
 *     current at cme_init.  The caller owns every pointer it passes; the
 *     library never frees or reallocates caller memory.
 *   - All compute calls are asynchronous on the plan's stream and return a
 *     launch status.  Numerical failure (a non-finite amplitude) is reported
 *     per instance by cme_status, which synchronises the stream.
 */
#ifndef CME_H
#define CME_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes: 0 on success, negative on error (see cme_strerror). */
enum {
  CME_OK = 0,
  CME_EINVAL = -1,       /* invalid argument: null pointer, N not a power of
                            two or out of range, h <= 0, bad offsets, ...   */
  CME_ENOMEM = -2,       /* device or host allocation failed                */
  CME_EHIP = -3,         /* a HIP runtime call failed                       */
  CME_EUNSTABLE = -4,    /* classic RK4 step outside its stability region:
                            |R(h (-kappa_mu/2 + i(omega'_mu - sigma)))| > 1
                            for some mode, instance and detuning, with
                            R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24           */
  CME_ENONFINITE = -5,   /* non-finite input (kappa, omega', pump, ...)    */
  CME_EUNSUPPORTED = -6, /* valid request the library does not provide     */
  CME_ENODEVICE = -7,    /* no gfx950 device / kernels not loadable        */
  CME_ESCRATCH = -8      /* cme_adjoint_noalloc: the request needs more than
                            CME_NOALLOC_SCRATCH_BYTES of scratch            */
};

/* Size of the library's fixed device scratch array (one per GPU, held until
 * the process ends), the only working memory of cme_adjoint_noalloc. */
#define CME_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

enum { CME_F64 = 0, CME_F32 = 1 };        /* arithmetic precision            */
enum { CME_RK4 = 0, CME_RK4IP = 1, CME_SPLIT_STEP = 2 }; /* integrator       */
enum {
  CME_FWM_CYCLIC = 0, /* FWM sum taken modulo N (Eq. (4))                       */
  CME_FWM_PADDED = 1  /* FWM sum over the instance's own modes only (the literal
                         Kronecker delta of Eq. (2)), computed on 2N-point
                         transforms with the upper half held at zero; RK4,
                         FP64, N = 128 ... 32768, no adjoint                 */
};

/* Flags of cme_init (bitwise or). */
enum {
  CME_INIT_DEFAULT = 0,
  CME_INIT_SKIP_STABILITY = 1, /* do not refuse steps past the RK4 bound     */
  CME_INIT_AUTOTUNE = 2        /* time the kernel variants for each N once and
                                  keep the fastest (otherwise a fixed table) */
};

/* One resonator: the scalar symbols of Eq. (1). */
typedef struct {
  int32_t n_modes;      /* N: power of two, 16 <= N <= 65536                  */
  int32_t reserved;     /* must be 0                                          */
  int64_t mode_offset;  /* first element of this instance in per-mode arrays  */
  double kappa_ext;     /* external coupling loss kappa_ext >= 0              */
  double g0;            /* Kerr coefficient g0                                */
  double a_in_re;       /* pump amplitude A_in (drives mu = 0 only)           */
  double a_in_im;
  double sigma0;        /* detuning sigma = omega_in - omega_0 at tau = 0     */
  double sigma1;        /* detuning for tau >= tau_ramp                       */
  double tau_ramp;      /* sigma(tau) = sigma0 + (sigma1 - sigma0)
                           * min(tau, tau_ramp) / tau_ramp if tau_ramp > 0,
                           sigma0 otherwise                                   */
} cme_instance;

typedef struct cme_plan cme_plan;

/* Create a plan for a batch of `batch` instances (Eq. (1) parameters).
 *   inst   host array [batch]; copied.
 *   kappa  device array [total] of FP64 kappa_mu (total loss per mode); copied
 *          into plan-owned memory, so it may be freed after the call.  An
 *          instance whose kappa_mu is the same for every mode runs a faster
 *          path of the N = 2048 paired kernel and the N = 8192 LDS-resident
 *          kernels (one loss value instead of one per mode); results agree
 *          with the per-mode path to rounding.
 *   omega  device array [total] of FP64 omega'_mu; copied likewise.
 *   precision CME_F64 or CME_F32 (FP32 state and transforms; the time and
 *          detuning bookkeeping stays FP64).
 *   integrator CME_RK4 (classic fourth-order Runge-Kutta, Sec. 2),
 *          CME_RK4IP (interaction-picture RK4, not in the paper: RK4 on
 *          exp(-int L) A with the linear rate L_mu = -kappa_mu/2 +
 *          i(omega'_mu - sigma(t)) integrated exactly, the Kerr term and the
 *          pump through the stages; no RK4 stability check, since the
 *          dispersion no longer bounds the step; no adjoint, cyclic sum
 *          only) or
 *          CME_SPLIT_STEP (frequency-domain Strang split-step, Sec. 2: exact
 *          linear half steps per mode around the exact Kerr phase rotation
 *          of the transformed field; N >= 128, FP32 up to N = 4096, no
 *          adjoint).
 *   fwm    CME_FWM_CYCLIC or CME_FWM_PADDED (see above).
 *   h      step size (> 0) in the time units of kappa.
 *   stream hipStream_t the plan enqueues on (NULL: the null stream).
 *   flags  CME_INIT_* bits.
 * The RK4 stability check uses the detuning range [min(sigma0, sigma1),
 * max(sigma0, sigma1)] of every instance.  On error *plan is set to NULL. */
int cme_init(cme_plan **plan, int32_t batch, const cme_instance *inst,
             const double *kappa, const double *omega, int32_t precision,
             int32_t integrator, int32_t fwm, double h, void *stream, uint32_t flags);

/* Advance the packed state A (device, complex [total], in/out) by one RK4
 * step from step index step0.  Same as cme_run with n_steps = 1. */
int cme_step(cme_plan *plan, void *A, int64_t step0);

/* Advance A by n_steps >= 0 RK4 steps starting at step index step0 >= 0.
 * Each instance stays on one GPU workgroup for the whole call (persistent),
 * except for N >= 16384 (and N = 8192 when the staged variant is selected):
 * there the transforms are four-step transforms with the transpose through
 * global memory, each instance spans several workgroups, a step is eight
 * launches, and the plan owns a workspace of 3 N complex values per instance.
 *   ckpt_every  0, or store the state after every ckpt_every steps into
 *   ckpt        device complex [n_steps / ckpt_every][total]: slot j holds
 *               A after (j + 1) * ckpt_every steps of this call. */
int cme_run(cme_plan *plan, void *A, int64_t step0, int64_t n_steps,
            int32_t ckpt_every, void *ckpt);

/* The four-wave-mixing sum alone, for every instance of the plan:
 *   K_mu = sum over alpha - beta + gamma = mu (mod N) of A_alpha conj(A_beta) A_gamma
 * (Eq. (1) with the cyclic sum of Eq. (4)), evaluated with the library's
 * transforms as Eq. (4) states it: a = IDFT(A), b = |a|^2 a, K = DFT(b) / N.
 *   A  device complex [total], read only (packed like the state)
 *   K  device complex [total], written (same packing; K may not alias A)
 * Plans with CME_FWM_PADDED compute the truncated sum (alpha, beta, gamma
 * and mu within the instance's modes) on their 2N-point transforms.  FP32
 * plans with N > 8192: CME_EUNSUPPORTED.
 * Asynchronous on the plan's
 * stream.  Exposes steps a3-a5 of the solver for direct tests. */
int cme_fwm(cme_plan *plan, const void *A, void *K);

/* Discrete adjoint of cme_run (not in the paper: the gradient form of the
 * method).  Given the state A0 at step0 (device complex [total]) and the
 * cotangent gA_T = dL/dRe A(T) + i dL/dIm A(T) of the state after n_steps
 * steps, computes by checkpointed recomputation (segments of ckpt_every steps,
 * 0 = one segment):
 *   gA_0     device complex [total] or NULL: cotangent of A0 (written)
 *   g_omega  device FP64 [total] or NULL: += dL/domega'_mu
 *   g_kappa  device FP64 [total] or NULL: += dL/dkappa_mu
 *   g_ain    device FP64 [2 * batch] or NULL: += (dL/dRe A_in, dL/dIm A_in)
 * ckpt: device complex [n_steps / ckpt_every][total] as written by cme_run
 * with the same step0 / ckpt_every, or NULL (the adjoint then runs the
 * forward pass itself).  A0 is not modified.  Uses plan-owned device scratch
 * of 8 * ckpt_every * total complex values per record buffer, two when the
 * run has more than one segment (allocated on first use), and a plan-owned
 * stream on which each segment's recompute runs beside the reverse sweep of
 * the segment after it; the call stays ordered on the plan's stream.  FP64
 * RK4 with the cyclic sum and N <= 8192 only (CME_EUNSUPPORTED otherwise); a
 * size running the staged variant recomputes and reverses with a variant of
 * the same size that has a reverse sweep. */
int cme_adjoint(cme_plan *plan, const void *A0, const void *ckpt, int64_t step0,
                int64_t n_steps, int32_t ckpt_every, const void *gA_T, void *gA_0,
                double *g_omega, double *g_kappa, double *g_ain);

/* cme_adjoint without allocation, for callers that cannot allocate device
 * memory while they run (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and
 * restrictions as cme_adjoint, computed by the same kernels; it calls no
 * hipMalloc, hipFree or other allocating routine and creates no stream or
 * event.  Its working memory is the library's fixed device array of
 * CME_NOALLOC_SCRATCH_BYTES (one copy per GPU), laid out per call as
 *   one stage-record buffer   8 * K * total complex values
 *   kbar of the segment       4 * K * total (the FP64 two-level kernels)
 *   state and cotangent       2 * total
 *   segment starts            (ceil(n_steps / K) - 1) * total, only if ckpt is NULL
 * with K = min(ckpt_every, n_steps) (n_steps if ckpt_every is 0), each part
 * rounded up to 256 bytes; a larger request returns CME_ESCRATCH before
 * anything is enqueued.  The recompute of each segment and its reverse sweep
 * run one after the other on the plan's stream (cme_adjoint overlaps them on
 * a second stream), so it is slower.  Every call on a GPU uses the same
 * array: calls that overlap in time on one GPU (two streams, two threads)
 * race and must not be issued. */
int cme_adjoint_noalloc(cme_plan *plan, const void *A0, const void *ckpt, int64_t step0,
                        int64_t n_steps, int32_t ckpt_every, const void *gA_T, void *gA_0,
                        double *g_omega, double *g_kappa, double *g_ain);

/* Synchronise the plan's stream and report per-instance status into the host
 * array flags[batch] (0: finite; 1: a non-finite amplitude was seen).  Returns
 * CME_ENONFINITE if any flag is set, CME_OK otherwise.  Clears the flags. */
int cme_status(cme_plan *plan, int32_t *flags);

/* Change the stream later calls enqueue on. */
int cme_set_stream(cme_plan *plan, void *stream);

/* Kernel variants.  Each compiled kernel variant has an integer id.  A plan
 * uses one variant per mode count present in its batch: a fixed default, or
 * the fastest measured one with CME_INIT_AUTOTUNE, or the one forced by
 * cme_plan_select. */

/* Id of the variant the plan uses for mode count n_modes.  CME_EINVAL if the
 * plan has no instance of that size. */
int cme_plan_kernel(const cme_plan *plan, int32_t n_modes, int32_t *kernel_id);

/* Force variant kernel_id for mode count n_modes.  CME_EINVAL if the plan has
 * no instance of that size, CME_EUNSUPPORTED if the id is not a variant for
 * that size and the plan's precision. */
int cme_plan_select(cme_plan *plan, int32_t n_modes, int32_t kernel_id);

/* Ids of the variants compiled for a precision and mode count: writes up to
 * `cap` ids into ids[] and returns how many exist. */
int cme_list_kernels(int32_t precision, int32_t n_modes, int32_t *ids, int32_t cap);

/* Shape of variant kernel_id, written into info[0..min(cap, 10)-1]:
 * precision, modes N, modes per thread E, wave-local sub-transforms per wave
 * V, LDS padding shift (one pad element every 2^shift), kind (0: one
 * transform per team of threads, ordered by workgroup barriers, or at
 * wavefront scope when the workgroup is one wavefront, 1: two-level
 * transform with one workgroup barrier per transform, 2: two-level
 * transforms in four rounds of two interleaved transforms per RK4 step
 * (V = 2: N = 2048 as an 8-point step over each thread's modes and two
 * 256-point sub-transforms per wavefront),
 * 3: two-level transform with twiddles rebuilt on use, sized for two
 * wavefronts per SIMD, 4: split-step map, 5: RK4 with the padded sum on
 * N-point transforms for instances of N/2 modes, 6: four-step transforms
 * staged through global memory, several workgroups per instance, 7:
 * interaction-picture RK4 on the
 * two-level transform, 8: interaction-picture RK4 on the staged
 * transforms, 9: split-step map on the staged transforms, 10: RK4 with
 * the padded sum on the staged transforms, 11: RK4 with the padded sum on
 * the two-level transform with twiddles rebuilt on use, 12: interaction-
 * picture RK4 on that transform, 13: RK4 on the two-level transform with
 * the state, the stage input and the accumulated derivative in global
 * memory (one instance per workgroup; the plan holds a workspace of 2 N
 * complex values per instance), 14: interaction-picture RK4 on that layout
 * (a workspace of 3 N); the staged kinds 6, 8, 9, 10 carry the
 * row length N1 in the V field), instances per workgroup,
 * workgroup size, LDS bytes, and a kind-specific tuning field (kind 1:
 * sub-transform exchange, 0 all through LDS, 1 high lane bits in registers;
 * kind 2: VALU instructions scheduled per LDS instruction, + 16 when all
 * twiddles are held in registers, + 32 when the twiddled butterflies are
 * fused multiply-adds; kinds 6, 8, 9, 10: wavefronts per
 * workgroup; kind 13: operand prefetch distance of the stage arithmetic, + 16
 * when the sub-transform twiddles are formed from one base per pass, + 32 with
 * the state and + 64 with omega' held in registers; kind 14: the prefetch
 * distance).
 * Returns 10, or CME_EINVAL. */
int cme_kernel_info(int32_t kernel_id, int32_t *info, int32_t cap);

/* Release the plan and everything it owns.  NULL is accepted. */
int cme_destroy(cme_plan *plan);

/* Static description of a status code. */
const char *cme_strerror(int code);

/* Library version as major * 10000 + minor * 100 + patch. */
int cme_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CME_H */
