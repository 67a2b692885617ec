// cme_api.hip -- host runtime behind the C ABI declared in include/cme.h.
//
// A plan owns: the per-instance device descriptors, copies of the per-mode
// loss and frequency arrays, one twiddle table exp(-2 pi i k / N) per mode
// count (computed on the host in long double), the per-size launch order,
// the non-finite flags, the staged kernels' workspace and, on first use, the
// adjoint's scratch.  Instances are grouped by transform length; each group
// runs as one persistent launch of the kernel variant chosen for that size
// (eight launches per step for the staged kernels), the groups concurrently
// on forked streams; the variant comes from a fixed table, or is the fastest
// measured once when CME_INIT_AUTOTUNE is set.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/cme.h"
#include "cme_internal.hpp"

using cme::DevInst;
using cme::Variant;

namespace cme {
const Variant *variants(int *count) {
  static const std::vector<Variant> all = [] {
    std::vector<Variant> v;
    int n = 0;
    const Variant *a = variants_duo(&n);
    v.insert(v.end(), a, a + n);
    a = variants_wave(&n);
    v.insert(v.end(), a, a + n);
    a = variants_lean(&n);
    v.insert(v.end(), a, a + n);
    a = variants_split(&n);
    v.insert(v.end(), a, a + n);
    a = variants_pad(&n);
    v.insert(v.end(), a, a + n);
    a = variants_team(&n);
    v.insert(v.end(), a, a + n);
    a = variants_duo_f32(&n);
    v.insert(v.end(), a, a + n);
    a = variants_wave_f32(&n);
    v.insert(v.end(), a, a + n);
    a = variants_stream(&n);
    v.insert(v.end(), a, a + n);
    a = variants_staged(&n);
    v.insert(v.end(), a, a + n);
    // at N = 8192 the staged RK4IP comes first (the wave kernel spills there)
    a = variants_staged_ip(&n);
    v.insert(v.end(), a, a + n);
    a = variants_rk4ip(&n);
    v.insert(v.end(), a, a + n);
    a = variants_staged_split(&n);
    v.insert(v.end(), a, a + n);
    a = variants_staged_pad(&n);
    v.insert(v.end(), a, a + n);
    return v;
  }();
  *count = (int)all.size();
  return all.data();
}
}  // namespace cme

// Fixed device scratch of cme_adjoint_noalloc: every GPU the library runs on
// holds one copy of it until the process ends.  Host code never uses this
// name as an address; it uses the per-device pointer from scratch_on().
static __device__ __align__(256) unsigned char scratch[CME_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on `device`, which must be current: looked up
// once per device and kept.
int scratch_on(int device, void **out) {
  static std::mutex mu;
  static void *addr[256] = {};
  if (device < 0 || device >= 256) return CME_ENODEVICE;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return CME_EHIP;
    addr[device] = ptr;
  }
  *out = addr[device];
  return CME_OK;
}

struct SizeClass {
  int n = 0;
  const Variant *var = nullptr;
  std::vector<int32_t> ids;
  int32_t *d_order = nullptr;
  void *d_tw = nullptr;
  // classes after the first run on their own plan-owned stream, forked from
  // and joined back into the caller's stream with events
  hipStream_t side = nullptr;
  hipEvent_t done = nullptr;
  // workspace of the staged variants (grown when such a variant is chosen)
  void *d_work = nullptr;
  size_t work_bytes = 0;
};

}  // namespace

struct cme_plan {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t batch = 0;
  int32_t precision = CME_F64;
  int32_t integrator = CME_RK4;
  int32_t fwm = CME_FWM_CYCLIC;
  double h = 0.0;
  uint32_t flags = 0;
  int64_t total = 0;
  size_t elem = 16;  // bytes per complex element
  std::vector<cme_instance> inst;
  DevInst *d_inst = nullptr;
  double *d_kappa = nullptr;
  double *d_omega = nullptr;
  int32_t *d_flags = nullptr;
  std::vector<SizeClass> classes;
  hipEvent_t fork = nullptr;  // recorded on the caller's stream before the side launches
  // adjoint scratch (grown on demand)
  void *d_stages = nullptr;
  size_t stages_bytes = 0;
  void *d_ckpt = nullptr;
  size_t ckpt_bytes = 0;
  void *d_state = nullptr;
  size_t state_bytes = 0;
  void *d_gA = nullptr;
  size_t gA_bytes = 0;
  // the adjoint's second stage-record buffer, and the stream and events that
  // let a segment's recompute run beside the previous segment's reverse sweep
  void *d_stages2 = nullptr;
  size_t stages2_bytes = 0;
  void *d_kbar = nullptr;   // kbar_s of a segment for the parameter cotangents
  size_t kbar_bytes = 0;
  hipStream_t adj_stream = nullptr;
  hipEvent_t adj_entry = nullptr;
  hipEvent_t rec_done[2] = {nullptr, nullptr};
  hipEvent_t rev_done[2] = {nullptr, nullptr};
  // this device's copy of the library's fixed scratch array (cme_adjoint_noalloc)
  void *d_scratch = nullptr;
};

namespace {

#define HIP_TRY(expr)                     \
  do {                                    \
    if ((expr) != hipSuccess) return CME_EHIP; \
  } while (0)

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

const Variant *all_variants(int *count) { return cme::variants(count); }

// kinds 4 and 9 step the split-step map, kinds 5, 10, 11 RK4 with the padded sum,
// kinds 7, 8, 12 interaction-picture RK4, all others RK4 with the cyclic sum;
// `integrator` encodes both choices as integrator + 16 fwm
bool integrates(const Variant &v, int integrator) {
  const int fwm = integrator >> 4, integ = integrator & 15;
  if (fwm == CME_FWM_PADDED) return v.kind == 5 || v.kind == 10 || v.kind == 11;
  if (v.kind == 5 || v.kind == 10 || v.kind == 11) return false;
  if (v.kind == 4 || v.kind == 9) return integ == CME_SPLIT_STEP;
  if (v.kind == 7 || v.kind == 8 || v.kind == 12 || v.kind == 14) return integ == CME_RK4IP;
  return integ == CME_RK4;
}

// Default kernel of a size when the plan is not autotuned: the first
// variant of that size in table order (the paired-transform kernels come
// first; their tables list the preferred shape first).
const Variant *default_variant(int precision, int n, int integrator) {
  int cnt = 0;
  const Variant *v = all_variants(&cnt);
  for (int i = 0; i < cnt; ++i)
    if (v[i].precision == precision && v[i].n == n && integrates(v[i], integrator)) return &v[i];
  return nullptr;
}

// Classic RK4 (cyclic sum) at N = 8192, by measured crossover (us per step
// for the whole class, per-mode kappa):
//   FP64: the staged kernels spread each instance over many CUs and win
//   for small classes (four-wave workgroups: 42.7 at 1 instance, 45.6 at 8,
//   49.1 at 16, 53.1 at 24, 57.1 at 32); rk4_stream in the 16 x 512 layout,
//   one instance per CU with the state in global memory, from 12 on (47.2
//   at 1, 47.1 at 8 to 32, 54.0 at 128);
//   FP32: rk4_stream at every size (27.3 at 1 to 27.4 at 128, against
//   38.3 ... 38.8 for the one-transform wave kernel, which spills).
// RK4IP at N = 8192:
//   FP64: rk4ip_stream at every size (44.3 at 1, 48.6 at 64, 52.6 at 128
//   instances, against 58.4, 77.9 and 96.5 for the staged kernels and 96 to
//   126 for the one-transform wave kernel);
//   FP32: the wave kernel, its state in registers, for small classes (30.9
//   at 16, 31.2 at 64, 35.0 at 100), rk4ip_stream from 80 on (32.0 at 16,
//   32.2 at 64, 32.9 at 100, 33.2 at 128, against 39.0 for the wave
//   kernel, whose spill traffic grows with the class).
const Variant *class_default(int precision, int n, int integrator, size_t count) {
  const Variant *v = default_variant(precision, n, integrator);
  if (n != 8192 || (integrator != CME_RK4 && integrator != CME_RK4IP)) return v;
  int cnt = 0;
  const Variant *all = all_variants(&cnt);
  auto find = [&](int kind, int threads) -> const Variant * {
    for (int i = 0; i < cnt; ++i)
      if (all[i].precision == precision && all[i].n == n && all[i].kind == kind &&
          (threads == 0 || all[i].threads == threads))
        return &all[i];
    return nullptr;
  };
  const Variant *pick = nullptr;
  if (integrator == CME_RK4IP)
    pick = precision == CME_F32 && count < 80 ? find(7, 0) : find(14, 0);
  else if (precision == CME_F64) pick = count < 12 ? find(6, 256) : find(13, 0);
  else pick = find(13, 0);
  return pick ? pick : v;
}

// compiled variants for a precision and size; integrator < 0: any
std::vector<const Variant *> candidates(int precision, int n, int integrator) {
  int cnt = 0;
  const Variant *v = all_variants(&cnt);
  std::vector<const Variant *> out;
  for (int i = 0; i < cnt; ++i)
    if (v[i].precision == precision && v[i].n == n &&
        (integrator < 0 || integrates(v[i], integrator)))
      out.push_back(&v[i]);
  return out;
}

int variant_id(const Variant *x) {
  int cnt = 0;
  const Variant *v = all_variants(&cnt);
  return (int)(x - v);
}

// Classic RK4 stability polynomial R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24.
double rk4_growth(double zr, double zi) {
  // Horner in complex arithmetic
  double pr = 1.0 / 24.0, pi = 0.0;
  const double c[4] = {1.0 / 6.0, 0.5, 1.0, 1.0};
  for (double ck : c) {
    const double nr = pr * zr - pi * zi + ck, ni = pr * zi + pi * zr;
    pr = nr;
    pi = ni;
  }
  return std::sqrt(pr * pr + pi * pi);
}

int upload_twiddles(int n, int precision, void **out) {
  const size_t elem = precision == CME_F64 ? 16 : 8;
  std::vector<unsigned char> host(elem * (size_t)n);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int k = 0; k < n; ++k) {
    const long double ang = -two_pi * (long double)k / (long double)n;
    const long double c = cosl(ang), s = sinl(ang);
    if (precision == CME_F64) {
      double v[2] = {(double)c, (double)s};
      std::memcpy(&host[elem * k], v, 16);
    } else {
      float v[2] = {(float)c, (float)s};
      std::memcpy(&host[elem * k], v, 8);
    }
  }
  HIP_TRY(hipMalloc(out, host.size()));
  HIP_TRY(hipMemcpy(*out, host.data(), host.size(), hipMemcpyHostToDevice));
  return CME_OK;
}

int grow(void **p, size_t *have, size_t need) {
  if (*have >= need) return CME_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  if (hipMalloc(p, need) != hipSuccess) {
    *p = nullptr;
    return CME_ENOMEM;
  }
  *have = need;
  return CME_OK;
}

// workspace a variant needs for a class, allocated before it first runs
int ensure_work(const cme_plan *p, SizeClass &c, const Variant *v) {
  if (v->work == 0) return CME_OK;
  return grow(&c.d_work, &c.work_bytes,
              p->elem * (size_t)v->work * (size_t)c.n * c.ids.size());
}

// the variant a class uses for the adjoint: its own if that has a reverse
// sweep, else the first compiled variant of its size that has one
const Variant *adjoint_variant(const cme_plan *p, const SizeClass &c) {
  if (c.var->adj) return c.var;
  for (const Variant *v : candidates(p->precision, c.n, p->integrator + 16 * p->fwm))
    if (v->adj) return v;
  return nullptr;
}

void free_plan(cme_plan *p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  for (auto &c : p->classes) {
    if (c.d_order) (void)hipFree(c.d_order);
    if (c.d_tw) (void)hipFree(c.d_tw);
    if (c.d_work) (void)hipFree(c.d_work);
    if (c.done) (void)hipEventDestroy(c.done);
    if (c.side) (void)hipStreamDestroy(c.side);
  }
  if (p->fork) (void)hipEventDestroy(p->fork);
  hipEvent_t evs[] = {p->adj_entry, p->rec_done[0], p->rec_done[1], p->rev_done[0], p->rev_done[1]};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  if (p->adj_stream) (void)hipStreamDestroy(p->adj_stream);
  void *bufs[] = {p->d_inst, p->d_kappa, p->d_omega, p->d_flags, p->d_stages,
                  p->d_ckpt, p->d_state, p->d_gA, p->d_stages2, p->d_kbar};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  (void)hipSetDevice(cur);
  delete p;
}

cme::RunArgs run_args(const cme_plan *p, const SizeClass &c, void *A, int64_t step0,
                      int64_t n_steps, int32_t ckpt_every, void *ckpt, void *stages) {
  cme::RunArgs a{};
  a.inst = p->d_inst;
  a.order = c.d_order;
  a.count = (int32_t)c.ids.size();
  a.ckpt_every = ckpt ? ckpt_every : 0;
  a.A = A;
  a.kappa = p->d_kappa;
  a.omega = p->d_omega;
  a.twiddle = c.d_tw;
  a.h = p->h;
  a.step0 = step0;
  a.n_steps = n_steps;
  a.ckpt = ckpt;
  a.total = p->total;
  a.flags = p->d_flags;
  a.stages = stages;
  a.work = c.d_work;
  return a;
}

// One launch per size class.  The classes touch disjoint instances, so all
// but the first run on side streams that wait for everything enqueued before
// on the caller's stream and are joined back into it: the classes share the
// chip, and the call stays ordered on the caller's stream (and capturable
// into a graph, where it becomes parallel branches).
// (on `base`, the plan's stream unless the adjoint's own stream is given)
// Fork the side streams of classes 1..nc-1 from `base`; returns how many
// were forked (a failure part way leaves the earlier ones forked).
size_t fork_classes(cme_plan *p, hipStream_t base, int *rc) {
  const size_t nc = p->classes.size();
  *rc = CME_OK;
  if (nc <= 1) return 0;
  if (hipEventRecord(p->fork, base) != hipSuccess) {
    *rc = CME_EHIP;
    return 0;
  }
  size_t forked = 0;
  for (size_t i = 1; i < nc; ++i, ++forked)
    if (hipStreamWaitEvent(p->classes[i].side, p->fork, 0) != hipSuccess) {
      *rc = CME_EHIP;
      break;
    }
  return forked;
}

// Join the first `forked` side streams back into `base`, also after a
// failure, so that no fork is left open (under graph capture, an unjoined
// fork invalidates the capture).
int join_classes(cme_plan *p, hipStream_t base, size_t forked) {
  int rc = CME_OK;
  for (size_t i = 1; i <= forked; ++i)
    if (hipEventRecord(p->classes[i].done, p->classes[i].side) != hipSuccess ||
        hipStreamWaitEvent(base, p->classes[i].done, 0) != hipSuccess)
      rc = CME_EHIP;
  return rc;
}

int launch_forward(cme_plan *p, void *A, int64_t step0, int64_t n_steps, int32_t ckpt_every,
                   void *ckpt, void *stages, hipStream_t base) {
  const size_t nc = p->classes.size();
  int rc = CME_OK;
  const size_t forked = fork_classes(p, base, &rc);
  for (size_t i = 0; i < nc && rc == CME_OK; ++i) {
    SizeClass &c = p->classes[i];
    const cme::RunArgs a = run_args(p, c, A, step0, n_steps, ckpt_every, ckpt, stages);
    if (c.var->fwd(a, i == 0 ? base : c.side) != hipSuccess) rc = CME_EHIP;
  }
  const int jr = join_classes(p, base, forked);
  return rc != CME_OK ? rc : jr;
}

int launch_forward(cme_plan *p, void *A, int64_t step0, int64_t n_steps, int32_t ckpt_every,
                   void *ckpt, void *stages) {
  return launch_forward(p, A, step0, n_steps, ckpt_every, ckpt, stages, p->stream);
}

// the adjoint's stream and events, created on first use (default priority)
int adjoint_streams(cme_plan *p) {
  if (p->adj_stream) return CME_OK;
  HIP_TRY(hipStreamCreateWithFlags(&p->adj_stream, hipStreamNonBlocking));
  hipEvent_t *evs[] = {&p->adj_entry, &p->rec_done[0], &p->rec_done[1], &p->rev_done[0],
                       &p->rev_done[1]};
  for (hipEvent_t *e : evs) HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
  return CME_OK;
}

// Time every compiled variant of each size on plan-owned zero state and keep
// the fastest: two short warm-up launches per variant, then two round-robin
// passes of one launch of about 8 ms per variant, the faster pass counting.
// Runs at init on the plan's stream.
int autotune(cme_plan *p) {
  void *state = nullptr;
  const size_t bytes = p->elem * (size_t)p->total;
  HIP_TRY(hipMalloc(&state, bytes));
  int rc = CME_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = CME_EHIP;
  if (rc == CME_OK && hipMemsetAsync(state, 0, bytes, p->stream) != hipSuccess) rc = CME_EHIP;
  // one launch of n steps of variant v, its time in ms (< 0: HIP error)
  auto timed = [&](SizeClass &c, const Variant *v, int64_t n) -> float {
    SizeClass tmp = c;
    tmp.var = v;
    const cme::RunArgs a = run_args(p, tmp, state, 0, n, 0, nullptr, nullptr);
    float ms = 0.f;
    if (hipEventRecord(e0, p->stream) != hipSuccess || v->fwd(a, p->stream) != hipSuccess ||
        hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return -1.f;
    return ms;
  };
  for (auto &c : p->classes) {
    if (rc != CME_OK) break;
    // warm-up length, scaled down for large sizes; the timed launches are
    // lengthened to about kTuneMs each (single launches of a millisecond
    // differ by several percent from run to run, more than the variants do)
    const int64_t base = std::max<int64_t>(4, (int64_t)(262144 / c.n));
    constexpr float kTuneMs = 8.f;
    // the default first
    std::vector<const Variant *> order{c.var};
    for (const Variant *v : candidates(p->precision, c.n, p->integrator + 16 * p->fwm))
      if (v != c.var) order.push_back(v);
    std::vector<int64_t> steps(order.size(), base);
    std::vector<float> per(order.size(), 1e30f);  // ms per step, the faster pass
    // two passes over all variants: in the first the clock is still rising
    // and each kernel's first launch also loads its code, so neither the
    // first variant nor the first launch of any decides alone
    for (int pass = 0; pass < 2 && rc == CME_OK; ++pass) {
      for (size_t j = 0; j < order.size(); ++j) {
        const Variant *v = order[j];
        if (pass == 0) {
          if ((rc = ensure_work(p, c, v)) != CME_OK) break;
          float warm = timed(c, v, base);
          if (warm >= 0.f) warm = timed(c, v, base);
          if (warm < 0.f) { rc = CME_EHIP; break; }
          steps[j] = base * std::min<int64_t>(
                                64, std::max<int64_t>(1, (int64_t)(kTuneMs / std::max(warm, 1e-3f))));
        }
        const float ms = timed(c, v, steps[j]);
        if (ms < 0.f) { rc = CME_EHIP; break; }
        per[j] = std::min(per[j], ms / (float)steps[j]);
      }
    }
    if (rc != CME_OK) break;
    // another variant replaces the best so far only when it is more than 5%
    // faster, so timing noise does not flip the choice
    float best = 1e30f;
    const Variant *pick = c.var;
    for (size_t j = 0; j < order.size(); ++j)
      if (per[j] < 0.95f * best) {
        best = per[j];
        pick = order[j];
      }
    c.var = pick;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(p->stream);
  (void)hipFree(state);
  if (rc == CME_OK && hipMemsetAsync(p->d_flags, 0, sizeof(int32_t) * p->batch, p->stream) != hipSuccess)
    rc = CME_EHIP;
  return rc;
}

int validate_instances(int32_t batch, const cme_instance *inst, int64_t *total) {
  std::vector<std::pair<int64_t, int64_t>> ranges;
  ranges.reserve(batch);
  int64_t tot = 0;
  for (int32_t b = 0; b < batch; ++b) {
    const cme_instance &x = inst[b];
    if (!is_pow2(x.n_modes) || x.n_modes < 16 || x.n_modes > 65536) return CME_EINVAL;
    if (x.reserved != 0 || x.mode_offset < 0) return CME_EINVAL;
    const double vals[] = {x.kappa_ext, x.g0, x.a_in_re, x.a_in_im, x.sigma0, x.sigma1, x.tau_ramp};
    for (double v : vals)
      if (!std::isfinite(v)) return CME_ENONFINITE;
    if (x.kappa_ext < 0.0 || x.tau_ramp < 0.0) return CME_EINVAL;
    ranges.emplace_back(x.mode_offset, x.mode_offset + x.n_modes);
    tot = std::max(tot, x.mode_offset + (int64_t)x.n_modes);
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second) return CME_EINVAL;
  *total = tot;
  return CME_OK;
}


// ---------------------------------------------------------------------------
// Adjoint (cme_adjoint and its allocation-free variant share all of this).

struct AdjCall {
  const void *A0;
  const void *ckpt;
  int64_t step0, n_steps;
  int32_t ckpt_every;
  const void *gA_T;
  void *gA_0;
  double *g_omega, *g_kappa, *g_ain;
};

struct AdjShape {
  int64_t K = 0, nseg = 0;
  size_t vec = 0;          // bytes of one packed state
  size_t stage_bytes = 0;  // one stage-record buffer: u_s and a_s of K steps
  size_t kbar_bytes = 0;   // kbar_s of K steps (0: no class stores them)
  size_t ckpt_bytes = 0;   // segment starts of the adjoint's own forward pass
};

struct AdjBuffers {
  void *stages[2];  // record buffers of alternate segments (equal when !overlap)
  void *kbar;
  void *state;
  void *gA;
  void *ckpt;
  bool overlap;     // recompute on the adjoint's stream beside the reverse sweep
};

int adjoint_check(const cme_plan *p, const AdjCall &c) {
  if (!p || !c.A0 || !c.gA_T || c.step0 < 0 || c.n_steps < 0 || c.ckpt_every < 0)
    return CME_EINVAL;
  if (c.ckpt && c.ckpt_every == 0) return CME_EINVAL;
  if (p->precision != CME_F64 || p->integrator != CME_RK4 || p->fwm != CME_FWM_CYCLIC)
    return CME_EUNSUPPORTED;
  for (const auto &cl : p->classes)
    if (!adjoint_variant(p, cl)) return CME_EUNSUPPORTED;
  if (c.n_steps == 0 && c.gA_0) {
    HIP_TRY(hipMemcpyAsync(c.gA_0, c.gA_T, p->elem * (size_t)p->total, hipMemcpyDefault,
                           p->stream));
  }
  return CME_OK;
}

// A class whose forward kernel has no reverse sweep (the staged kernels)
// recomputes and reverses with a variant of its size that has one; the
// forward kernels are restored when this goes out of scope.  Fixed storage:
// at most one class per power of two from 16 to 65536.
struct VariantSwap {
  cme_plan *p;
  const Variant *saved[16] = {};
  bool ok = true;
  explicit VariantSwap(cme_plan *q) : p(q) {
    if (p->classes.size() > 16) {
      ok = false;
      return;
    }
    for (size_t i = 0; i < p->classes.size(); ++i) {
      saved[i] = p->classes[i].var;
      p->classes[i].var = adjoint_variant(p, p->classes[i]);
    }
  }
  ~VariantSwap() {
    if (!ok) return;
    for (size_t i = 0; i < p->classes.size(); ++i) p->classes[i].var = saved[i];
  }
};

AdjShape adjoint_shape(const cme_plan *p, const AdjCall &c) {
  AdjShape s;
  s.K = c.ckpt_every > 0 ? std::min<int64_t>(c.ckpt_every, c.n_steps) : c.n_steps;
  s.nseg = (c.n_steps + s.K - 1) / s.K;
  s.vec = p->elem * (size_t)p->total;
  s.stage_bytes = s.vec * 8 * (size_t)s.K;
  bool kbar = false;
  for (const auto &cl : p->classes) kbar |= cl.var->adj_kbar != 0;
  s.kbar_bytes = kbar ? s.vec * 4 * (size_t)s.K : 0;
  s.ckpt_bytes = (!c.ckpt && s.nseg > 1) ? s.vec * (size_t)(s.nseg - 1) : 0;
  return s;
}

// Checkpointed recomputation and the reverse sweep, segment by segment from
// the last.  With b.overlap the recompute of segment s - 1 runs on the
// adjoint's stream beside the reverse sweep of segment s (two record
// buffers; events order each buffer's reuse and join every recompute back
// into the plan's stream); without it everything runs in order on the
// plan's stream with one record buffer.
int adjoint_run(cme_plan *p, const AdjCall &c, const AdjShape &s, const AdjBuffers &b) {
  const size_t vec = s.vec;
  const int64_t K = s.K, nseg = s.nseg, n_steps = c.n_steps, step0 = c.step0;
  const unsigned char *ck = (const unsigned char *)c.ckpt;
  int rc = CME_OK;
  if (!ck && nseg > 1) {
    // no checkpoints given: run the forward pass once, keeping segment starts
    HIP_TRY(hipMemcpyAsync(b.state, c.A0, vec, hipMemcpyDefault, p->stream));
    rc = launch_forward(p, b.state, step0, (nseg - 1) * K, (int32_t)K, b.ckpt, nullptr);
    if (rc != CME_OK) return rc;
    ck = (const unsigned char *)b.ckpt;
  }
  HIP_TRY(hipMemcpyAsync(b.gA, c.gA_T, vec, hipMemcpyDefault, p->stream));
  hipStream_t rs = b.overlap ? p->adj_stream : p->stream;  // the recompute's stream
  if (b.overlap) {
    HIP_TRY(hipEventRecord(p->adj_entry, p->stream));
    HIP_TRY(hipStreamWaitEvent(p->adj_stream, p->adj_entry, 0));
  }
  auto recompute = [&](int64_t seg) -> int {
    const int k = (int)(seg & 1);
    const int64_t first = seg * K;
    const int64_t len = std::min<int64_t>(K, n_steps - first);
    // the reverse sweep of segment seg + 2 read this buffer last
    if (b.overlap && seg + 2 < nseg) HIP_TRY(hipStreamWaitEvent(rs, p->rev_done[k], 0));
    const void *start = seg == 0 ? c.A0 : (const void *)(ck + (size_t)(seg - 1) * vec);
    HIP_TRY(hipMemcpyAsync(b.state, start, vec, hipMemcpyDefault, rs));
    const int r = launch_forward(p, b.state, step0 + first, len, 0, nullptr, b.stages[k], rs);
    if (r != CME_OK) return r;
    if (b.overlap) HIP_TRY(hipEventRecord(p->rec_done[k], rs));
    return CME_OK;
  };
  if (b.overlap && (rc = recompute(nseg - 1)) != CME_OK) return rc;
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int k = (int)(seg & 1);
    const int64_t first = seg * K;
    const int64_t len = std::min<int64_t>(K, n_steps - first);
    if (b.overlap) {
      if (seg >= 1 && (rc = recompute(seg - 1)) != CME_OK) return rc;
      HIP_TRY(hipStreamWaitEvent(p->stream, p->rec_done[k], 0));
    } else if ((rc = recompute(seg)) != CME_OK) {
      return rc;
    }
    for (auto &cl : p->classes) {
      cme::AdjArgs a{};
      a.inst = p->d_inst;
      a.order = cl.d_order;
      a.count = (int32_t)cl.ids.size();
      a.n_seg = (int32_t)len;
      a.stages = b.stages[k];
      a.gA = b.gA;
      a.kappa = p->d_kappa;
      a.omega = p->d_omega;
      a.twiddle = cl.d_tw;
      a.h = p->h;
      a.step_first = step0 + first;
      a.total = p->total;
      a.g_omega = c.g_omega;
      a.g_kappa = c.g_kappa;
      a.g_ain = c.g_ain;
      a.kbar = cl.var->adj_kbar ? b.kbar : nullptr;
      if (cl.var->adj(a, p->stream) != hipSuccess) return CME_EHIP;
      if (cl.var->adj_kbar && cme::launch_adj_params(cl.n, a, p->stream) != hipSuccess)
        return CME_EHIP;
    }
    if (b.overlap) HIP_TRY(hipEventRecord(p->rev_done[k], p->stream));
  }
  if (c.gA_0) HIP_TRY(hipMemcpyAsync(c.gA_0, b.gA, vec, hipMemcpyDefault, p->stream));
  return CME_OK;
}

}  // namespace

extern "C" {

int cme_version(void) { return 10000; }

const char *cme_strerror(int code) {
  switch (code) {
    case CME_OK: return "success";
    case CME_EINVAL: return "invalid argument";
    case CME_ENOMEM: return "out of memory";
    case CME_EHIP: return "HIP runtime error";
    case CME_EUNSTABLE: return "step size outside the RK4 stability region";
    case CME_ENONFINITE: return "non-finite value";
    case CME_EUNSUPPORTED: return "unsupported request";
    case CME_ENODEVICE: return "no gfx950 device available";
    case CME_ESCRATCH: return "request exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown status code";
  }
}

int cme_init(cme_plan **plan, int32_t batch, const cme_instance *inst, const double *kappa,
             const double *omega, int32_t precision, int32_t integrator, int32_t fwm, double h,
             void *stream, uint32_t flags) {
  if (!plan) return CME_EINVAL;
  *plan = nullptr;
  if (batch <= 0 || !inst || !kappa || !omega) return CME_EINVAL;
  if (precision != CME_F64 && precision != CME_F32) return CME_EINVAL;
  if ((integrator != CME_RK4 && integrator != CME_RK4IP && integrator != CME_SPLIT_STEP) ||
      (fwm != CME_FWM_CYCLIC && fwm != CME_FWM_PADDED))
    return CME_EINVAL;
  if (fwm == CME_FWM_PADDED && (precision != CME_F64 || integrator != CME_RK4))
    return CME_EUNSUPPORTED;
  if (!(h > 0.0) || !std::isfinite(h)) return CME_EINVAL;
  if (flags & ~(uint32_t)(CME_INIT_SKIP_STABILITY | CME_INIT_AUTOTUNE)) return CME_EINVAL;
  int64_t total = 0;
  int rc = validate_instances(batch, inst, &total);
  if (rc != CME_OK) return rc;
  // transforms of up to 65536 points; longer than 8192 only on the staged
  // kernels: FP64 with any integrator (classic RK4 for the padded sum) or
  // FP32 with classic RK4 or RK4IP
  for (int32_t b = 0; b < batch; ++b) {
    const int64_t tn = (fwm == CME_FWM_PADDED ? 2 : 1) * (int64_t)inst[b].n_modes;
    if (tn > 65536 || (tn > 8192 && precision != CME_F64 && integrator == CME_SPLIT_STEP))
      return CME_EUNSUPPORTED;
  }

  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return CME_ENODEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return CME_ENODEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return CME_ENODEVICE;
  void *scratch_ptr = nullptr;
  if (int r = scratch_on(device, &scratch_ptr); r != CME_OK) return r;

  // parameters to the host for validation (kappa / omega may be host or device)
  std::vector<double> hk((size_t)total), ho((size_t)total);
  if (hipMemcpy(hk.data(), kappa, sizeof(double) * total, hipMemcpyDefault) != hipSuccess ||
      hipMemcpy(ho.data(), omega, sizeof(double) * total, hipMemcpyDefault) != hipSuccess)
    return CME_EHIP;
  for (int32_t b = 0; b < batch; ++b) {
    const cme_instance &x = inst[b];
    const double lo = std::min(x.sigma0, x.sigma1), hi = std::max(x.sigma0, x.sigma1);
    for (int64_t i = x.mode_offset; i < x.mode_offset + x.n_modes; ++i) {
      if (!std::isfinite(hk[i]) || !std::isfinite(ho[i])) return CME_ENONFINITE;
      if ((flags & CME_INIT_SKIP_STABILITY) || integrator != CME_RK4) continue;
      for (double sg : {lo, hi}) {
        const double zr = -0.5 * hk[i] * h, zi = (ho[i] - sg) * h;
        if (rk4_growth(zr, zi) > 1.0 + 1e-12) return CME_EUNSTABLE;
      }
    }
  }

  cme_plan *p = new (std::nothrow) cme_plan();
  if (!p) return CME_ENOMEM;
  p->device = device;
  p->d_scratch = scratch_ptr;
  p->stream = (hipStream_t)stream;
  p->batch = batch;
  p->precision = precision;
  p->integrator = integrator;
  p->fwm = fwm;
  p->h = h;
  p->flags = flags;
  p->total = total;
  p->elem = precision == CME_F64 ? 16 : 8;
  p->inst.assign(inst, inst + batch);

  // Padded plans run each instance of N modes on a 2N-point transform: the
  // plan keeps kappa / omega' per transform point (the instance's values in
  // the middle half, kappa = 1, omega' = 0 elsewhere, where the kernels hold
  // the field at zero) and addresses the caller's state separately.
  const bool pad = fwm == CME_FWM_PADDED;
  const int tf = pad ? 2 : 1;  // transform points per mode
  std::vector<DevInst> dv((size_t)batch);
  std::vector<double> pk, po;
  int64_t ptotal = 0;
  for (int32_t b = 0; b < batch; ++b) {
    const cme_instance &x = inst[b];
    const double sk = std::sqrt(x.kappa_ext);
    const int nt = tf * x.n_modes;
    DevInst &d = dv[b];
    d.offset = pad ? ptotal : x.mode_offset;
    d.a_offset = x.mode_offset;
    d.pump_re = sk * x.a_in_re;
    d.pump_im = sk * x.a_in_im;
    d.g0n = x.g0 / (double)nt;
    d.sqrt_kext = sk;
    d.sigma0 = x.sigma0;
    d.sigma1 = x.sigma1;
    d.tau_ramp = x.tau_ramp;
    d.n = nt;
    {
      const double *kx = hk.data() + x.mode_offset;
      bool same = !pad;
      for (int i = 1; same && i < x.n_modes; ++i) same = kx[i] == kx[0];
      d.kappa_uniform = same ? 1 : 0;
      d.kappa0 = kx[0];
    }
    if (pad) {
      pk.resize((size_t)(ptotal + nt), 1.0);
      po.resize((size_t)(ptotal + nt), 0.0);
      for (int i = 0; i < x.n_modes; ++i) {
        pk[(size_t)(ptotal + x.n_modes / 2 + i)] = hk[(size_t)(x.mode_offset + i)];
        po[(size_t)(ptotal + x.n_modes / 2 + i)] = ho[(size_t)(x.mode_offset + i)];
      }
    }
    ptotal += nt;
  }
  const int64_t ktotal = pad ? ptotal : total;
  const double *kh = pad ? pk.data() : hk.data(), *oh = pad ? po.data() : ho.data();
  rc = CME_OK;
  if (hipMalloc((void **)&p->d_inst, sizeof(DevInst) * batch) != hipSuccess ||
      hipMalloc((void **)&p->d_kappa, sizeof(double) * ktotal) != hipSuccess ||
      hipMalloc((void **)&p->d_omega, sizeof(double) * ktotal) != hipSuccess ||
      hipMalloc((void **)&p->d_flags, sizeof(int32_t) * batch) != hipSuccess)
    rc = CME_ENOMEM;
  if (rc == CME_OK &&
      (hipMemcpy(p->d_inst, dv.data(), sizeof(DevInst) * batch, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(p->d_kappa, kh, sizeof(double) * ktotal, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(p->d_omega, oh, sizeof(double) * ktotal, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemset(p->d_flags, 0, sizeof(int32_t) * batch) != hipSuccess))
    rc = CME_EHIP;

  // size classes (by transform length), largest first (longest work first
  // when they share the chip)
  std::map<int, std::vector<int32_t>, std::greater<int>> groups;
  for (int32_t b = 0; b < batch; ++b) groups[tf * inst[b].n_modes].push_back(b);
  for (auto &g : groups) {
    if (rc != CME_OK) break;
    SizeClass c;
    c.n = g.first;
    c.ids = g.second;
    c.var = class_default(precision, c.n, integrator + 16 * fwm, c.ids.size());
    if (!c.var) {
      rc = CME_EUNSUPPORTED;
      break;
    }
    if (hipMalloc((void **)&c.d_order, sizeof(int32_t) * c.ids.size()) != hipSuccess) {
      rc = CME_ENOMEM;
      p->classes.push_back(c);
      break;
    }
    if (hipMemcpy(c.d_order, c.ids.data(), sizeof(int32_t) * c.ids.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
      rc = CME_EHIP;
    if (rc == CME_OK) rc = upload_twiddles(c.n, precision, &c.d_tw);
    if (rc == CME_OK) rc = ensure_work(p, c, c.var);
    if (rc == CME_OK && !p->classes.empty() &&
        (hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess))
      rc = CME_EHIP;
    p->classes.push_back(c);
  }
  if (rc == CME_OK && p->classes.size() > 1 &&
      hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess)
    rc = CME_EHIP;
  if (rc == CME_OK && (flags & CME_INIT_AUTOTUNE)) rc = autotune(p);
  if (rc != CME_OK) {
    free_plan(p);
    return rc;
  }
  *plan = p;
  return CME_OK;
}

int cme_set_stream(cme_plan *p, void *stream) {
  if (!p) return CME_EINVAL;
  p->stream = (hipStream_t)stream;
  return CME_OK;
}

int cme_run(cme_plan *p, void *A, int64_t step0, int64_t n_steps, int32_t ckpt_every,
            void *ckpt) {
  if (!p || !A || step0 < 0 || n_steps < 0 || ckpt_every < 0) return CME_EINVAL;
  if (ckpt && ckpt_every == 0) return CME_EINVAL;
  if (n_steps == 0) return CME_OK;
  if (n_steps > (int64_t)1 << 52) return CME_EINVAL;  // step index stays exact in FP64
  return launch_forward(p, A, step0, n_steps, ckpt_every, ckpt, nullptr);
}

int cme_step(cme_plan *p, void *A, int64_t step0) { return cme_run(p, A, step0, 1, 0, nullptr); }

int cme_fwm(cme_plan *p, const void *A, void *K) {
  if (!p || !A || !K) return CME_EINVAL;
  const size_t nc = p->classes.size();
  // every class is checked before anything is enqueued
  for (const SizeClass &c : p->classes)
    if (c.n > 8192 && (!c.d_work || p->precision != CME_F64)) return CME_EUNSUPPORTED;
  int rc = CME_OK;
  const size_t forked = fork_classes(p, p->stream, &rc);
  for (size_t i = 0; i < nc && rc == CME_OK; ++i) {
    SizeClass &c = p->classes[i];
    const cme::RunArgs a = run_args(p, c, const_cast<void *>(A), 0, 1, 0, K, nullptr);
    if (cme::launch_fwm(p->precision, c.n, p->fwm == CME_FWM_PADDED, a,
                        i == 0 ? p->stream : c.side) != hipSuccess)
      rc = CME_EHIP;
  }
  const int jr = join_classes(p, p->stream, forked);
  return rc != CME_OK ? rc : jr;
}

int cme_adjoint(cme_plan *p, const void *A0, const void *ckpt, int64_t step0, int64_t n_steps,
                int32_t ckpt_every, const void *gA_T, void *gA_0, double *g_omega,
                double *g_kappa, double *g_ain) {
  AdjCall c{A0, ckpt, step0, n_steps, ckpt_every, gA_T, gA_0, g_omega, g_kappa, g_ain};
  int rc = adjoint_check(p, c);
  if (rc != CME_OK || n_steps == 0) return rc;
  VariantSwap swap(p);
  if (!swap.ok) return CME_EUNSUPPORTED;
  const AdjShape s = adjoint_shape(p, c);
  if (s.K > (1 << 20)) return CME_EINVAL;
  AdjBuffers b{};
  if ((rc = grow(&p->d_stages, &p->stages_bytes, s.stage_bytes)) != CME_OK) return rc;
  if (s.nseg > 1 && (rc = grow(&p->d_stages2, &p->stages2_bytes, s.stage_bytes)) != CME_OK)
    return rc;
  if ((rc = grow(&p->d_state, &p->state_bytes, s.vec)) != CME_OK) return rc;
  if ((rc = grow(&p->d_gA, &p->gA_bytes, s.vec)) != CME_OK) return rc;
  if (s.kbar_bytes && (rc = grow(&p->d_kbar, &p->kbar_bytes, s.kbar_bytes)) != CME_OK) return rc;
  if (s.ckpt_bytes && (rc = grow(&p->d_ckpt, &p->ckpt_bytes, s.ckpt_bytes)) != CME_OK) return rc;
  if ((rc = adjoint_streams(p)) != CME_OK) return rc;
  b.stages[0] = p->d_stages;
  b.stages[1] = s.nseg > 1 ? p->d_stages2 : p->d_stages;
  b.kbar = p->d_kbar;
  b.state = p->d_state;
  b.gA = p->d_gA;
  b.ckpt = p->d_ckpt;
  b.overlap = true;
  return adjoint_run(p, c, s, b);
}

int cme_adjoint_noalloc(cme_plan *p, const void *A0, const void *ckpt, int64_t step0,
                        int64_t n_steps, int32_t ckpt_every, const void *gA_T, void *gA_0,
                        double *g_omega, double *g_kappa, double *g_ain) {
  AdjCall c{A0, ckpt, step0, n_steps, ckpt_every, gA_T, gA_0, g_omega, g_kappa, g_ain};
  int rc = adjoint_check(p, c);
  if (rc != CME_OK || n_steps == 0) return rc;
  void *base = p->d_scratch;
  if (!base) return CME_EHIP;
  VariantSwap swap(p);
  if (!swap.ok) return CME_EUNSUPPORTED;
  const AdjShape s = adjoint_shape(p, c);
  // one stage-record buffer (no overlap), then kbar, the state, the cotangent
  // and the forward pass's segment starts, each at a 256-byte boundary
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t need = up(s.stage_bytes) + up(s.kbar_bytes) + 2 * up(s.vec) + up(s.ckpt_bytes);
  if (s.K > (1 << 20) || need > (size_t)CME_NOALLOC_SCRATCH_BYTES) return CME_ESCRATCH;
  unsigned char *q = (unsigned char *)base;
  AdjBuffers b{};
  b.stages[0] = b.stages[1] = q;
  q += up(s.stage_bytes);
  b.kbar = s.kbar_bytes ? (void *)q : nullptr;
  q += up(s.kbar_bytes);
  b.state = q;
  q += up(s.vec);
  b.gA = q;
  q += up(s.vec);
  b.ckpt = s.ckpt_bytes ? (void *)q : nullptr;
  b.overlap = false;
  return adjoint_run(p, c, s, b);
}

int cme_status(cme_plan *p, int32_t *flags) {
  if (!p || !flags) return CME_EINVAL;
  HIP_TRY(hipStreamSynchronize(p->stream));
  HIP_TRY(hipMemcpy(flags, p->d_flags, sizeof(int32_t) * p->batch, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(p->d_flags, 0, sizeof(int32_t) * p->batch));
  for (int32_t b = 0; b < p->batch; ++b)
    if (flags[b]) return CME_ENONFINITE;
  return CME_OK;
}

// size class of an instance size (padded plans: twice the modes)
int class_size(const cme_plan *p, int32_t n_modes) {
  return p->fwm == CME_FWM_PADDED ? 2 * n_modes : n_modes;
}

int cme_plan_kernel(const cme_plan *p, int32_t n_modes, int32_t *kernel_id) {
  if (!p || !kernel_id) return CME_EINVAL;
  for (const auto &c : p->classes) {
    if (c.n != class_size(p, n_modes)) continue;
    *kernel_id = variant_id(c.var);
    return CME_OK;
  }
  return CME_EINVAL;
}

int cme_plan_select(cme_plan *p, int32_t n_modes, int32_t kernel_id) {
  if (!p) return CME_EINVAL;
  int cnt = 0;
  const Variant *v = all_variants(&cnt);
  for (auto &c : p->classes) {
    if (c.n != class_size(p, n_modes)) continue;
    if (kernel_id < 0 || kernel_id >= cnt || v[kernel_id].n != c.n ||
        v[kernel_id].precision != p->precision ||
        !integrates(v[kernel_id], p->integrator + 16 * p->fwm))
      return CME_EUNSUPPORTED;
    const int rc = ensure_work(p, c, &v[kernel_id]);
    if (rc != CME_OK) return rc;
    c.var = &v[kernel_id];
    return CME_OK;
  }
  return CME_EINVAL;
}

int cme_list_kernels(int32_t precision, int32_t n_modes, int32_t *ids, int32_t cap) {
  const auto c = candidates(precision, n_modes, -1);
  for (size_t i = 0; i < c.size() && (int32_t)i < cap; ++i)
    if (ids) ids[i] = variant_id(c[i]);
  return (int32_t)c.size();
}

int cme_kernel_info(int32_t kernel_id, int32_t *info, int32_t cap) {
  int cnt = 0;
  const Variant *v = all_variants(&cnt);
  if (kernel_id < 0 || kernel_id >= cnt || !info || cap < 1) return CME_EINVAL;
  const Variant &x = v[kernel_id];
  const int32_t vals[10] = {x.precision, x.n, x.e, x.v, x.ps, x.kind, x.ipb, x.threads,
                            x.lds_bytes, x.tp};
  for (int i = 0; i < 10 && i < cap; ++i) info[i] = vals[i];
  return 10;
}

int cme_destroy(cme_plan *p) {
  if (!p) return CME_OK;
  (void)hipStreamSynchronize(p->stream);
  free_plan(p);
  return CME_OK;
}

}  // extern "C"
