"""Seeded synthetic inputs for the Kerr-comb coupled mode equations (CME).

Hansson, Modotto & Wabnitz, "On the numerical simulation of Kerr frequency
combs using coupled mode equations", arXiv:1307.3428.

This module only *draws* inputs: per-mode losses kappa_mu, mode-frequency
offsets omega'_mu, pump, detuning and an initial comb state.  It contains no
step of the solver (no four-wave-mixing sum, no right-hand side, no time
stepping), and both the HIP library and the CPU oracle take its arrays as
plain inputs.

Conventions (one place for all of them):

* Units are those of Eq. (1): time tau is measured in the units in which the
  losses kappa_mu are given (kappa_0 = kappa at mu = 0, normally 1).  The
  integrated equation is Eq. (1) in the frame rotating with the pump and the
  FSR grid (the frame of Eq. (2), not rescaled):

      dA_mu/dtau = (-kappa_mu/2 + i(omega'_mu - sigma(tau))) A_mu
                   + delta_mu0 sqrt(kappa_ext) A_in + i g0 K_mu(A),

  with omega'_mu = omega_mu - omega_0 - mu D1 (the FSR offset of Eq. (2) read
  as mu*D1) and K_mu the cyclic four-wave-mixing sum over
  alpha - beta + gamma = mu (mod N).
* Storage is centred: array index i holds mode mu = i - N/2, so the pump
  mode mu = 0 sits at index N/2.
* "Anomalous" dispersion coefficients D2, D3 > 0 are mapped to
  omega'_mu = -(D2 mu^2/2 + D3 mu^3/6).  With the +i sign of the Kerr term of
  Eq. (1), modulation instability and bright solitons need a negative
  curvature of omega'_mu; the paper's own Fig. 1 example uses
  Omega_mu = -0.00625 mu^2.
* The pump is given as a multiple m of the parametric threshold
  |A_in|^2_th = kappa_0^3 / (8 g0 kappa_ext), i.e. f^2 = 1 in the
  normalisation f_0 = sqrt(8 g0 kappa_ext / kappa_0^3) A_in of Eq. (2).
  A_in is real and positive.
* Complex Gaussian noise of level s has independent real and imaginary parts
  of variance s^2/2 (E|n|^2 = s^2), added to every mode.
* Seeds: numpy.random.default_rng(13073428 + 100*c + i) for workload c and
  instance i; inside an instance the draws come in the order: parameters,
  noise real parts [N], noise imaginary parts [N].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

SEED_BASE = 13073428


def seed_for(config: int, instance: int) -> int:
    return SEED_BASE + 100 * config + instance


@dataclasses.dataclass
class Instance:
    """One resonator: the symbols of Eq. (1) in the rotating frame."""

    n_modes: int
    kappa: np.ndarray          # float64 [N]: total loss kappa_mu per mode
    omega: np.ndarray          # float64 [N]: omega'_mu = omega_mu - omega_0 - mu*D1
    kappa_ext: float           # external coupling loss
    g0: float                  # Kerr coefficient
    a_in: complex              # pump amplitude A_in (drives mu = 0 only)
    sigma0: float              # detuning sigma = omega_in - omega_0 at tau = 0
    sigma1: float              # detuning at tau >= tau_ramp
    tau_ramp: float            # length of the linear ramp (0: constant sigma0)
    a0: np.ndarray             # complex128 [N]: initial state A_mu(0)

    def copy(self) -> "Instance":
        return dataclasses.replace(
            self, kappa=self.kappa.copy(), omega=self.omega.copy(), a0=self.a0.copy()
        )


@dataclasses.dataclass
class Workload:
    name: str
    instances: List[Instance]
    h: float
    n_steps: int
    description: str = ""
    extra: Dict[str, object] = dataclasses.field(default_factory=dict)

    @property
    def batch(self) -> int:
        return len(self.instances)

    @property
    def total_modes(self) -> int:
        return int(sum(inst.n_modes for inst in self.instances))

    def mode_steps(self, n_steps: Optional[int] = None) -> int:
        return self.total_modes * int(self.n_steps if n_steps is None else n_steps)


@dataclasses.dataclass
class Packed:
    """Instances packed back to back (int64 offsets), as the solver takes them."""

    n_modes: np.ndarray        # int32 [B]
    offsets: np.ndarray        # int64 [B]
    kappa: np.ndarray          # float64 [sum N]
    omega: np.ndarray          # float64 [sum N]
    a0: np.ndarray             # complex128 [sum N]
    kappa_ext: np.ndarray      # float64 [B]
    g0: np.ndarray             # float64 [B]
    a_in: np.ndarray           # complex128 [B]
    sigma0: np.ndarray         # float64 [B]
    sigma1: np.ndarray         # float64 [B]
    tau_ramp: np.ndarray       # float64 [B]

    @property
    def batch(self) -> int:
        return int(self.n_modes.shape[0])

    @property
    def total(self) -> int:
        return int(self.kappa.shape[0])

    def slice(self, i: int) -> slice:
        o = int(self.offsets[i])
        return slice(o, o + int(self.n_modes[i]))


def pack(instances: Sequence[Instance]) -> Packed:
    ns = np.array([inst.n_modes for inst in instances], dtype=np.int32)
    offs = np.zeros(len(instances), dtype=np.int64)
    if len(instances) > 1:
        offs[1:] = np.cumsum(ns[:-1].astype(np.int64))
    cat = lambda name, dt: (
        np.concatenate([np.asarray(getattr(x, name), dtype=dt) for x in instances])
        if instances else np.zeros(0, dtype=dt)
    )
    vec = lambda name, dt: np.array([getattr(x, name) for x in instances], dtype=dt)
    return Packed(
        n_modes=ns, offsets=offs,
        kappa=cat("kappa", np.float64), omega=cat("omega", np.float64),
        a0=cat("a0", np.complex128),
        kappa_ext=vec("kappa_ext", np.float64), g0=vec("g0", np.float64),
        a_in=vec("a_in", np.complex128), sigma0=vec("sigma0", np.float64),
        sigma1=vec("sigma1", np.float64), tau_ramp=vec("tau_ramp", np.float64),
    )


# ----------------------------------------------------------------------------
# Building blocks of the recipes
# ----------------------------------------------------------------------------

def mu_grid(n: int) -> np.ndarray:
    """Mode numbers of the centred storage: index i holds mu = i - N/2."""
    return np.arange(n, dtype=np.float64) - (n // 2)


def dispersion_profile(n: int, d2: float, d3: float = 0.0) -> np.ndarray:
    """omega'_mu for anomalous coefficients D2, D3 (sign convention above)."""
    mu = mu_grid(n)
    return -(d2 * mu * mu / 2.0 + d3 * mu * mu * mu / 6.0)


def threshold_power(kappa0: float, g0: float, kappa_ext: float) -> float:
    """|A_in|^2 at f^2 = 1 (f_0 as defined under Eq. (2))."""
    return kappa0 ** 3 / (8.0 * g0 * kappa_ext)


def pump_for_multiple(m: float, kappa0: float, g0: float, kappa_ext: float) -> complex:
    return complex(math.sqrt(m * threshold_power(kappa0, g0, kappa_ext)), 0.0)


def cw_state(a_in: complex, sigma: float, omega0: float, kappa0: float,
             g0: float, kappa_ext: float) -> complex:
    """Single-mode (homogeneous) steady state on the lower branch.

    With only the pump mode populated the four-wave-mixing sum reduces to
    |A|^2 A, and a stationary A satisfies
        A = sqrt(kappa_ext) A_in / (kappa0/2 + i(sigma - omega0 - g0 |A|^2)).
    In the normalised variables of Eq. (2) the intracavity power x = 2 g0 |A|^2
    / kappa0 solves x (1 + (zeta - x)^2) = f^2 with zeta = 2(sigma - omega0) /
    kappa0; the lowest positive real root is taken.
    """
    s = math.sqrt(kappa_ext) * a_in
    if abs(s) == 0.0:
        return 0j
    zeta = 2.0 * (sigma - omega0) / kappa0
    f2 = 8.0 * g0 * kappa_ext * abs(a_in) ** 2 / kappa0 ** 3
    roots = np.roots([1.0, -2.0 * zeta, 1.0 + zeta * zeta, -f2])
    real = sorted(r.real for r in roots if abs(r.imag) <= 1e-9 * max(1.0, abs(r)) and r.real > 0)
    x = real[0]
    # one Newton polish in double precision
    for _ in range(3):
        g = x * (1.0 + (zeta - x) ** 2) - f2
        dg = 1.0 + (zeta - x) ** 2 - 2.0 * x * (zeta - x)
        if dg != 0.0:
            x -= g / dg
    p = kappa0 * x / (2.0 * g0)
    return s / complex(kappa0 / 2.0, sigma - omega0 - g0 * p)


def complex_noise(rng: np.random.Generator, n: int, level: float) -> np.ndarray:
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return (re + 1j * im) * (level / math.sqrt(2.0))


def sech_seed(n: int, zeta: float, d2: float, theta0: float, kappa0: float, g0: float) -> np.ndarray:
    """Mode amplitudes of the textbook NLS bright soliton sqrt(2 zeta) sech(sqrt(zeta/d2) theta).

    The profile lives on the 'time' grid theta_j = 2 pi j / N that the
    transform over the mode number defines (Eq. (4)); its mode amplitudes in
    the normalisation of Eq. (2) are (1/N) sum_j psi_j exp(-i theta_j mu),
    then rescaled to A = sqrt(kappa0 / (2 g0)) * A~.
    """
    theta = 2.0 * np.pi * np.arange(n) / n
    d = np.angle(np.exp(1j * (theta - theta0)))   # wrapped to (-pi, pi]
    psi = math.sqrt(2.0 * zeta) / np.cosh(math.sqrt(zeta / d2) * d)
    coeff = np.fft.fft(psi) / n                  # coefficient of mu = k (mod N)
    centred = np.fft.fftshift(coeff)             # index i <-> mu = i - N/2
    return centred * math.sqrt(kappa0 / (2.0 * g0))


def make_instance(n: int, *, kappa: float = 1.0, kappa_ext: float = 0.5, g0: float = 1.0,
                  d2: float = 0.0, d3: float = 0.0, omega: Optional[np.ndarray] = None,
                  pump_multiple: float = 1.0, sigma0: float = 0.0,
                  sigma1: Optional[float] = None, tau_ramp: float = 0.0,
                  noise: float = 0.0, rng: Optional[np.random.Generator] = None,
                  start: str = "cw", seed_shift: float = 0.0) -> Instance:
    kap = np.full(n, float(kappa))
    om = dispersion_profile(n, d2, d3) if omega is None else np.asarray(omega, np.float64).copy()
    a_in = pump_for_multiple(pump_multiple, kappa, g0, kappa_ext)
    a0 = np.zeros(n, dtype=np.complex128)
    if start in ("cw", "sech"):
        a0[n // 2] = cw_state(a_in, sigma0, om[n // 2], kappa, g0, kappa_ext)
    if start == "sech":
        zeta = 2.0 * sigma0 / kappa
        a0 += sech_seed(n, zeta, d2 / kappa, seed_shift, kappa, g0)
    if noise > 0.0:
        assert rng is not None
        a0 += complex_noise(rng, n, noise)
    return Instance(
        n_modes=n, kappa=kap, omega=om, kappa_ext=float(kappa_ext), g0=float(g0),
        a_in=a_in, sigma0=float(sigma0), sigma1=float(sigma0 if sigma1 is None else sigma1),
        tau_ramp=float(tau_ramp), a0=a0,
    )


# ----------------------------------------------------------------------------
# The workloads.  Each takes optional overrides of batch size / horizon so that
# tests can run the same recipe at reduced cost.
# ----------------------------------------------------------------------------

def plain_n128(n_steps: int = 20000) -> Workload:
    """N=128, mu = -64..63, kappa = 1, kappa_ext = 0.5, g0 = 1, D2 = 0.04,
    sigma = 2, pump 3x threshold, CW state + noise 1e-4, RK4 h = 1e-3."""
    rng = np.random.default_rng(seed_for(0, 0))
    inst = make_instance(128, d2=0.04, pump_multiple=3.0, sigma0=2.0, noise=1e-4, rng=rng)
    return Workload("plain_n128", [inst], h=1e-3, n_steps=n_steps,
                    description="single instance, N=128, CW + noise")


def turing_n128(n_steps: int = 100000) -> Workload:
    """Companion of plain_n128 inside the modulation-instability band:
    sigma = 0.5 (zeta = 1), pump 3x threshold -> Turing roll pattern."""
    rng = np.random.default_rng(seed_for(0, 1))
    inst = make_instance(128, d2=0.04, pump_multiple=3.0, sigma0=0.5, noise=1e-4, rng=rng)
    return Workload("turing_n128", [inst], h=1e-3, n_steps=n_steps,
                    description="single instance, N=128, Turing pattern from noise")


def soliton_ramp_n1024(n_steps: int = 400000) -> Workload:
    """N=1024, D2 = 0.004, D3 = 1e-5, sigma ramped -2 -> 8 over tau in [0, 200],
    pump 4x threshold, noise 1e-6, RK4 h = 5e-4."""
    rng = np.random.default_rng(seed_for(1, 0))
    inst = make_instance(1024, d2=0.004, d3=1e-5, pump_multiple=4.0, sigma0=-2.0,
                         sigma1=8.0, tau_ramp=200.0, noise=1e-6, rng=rng)
    return Workload("soliton_ramp_n1024", [inst], h=5e-4, n_steps=n_steps,
                    description="single instance, N=1024, detuning ramp")


def soliton_held_n1024(n_steps: int = 40000) -> Workload:
    """Companion of the ramp: fixed sigma = 1.5 (zeta = 3), pump 4x threshold,
    sech seed on the CW background -> a single soliton is held."""
    rng = np.random.default_rng(seed_for(1, 1))
    theta0 = float(rng.uniform(-np.pi, np.pi))
    inst = make_instance(1024, d2=0.004, d3=1e-5, pump_multiple=4.0, sigma0=1.5,
                         noise=1e-6, rng=rng, start="sech", seed_shift=theta0)
    return Workload("soliton_held_n1024", [inst], h=5e-4, n_steps=n_steps,
                    description="single soliton held at fixed detuning")


def sweep_n2048(batch: int = 256, n_steps: int = 50000, indices: Optional[Sequence[int]] = None) -> Workload:
    """B=256 instances of N=2048, D2 = 0.002, D3 = 2e-6, sigma_i evenly spaced
    in [-2, 10], pump 5x threshold, noise 1e-6, RK4 h = 5e-4.

    `indices` picks a subset of the full 256-instance sweep (same seeds)."""
    full = 256
    idx = list(range(batch)) if indices is None else list(indices)
    insts = []
    for i in idx:
        rng = np.random.default_rng(seed_for(2, i))
        sigma = -2.0 + 12.0 * i / (full - 1)
        insts.append(make_instance(2048, d2=0.002, d3=2e-6, pump_multiple=5.0, sigma0=sigma,
                                   noise=1e-6, rng=rng))
    return Workload("sweep_n2048", insts, h=5e-4, n_steps=n_steps,
                    description=f"detuning sweep, {len(insts)} x N=2048")


def uneven_octave(batch: int = 512, n_steps: int = 20000, indices: Optional[Sequence[int]] = None,
                  sizes: Sequence[int] = (1024, 2048, 4096, 8192)) -> Workload:
    """512 instances, N ~ U{1024, 2048, 4096, 8192}, D2 ~ U[1e-4, 1e-3],
    D3 ~ U[-1e-6, 1e-6], sigma ~ U[0, 15], pump ~ U[2, 20] x threshold,
    noise 1e-6, h = 2e-4."""
    idx = list(range(batch)) if indices is None else list(indices)
    insts = []
    for i in idx:
        rng = np.random.default_rng(seed_for(3, i))
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        d2 = float(rng.uniform(1e-4, 1e-3))
        d3 = float(rng.uniform(-1e-6, 1e-6))
        sigma = float(rng.uniform(0.0, 15.0))
        m = float(rng.uniform(2.0, 20.0))
        insts.append(make_instance(n, d2=d2, d3=d3, pump_multiple=m, sigma0=sigma,
                                   noise=1e-6, rng=rng))
    return Workload("uneven_octave", insts, h=2e-4, n_steps=n_steps,
                    description=f"{len(insts)} instances, N in {tuple(sizes)}")


def adjoint_n2048(n_steps: int = 5000, sigma: float = 6.0, config_id: int = 4,
                  n_modes: int = 2048) -> Workload:
    """N=2048, D2 = 0.002 (omega' = -0.001 mu^2), sigma = 6, pump 4x threshold,
    CW + sech seed (seeded position) + noise 1e-6, 5000 steps of h = 5e-4.

    extra['target'] is a seeded smooth sech^2 envelope t_mu for the loss
    L = sum_mu (|A_mu(T)|^2 - t_mu)^2."""
    rng = np.random.default_rng(seed_for(config_id, 0))
    theta0 = float(rng.uniform(-np.pi, np.pi))
    c_scale = float(rng.uniform(0.5, 1.5))
    mu_c = float(rng.uniform(-20.0, 20.0))
    width = float(rng.uniform(30.0, 80.0))
    inst = make_instance(n_modes, d2=0.002, pump_multiple=4.0, sigma0=sigma, noise=1e-6,
                         rng=rng, start="sech", seed_shift=theta0)
    mu = mu_grid(n_modes)
    side = np.abs(inst.a0) ** 2
    side[n_modes // 2] = 0.0
    target = c_scale * side.max() / np.cosh((mu - mu_c) / width) ** 2
    return Workload("adjoint_n2048" if config_id == 4 else f"adjoint_n{n_modes}_s{sigma:g}", [inst],
                    h=5e-4, n_steps=n_steps, description="gradient of a spectral loss",
                    extra={"target": target, "ckpt_every": 100})


def adjoint_soliton_n2048(n_steps: int = 5000) -> Workload:
    """Soliton-regime companion of adjoint_n2048: the same recipe at sigma = 3
    (zeta = 3, inside the soliton existence range at 4x threshold), so the
    seeded sech pulse is held rather than decaying."""
    return adjoint_n2048(n_steps=n_steps, sigma=3.0, config_id=6)


def fig1_ensemble(n_steps: Optional[int] = None, h: float = 1e-3, noise: float = 1e-6) -> Workload:
    """Parameters of the paper's Fig. 1: N = 256, normalised time 128 pi,
    Omega_mu = -0.00625 mu^2, kappa_mu = kappa_0, f0 in {1.01, 1.2, 1.8, 4} sqrt(2).

    In Eq. (1) units with kappa_0 = 1, g0 = 1, kappa_ext = 0.5: omega'_mu =
    Omega_mu kappa_0 / 2 and sigma = 0 (Omega_0 = 0), tau = 2 tau~ / kappa_0 =
    256 pi, and the pump multiple of threshold is f0^2 = 2 c^2 for f0 = c sqrt(2).
    The initial state (empty cavity + noise) and the step h are not given in
    the paper and are choices of this recipe.
    """
    tau_end = 2.0 * 128.0 * math.pi
    steps = int(round(tau_end / h)) if n_steps is None else n_steps
    insts = []
    for i, f in enumerate((1.01, 1.2, 1.8, 4.0)):
        rng = np.random.default_rng(seed_for(5, i))
        n = 256
        om = -0.00625 * mu_grid(n) ** 2 * 0.5
        m = 2.0 * f * f
        insts.append(make_instance(n, omega=om, pump_multiple=m, sigma0=0.0, noise=noise,
                                   rng=rng, start="zero"))
    return Workload("fig1_ensemble", insts, h=h, n_steps=steps,
                    description="Fig. 1 parameter set, 4 pump levels")


def random_batch(seed: int, sizes: Sequence[int], *, noise: float = 1e-3,
                 max_detuning: float = 40.0, sigma_range=(-2.0, 6.0), pump_range=(0.5, 6.0),
                 random_kappa: bool = True, random_phase_pump: bool = True) -> List[Instance]:
    """Generic seeded instances for parity tests: random per-mode kappa and
    omega' profiles (the dispersion is scaled with N so that max |omega'| stays
    below `max_detuning`), complex pump, detuning ramp, CW + noise start."""
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        half = max(1, n // 2)
        kap0 = float(rng.uniform(0.8, 1.2))
        kappa = kap0 * (1.0 + (0.2 * rng.uniform(-1, 1, n) if random_kappa else np.zeros(n)))
        kappa[n // 2] = kap0
        d2 = float(rng.uniform(0.05, 0.9)) * max_detuning * 2.0 / half ** 2
        d3 = float(rng.uniform(-1.0, 1.0)) * 0.1 * max_detuning * 6.0 / half ** 3
        omega = dispersion_profile(n, d2, d3)
        omega += rng.uniform(-0.05, 0.05, n)
        omega[n // 2] = 0.0
        kext = float(rng.uniform(0.2, 0.6)) * kap0
        g0 = float(rng.uniform(0.5, 1.5))
        m = float(rng.uniform(*pump_range))
        amp = math.sqrt(m * threshold_power(kap0, g0, kext))
        phase = float(rng.uniform(-np.pi, np.pi)) if random_phase_pump else 0.0
        a_in = amp * complex(math.cos(phase), math.sin(phase))
        s0 = float(rng.uniform(*sigma_range))
        s1 = float(rng.uniform(*sigma_range))
        ramp = float(rng.uniform(0.0, 2.0))
        a0 = complex_noise(rng, n, noise).astype(np.complex128)
        a0[n // 2] += cw_state(a_in, s0, 0.0, kap0, g0, kext)
        out.append(Instance(n_modes=int(n), kappa=kappa, omega=omega, kappa_ext=kext, g0=g0,
                            a_in=a_in, sigma0=s0, sigma1=s1, tau_ramp=ramp, a0=a0))
    return out


def loss_profile(n: int, kappa_abs0: float, abs_edge: float, kappa_ext0: float,
                 coupling_slope: float) -> np.ndarray:
    """Frequency-dependent total loss kappa_mu = absorption + coupling.

    The absorption rises quadratically toward both band edges,
    kappa_abs0 (1 + abs_edge x^2), and the coupling to the bus waveguide
    changes exponentially across the band, kappa_ext0 exp(coupling_slope x),
    with x = mu / (N/2).  At mu = 0 the coupling is kappa_ext0, the rate that
    carries the pump in.  (Sec. 3 names per-mode absorption and coupling as
    something the coupled mode form takes directly; the shapes are choices
    made here.)"""
    x = mu_grid(n) / max(1, n // 2)
    return kappa_abs0 * (1.0 + abs_edge * x * x) + kappa_ext0 * np.exp(coupling_slope * x)


def profile_instance(n: int, rng: np.random.Generator) -> Instance:
    """A seeded resonator with a frequency-dependent loss profile
    (loss_profile), anomalous dispersion scaled with N, pump 2-4x threshold
    and a detuning ramp, started from the CW state plus noise of total power
    ~0.1 so that every mode takes part in the four-wave mixing."""
    half = max(1, n // 2)
    kabs = float(rng.uniform(0.3, 0.6))
    kext = float(rng.uniform(0.3, 0.6))
    edge = float(rng.uniform(1.0, 4.0))
    slope = float(rng.uniform(-1.5, -0.3))
    kappa = loss_profile(n, kabs, edge, kext, slope)
    kap0 = float(kappa[n // 2])
    d2 = float(rng.uniform(10.0, 30.0)) * 2.0 / half ** 2
    omega = dispersion_profile(n, d2)
    g0 = float(rng.uniform(0.5, 1.5))
    a_in = pump_for_multiple(float(rng.uniform(2.0, 4.0)), kap0, g0, kext)
    s0 = float(rng.uniform(0.0, 3.0))
    s1 = float(rng.uniform(0.0, 3.0))
    a0 = complex_noise(rng, n, 0.3 / math.sqrt(n)).astype(np.complex128)
    a0[n // 2] += cw_state(a_in, s0, 0.0, kap0, g0, kext)
    return Instance(n_modes=int(n), kappa=kappa, omega=omega, kappa_ext=kext, g0=g0, a_in=a_in,
                    sigma0=s0, sigma1=s1, tau_ramp=float(rng.uniform(0.05, 0.2)), a0=a0)


WORKLOADS = {
    "plain_n128": plain_n128,
    "turing_n128": turing_n128,
    "soliton_ramp_n1024": soliton_ramp_n1024,
    "soliton_held_n1024": soliton_held_n1024,
    "sweep_n2048": sweep_n2048,
    "uneven_octave": uneven_octave,
    "adjoint_n2048": adjoint_n2048,
    "adjoint_soliton_n2048": adjoint_soliton_n2048,
    "fig1_ensemble": fig1_ensemble,
}
