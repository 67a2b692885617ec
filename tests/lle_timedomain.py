"""Time-domain Lugiato-Lefever (driven, damped NLS) model on the fast-time grid.

Test infrastructure, independent of both the CPU oracle and the HIP library:
it holds no mode amplitudes and no four-wave-mixing sum, and it uses no FFT.

Sec. 2 states that the coupled mode equations are a discrete Fourier
expansion of a driven, damped NLS equation, and that the frequency-domain
split-step scheme is the time-domain split-step Fourier method of the LLE with
the roles of the two domains exchanged.  This module writes that NLS equation
down as a PDE in the fast time theta and semi-discretises it by Fourier
collocation on theta_j = 2 pi j / N:

    d psi/dt = (-kappa0/2 - i sigma(t)) psi
               + (kappa2/2) d^2 psi/dtheta^2
               + i (d2/2) d^2 psi/dtheta^2 + i (d4/24) d^4 psi/dtheta^4
               + sqrt(kappa_ext) A_in + i g0 |psi|^2 psi.

It is the image of Eq. (1) under psi(theta) = sum_mu A_mu e^{i mu theta} for
the mode profiles kappa_mu = kappa0 + kappa2 mu^2 and
omega'_mu = -(d2/2) mu^2 + (d4/24) mu^4: the operator -i d/dtheta acts as
mu on e^{i mu theta}.  Only even powers of the derivative are used, so that
the grid's Nyquist mode (mu = -N/2) keeps the same eigenvalue as in mode
space.  The derivatives are the closed-form periodic spectral differentiation
matrix (the second-derivative matrix of the periodic sinc interpolant on an
even grid, Trefethen, Spectral Methods in MATLAB, ch. 3), applied as dense
N x N products.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.linalg


def theta_grid(n: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(n) / n


def second_derivative_matrix(n: int) -> np.ndarray:
    """Periodic spectral second-derivative matrix on n (even) points.

    Diagonal -pi^2/(3 dx^2) - 1/6; off the diagonal
    -(-1)^(j-k) / (2 sin^2((j-k) dx / 2)), with dx = 2 pi / n."""
    if n % 2:
        raise ValueError("even grids only")
    dx = 2.0 * np.pi / n
    j = np.arange(n)
    d = j[:, None] - j[None, :]
    with np.errstate(divide="ignore"):
        off = -((-1.0) ** d) / (2.0 * np.sin(d * dx / 2.0) ** 2)
    m = np.where(d == 0, -np.pi ** 2 / (3.0 * dx * dx) - 1.0 / 6.0, off)
    return m


@dataclasses.dataclass
class LLE:
    """One resonator in the time domain; sigma(t) is the linear ramp
    sigma0 -> sigma1 over [0, tau_ramp], constant afterwards."""
    n: int
    kappa0: float
    kappa2: float
    d2: float
    d4: float
    kappa_ext: float
    a_in: complex
    g0: float
    sigma0: float
    sigma1: float
    tau_ramp: float

    def __post_init__(self):
        D2 = second_derivative_matrix(self.n)
        # the sigma-free linear operator: loss + dispersion
        self.op = (-0.5 * self.kappa0) * np.eye(self.n) + (0.5 * self.kappa2) * D2 \
            + 1j * ((0.5 * self.d2) * D2 + (self.d4 / 24.0) * (D2 @ D2))
        self.drive = math.sqrt(self.kappa_ext) * complex(self.a_in)
        self._expm_cache = {}

    # mode profiles of the same resonator (centred storage: index i <-> mu = i - N/2)
    def kappa_modes(self) -> np.ndarray:
        mu = np.arange(self.n) - self.n // 2
        return self.kappa0 + self.kappa2 * mu * mu

    def omega_modes(self) -> np.ndarray:
        mu = (np.arange(self.n) - self.n // 2).astype(np.float64)
        return -(0.5 * self.d2) * mu ** 2 + (self.d4 / 24.0) * mu ** 4

    def sigma(self, t: float) -> float:
        if not self.tau_ramp > 0.0:
            return self.sigma0
        s = min(max(t, 0.0), self.tau_ramp)
        return self.sigma0 + (self.sigma1 - self.sigma0) * (s / self.tau_ramp)

    def rhs(self, t: float, psi: np.ndarray) -> np.ndarray:
        return (self.op @ psi - 1j * self.sigma(t) * psi + self.drive
                + 1j * self.g0 * (np.abs(psi) ** 2) * psi)

    def rk4(self, psi: np.ndarray, h: float, n_steps: int, step0: int = 0) -> np.ndarray:
        """Classic RK4 with the step index kept as an integer (t = (step0+s) h)."""
        y = np.array(psi, dtype=np.complex128)
        for s in range(n_steps):
            t = (step0 + s) * h
            k1 = self.rhs(t, y)
            k2 = self.rhs(t + 0.5 * h, y + 0.5 * h * k1)
            k3 = self.rhs(t + 0.5 * h, y + 0.5 * h * k2)
            k4 = self.rhs(t + h, y + h * k3)
            y = y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        return y

    def _linear_propagator(self, sig: float, dt: float):
        """(exp(L dt), int_0^dt exp(L s) ds * drive) for L = op - i sig, from
        the exponential of the (n+1) x (n+1) block matrix [[L, drive 1], [0, 0]]."""
        key = (sig, dt)
        hit = self._expm_cache.get(key)
        if hit is None:
            n = self.n
            m = np.zeros((n + 1, n + 1), dtype=np.complex128)
            m[:n, :n] = self.op - 1j * sig * np.eye(n)
            m[:n, n] = self.drive
            e = scipy.linalg.expm(m * dt)
            hit = (e[:n, :n].copy(), e[:n, n].copy())
            self._expm_cache[key] = hit
        return hit

    def split_step(self, psi: np.ndarray, h: float, n_steps: int, step0: int = 0) -> np.ndarray:
        """Time-domain Strang split-step: exact linear half step (sigma frozen
        at the half step's midpoint), exact Kerr phase rotation
        psi_j <- psi_j exp(i g0 h |psi_j|^2), exact linear half step."""
        y = np.array(psi, dtype=np.complex128)
        for s in range(n_steps):
            t0 = (step0 + s) * h
            e, f = self._linear_propagator(self.sigma(t0 + 0.25 * h), 0.5 * h)
            y = e @ y + f
            y = y * np.exp(1j * self.g0 * h * np.abs(y) ** 2)
            e, f = self._linear_propagator(self.sigma(t0 + 0.75 * h), 0.5 * h)
            y = e @ y + f
        return y

    def sigma_integral(self, a: float, b: float) -> float:
        """Integral of sigma over [a, b] (trapezoid rule on the linear pieces)."""
        knots = [a] + ([self.tau_ramp] if a < self.tau_ramp < b else []) + [b]
        return sum(0.5 * (c - d) * (self.sigma(c) + self.sigma(d)) for d, c in zip(knots, knots[1:]))

    def rk4ip(self, psi: np.ndarray, h: float, n_steps: int, step0: int = 0) -> np.ndarray:
        """Interaction-picture RK4 in the time domain: the linear operator
        (loss, dispersion, detuning) through its exact half-step propagator
        expm(op h/2) exp(-i int sigma), the Kerr term and the drive through
        the RK4 stages (classic RK4 on the interaction-picture field centred
        at the middle of each step)."""
        half = self._expm_cache.get(("ip", h))
        if half is None:
            half = scipy.linalg.expm(self.op * (0.5 * h))
            self._expm_cache[("ip", h)] = half
        nl = lambda u: self.drive + 1j * self.g0 * (np.abs(u) ** 2) * u
        y = np.array(psi, dtype=np.complex128)
        for s in range(n_steps):
            t0 = (step0 + s) * h
            c1 = np.exp(-1j * self.sigma_integral(t0, t0 + 0.5 * h))
            c2 = np.exp(-1j * self.sigma_integral(t0 + 0.5 * h, t0 + h))
            p1 = lambda v: c1 * (half @ v)
            p2 = lambda v: c2 * (half @ v)
            yi = p1(y)
            k1 = p1(nl(y))
            k2 = nl(yi + 0.5 * h * k1)
            k3 = nl(yi + 0.5 * h * k2)
            k4 = nl(p2(yi + h * k3))
            y = p2(yi + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3)) + (h / 6.0) * k4
        return y


def synthesis_matrix(n: int) -> np.ndarray:
    """T[j, i] = exp(i mu_i theta_j), mu_i = i - N/2: psi = T A."""
    mu = np.arange(n) - n // 2
    return np.exp(1j * np.outer(theta_grid(n), mu))


def to_time(a_modes: np.ndarray) -> np.ndarray:
    return synthesis_matrix(len(a_modes)) @ a_modes


def to_modes(psi: np.ndarray) -> np.ndarray:
    n = len(psi)
    return synthesis_matrix(n).conj().T @ psi / n


def random_resonator(rng: np.random.Generator, n: int, *, ramp: bool = True,
                     kappa2: Optional[float] = None) -> LLE:
    """A seeded resonator with the LLE's mode profiles: anomalous d2 scaled
    with N (max |omega'| ~ 10-30 kappa0), small quartic term, optional
    quadratic loss, complex pump 1.5-5x threshold, detuning ramp."""
    half = n // 2
    kappa0 = float(rng.uniform(0.8, 1.2))
    d2 = float(rng.uniform(10.0, 30.0)) * 2.0 / half ** 2
    d4 = float(rng.uniform(-1.0, 1.0)) * 2.0 * 24.0 / half ** 4
    k2 = float(rng.uniform(0.0, 2.0)) / half ** 2 if kappa2 is None else kappa2
    kext = float(rng.uniform(0.2, 0.6)) * kappa0
    g0 = float(rng.uniform(0.5, 1.5))
    m = float(rng.uniform(1.5, 5.0))
    amp = math.sqrt(m * kappa0 ** 3 / (8.0 * g0 * kext))
    ph = float(rng.uniform(-np.pi, np.pi))
    s0 = float(rng.uniform(-1.0, 4.0))
    s1 = float(rng.uniform(-1.0, 4.0)) if ramp else s0
    return LLE(n=n, kappa0=kappa0, kappa2=k2, d2=d2, d4=d4, kappa_ext=kext,
               a_in=amp * complex(math.cos(ph), math.sin(ph)), g0=g0,
               sigma0=s0, sigma1=s1, tau_ramp=float(rng.uniform(0.05, 0.5)) if ramp else 0.0)
