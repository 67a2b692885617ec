"""Interaction-picture RK4 (RK4IP): oracle pins (CPU) and GPU parity.

RK4IP integrates the linear part of Eq. (1) (loss, dispersion, detuning)
exactly and takes only the four-wave-mixing term and the pump through the
RK4 stages, so the stiffness of the dispersion does not bound the step.

Pins of the oracle (no GPU): the undriven linear problem is solved exactly
(closed-form propagator, the detuning integrated piece by piece) at steps
far past classic RK4's stability bound; the driven linear problem converges
at fourth order to its closed form; the full problem converges at fourth
order and agrees with classic RK4 where both are accurate.
"""
import math

import numpy as np
import pytest

from paper_1307_3428_amd import workloads as W


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sigma_of(inst, t):
    if not inst.tau_ramp > 0:
        return inst.sigma0
    return inst.sigma0 + (inst.sigma1 - inst.sigma0) * min(max(t, 0.0), inst.tau_ramp) / inst.tau_ramp


def sigma_quad(inst, a, b):
    """Integral of the piecewise-linear sigma over [a, b]: the trapezoid rule
    on the pieces (exact for a linear integrand)."""
    knots = [a] + ([inst.tau_ramp] if a < inst.tau_ramp < b else []) + [b]
    return sum(0.5 * (c - d) * (sigma_of(inst, c) + sigma_of(inst, d)) for d, c in zip(knots, knots[1:]))


def stiff_linear_batch(seed, n=64, batch=3):
    """Undriven, Kerr-free instances with dispersion far past the classic
    RK4 bound at h = 2e-3 (max |omega'| h ~ 10) and a detuning ramp."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(batch):
        kappa = rng.uniform(0.5, 1.5, n)
        omega = W.dispersion_profile(n, d2=float(rng.uniform(2.0, 4.0)))
        a0 = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2 * n)
        out.append(W.Instance(n_modes=n, kappa=kappa, omega=omega, kappa_ext=0.5, g0=0.0, a_in=0j,
                              sigma0=float(rng.uniform(-2, 2)), sigma1=float(rng.uniform(2, 6)),
                              tau_ramp=float(rng.uniform(0.1, 0.3)), a0=a0))
    return out


def test_sigma_integral_matches_quadrature(orc):
    insts = stiff_linear_batch(1, n=16, batch=2)
    insts[1].tau_ramp = 0.0
    p = W.pack(insts)
    for b, inst in enumerate(insts):
        for a, c in ((0.0, 0.05), (0.07, 0.2), (0.15, 0.45), (0.5, 0.9)):
            assert abs(orc.sigma_integral(p, b, a, c) - sigma_quad(inst, a, c)) <= 1e-13


def test_rk4ip_undriven_linear_problem_is_exact(orc):
    insts = stiff_linear_batch(2)
    p = W.pack(insts)
    h, steps = 2e-3, 250
    T = h * steps
    assert max(np.abs(p.omega)) * h > 2 * math.sqrt(2)   # classic RK4 is unstable here
    y = orc.rk4ip_run(p, h, steps)
    for b, inst in enumerate(insts):
        exact = inst.a0 * np.exp(-0.5 * inst.kappa * T + 1j * (inst.omega * T - sigma_quad(inst, 0.0, T)))
        err = rel_err(y[p.slice(b)], exact)
        print(f"instance {b}: RK4IP vs closed form {err:.2e}")
        assert err <= 1e-11
    y_rk4, _ = orc.run(p, h, steps)
    assert not np.all(np.isfinite(y_rk4)) or np.abs(y_rk4).max() > 1e6


def test_rk4ip_driven_linear_problem_is_fourth_order(orc):
    """g0 = 0 with the pump: A_0(t) = e^{Lt} A_0(0) + s (e^{Lt} - 1) / L at the
    pump mode (constant detuning), every other mode free decay."""
    n = 16
    rng = np.random.default_rng(3)
    kappa = np.full(n, 1.0)
    omega = W.dispersion_profile(n, d2=0.5)
    a_in = 1.3 * np.exp(0.4j)
    a0 = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 0.1
    inst = W.Instance(n_modes=n, kappa=kappa, omega=omega, kappa_ext=0.5, g0=0.0, a_in=a_in,
                      sigma0=1.5, sigma1=1.5, tau_ramp=0.0, a0=a0)
    p = W.pack([inst])
    T = 1.0
    L = -0.5 * kappa + 1j * (omega - 1.5)
    exact = a0 * np.exp(L * T)
    s = math.sqrt(0.5) * a_in
    exact[n // 2] += s * (np.exp(L[n // 2] * T) - 1) / L[n // 2]
    errs = [rel_err(orc.rk4ip_run(p, T / k, k), exact) for k in (10, 20, 40)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("errors", errs, "orders", rates)
    assert all(3.8 < r < 4.2 for r in rates)


def nonlinear_batch(seed, sizes):
    insts = W.random_batch(seed, sizes, noise=1.0)
    for inst in insts:
        inst.a0 = inst.a0 / math.sqrt(inst.n_modes)
        inst.a0[inst.n_modes // 2] += 0.5
    return insts


def test_rk4ip_full_problem_is_fourth_order(orc):
    p = W.pack(nonlinear_batch(4, [32]))
    T = 0.2
    ref = orc.rk4ip_run(p, T / 640, 640)
    errs = [rel_err(orc.rk4ip_run(p, T / k, k), ref) for k in (10, 20, 40)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("errors", errs, "orders", rates)
    assert all(3.7 < r < 4.3 for r in rates)


def test_rk4ip_agrees_with_classic_rk4_where_both_are_accurate(orc):
    """Two fourth-order methods for the same solution: their difference is
    small and falls 16x when h halves."""
    p = W.pack(nonlinear_batch(5, [64, 128]))
    T = 0.3
    diffs = []
    for steps in (150, 300):
        y_ip = orc.rk4ip_run(p, T / steps, steps)
        y_rk, _ = orc.run(p, T / steps, steps)
        diffs.append([rel_err(y_ip[p.slice(b)], y_rk[p.slice(b)]) for b in range(p.batch)])
        moved = [rel_err(p.a0[p.slice(b)], y_rk[p.slice(b)]) for b in range(p.batch)]
    print("RK4IP vs RK4", diffs, "moved", moved)
    for b in range(p.batch):
        assert diffs[1][b] <= 1e-7 and moved[b] > 1e-2
        assert 12.0 < diffs[0][b] / diffs[1][b] < 20.0
