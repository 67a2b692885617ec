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


# ---------------------------------------------------------------------------
# GPU (HIP solver through the C ABI)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cme():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1307_3428_amd import cme as C
    C.load_library()
    return C


def gpu_ip(C, p, h, steps, step0=0, precision=0, kid=None, ckpt_every=0):
    import torch
    with C.Plan(p, h, precision=precision, integrator=C.CME_RK4IP) as plan:
        n = int(p.n_modes[0])
        if kid is not None:
            plan.select(n, kid)
        A = plan.state(p.a0)
        ck = None
        if ckpt_every:
            ck = torch.zeros((steps // ckpt_every, p.total), dtype=A.dtype, device=A.device)
        plan.run(A, steps, step0=step0, ckpt_every=ckpt_every, ckpt=ck)
        torch.cuda.synchronize()
        st = plan.status()
        name = plan.kernel(n)["name"]
        out = A.cpu().numpy().astype(np.complex128)
        return out, (ck.cpu().numpy() if ck is not None else None), st, name


def _ip_params(precision):
    try:
        from paper_1307_3428_amd import cme as C
        return [(n, k) for n in (128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768, 65536)
                for k in C.cme_list_kernels(precision, n) if C.cme_kernel_info(k)["kind"] in (7, 8, 12, 14)]
    except Exception:
        return [(128, 0)]


@pytest.mark.gpu
@pytest.mark.parametrize("n,kid", _ip_params(0))
def test_gpu_rk4ip_variant_matches_oracle(cme, orc, n, kid):
    batch = 5 if cme.cme_kernel_info(kid)["instances_per_group"] > 1 else 2
    steps = 4
    if n >= 32768:   # the oracle's O(N^2) sum costs seconds per evaluation here
        batch, steps = 1, 2
    p = W.pack(nonlinear_batch(3000 + n, [n] * batch))
    h = 0.01
    y, _, st, name = gpu_ip(cme, p, h, steps, step0=5, kid=kid)
    ref = orc.rk4ip_run(p, h, steps, step0=5)
    errs = [rel_err(y[p.slice(b)], ref[p.slice(b)]) for b in range(batch)]
    print(name, errs, flush=True)
    assert max(errs) <= 1e-13 and not st.any()


@pytest.mark.gpu
@pytest.mark.parametrize("n,kid", _ip_params(1))
def test_gpu_rk4ip_fp32_variant_matches_fp64_oracle(cme, orc, n, kid):
    batch = 5 if cme.cme_kernel_info(kid)["instances_per_group"] > 1 else 2
    steps = 4
    if n >= 32768:   # the oracle's O(N^2) sum costs seconds per evaluation here
        batch, steps = 1, 2
    p = W.pack(nonlinear_batch(3100 + n, [n] * batch))
    h = 0.01
    y, _, st, name = gpu_ip(cme, p, h, steps, step0=5, precision=1, kid=kid)
    ref = orc.rk4ip_run(p, h, steps, step0=5)
    errs = [rel_err(y[p.slice(b)], ref[p.slice(b)]) for b in range(batch)]
    print(name, errs, flush=True)
    assert max(errs) <= 2e-6 and not st.any()


@pytest.mark.gpu
@pytest.mark.parametrize("n", [2048, 16384])
def test_gpu_rk4ip_undriven_linear_problem_is_exact(cme, n):
    """max |omega'| h ~ 10: the closed-form propagator, no oracle (N = 16384:
    the staged transforms)."""
    insts = stiff_linear_batch(7, n=n, batch=2)
    for b, inst in enumerate(insts):
        inst.omega = W.dispersion_profile(n, d2=(8e-3 + 1e-3 * b) * (2048 / n) ** 2)
    p = W.pack(insts)
    h, steps = 2e-3, 250
    T = h * steps
    assert max(np.abs(p.omega)) * h > 2 * math.sqrt(2)
    y, _, st, name = gpu_ip(cme, p, h, steps)
    for b, inst in enumerate(insts):
        exact = inst.a0 * np.exp(-0.5 * inst.kappa * T + 1j * (inst.omega * T - sigma_quad(inst, 0.0, T)))
        err = rel_err(y[p.slice(b)], exact)
        print(f"{name} instance {b}: vs closed form {err:.2e}")
        assert err <= 1e-11
    assert not st.any()


def _unstable_uneven(count):
    wl = W.uneven_octave(n_steps=1)
    bad = []
    for inst in wl.instances:
        for sg in (inst.sigma0, inst.sigma1):
            z = wl.h * (-0.5 * inst.kappa + 1j * (inst.omega - sg))
            if np.any(np.abs(1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24) > 1 + 1e-12):
                bad.append(inst)
                break
    return wl, bad[:count]


@pytest.mark.gpu
def test_gpu_rk4ip_runs_the_instances_classic_rk4_refuses(cme, orc):
    """Uneven-octave instances past the classic RK4 bound: cme_init refuses
    them for CME_RK4 and accepts them for CME_RK4IP; 10 steps against the
    oracle's RK4IP, then 2000 more stay finite with bounded power."""
    import torch
    wl, bad = _unstable_uneven(3)
    assert len(bad) == 3
    p = W.pack(bad)
    with pytest.raises(cme.CmeError):
        cme.Plan(p, wl.h)
    y, _, st, name = gpu_ip(cme, p, wl.h, 10)
    ref = orc.rk4ip_run(p, wl.h, 10)
    errs = [rel_err(y[p.slice(b)], ref[p.slice(b)]) for b in range(p.batch)]
    print(name, errs, flush=True)
    assert max(errs) <= 1e-12 and not st.any()
    with cme.Plan(p, wl.h, integrator=cme.CME_RK4IP) as plan:
        A = plan.state(p.a0)
        plan.run(A, 2000)
        torch.cuda.synchronize()
        a = A.cpu().numpy()
        assert not plan.status().any() and np.all(np.isfinite(a))
        for b, inst in enumerate(bad):
            # the Kerr and detuning terms conserve P = sum |A|^2, so
            # dP/dt <= -kappa_min P + 2 |s| sqrt(P) (s = sqrt(kappa_ext) A_in):
            # P stays below (2 |s| / kappa_min)^2 when it starts there
            bound = (2 * math.sqrt(inst.kappa_ext) * abs(inst.a_in) / inst.kappa.min()) ** 2
            assert np.sum(np.abs(inst.a0) ** 2) < bound
            assert np.sum(np.abs(a[p.slice(b)]) ** 2) < 1.001 * bound


@pytest.mark.gpu
def test_gpu_rk4ip_split_runs_and_checkpoints_are_bitwise(cme):
    import torch
    p = W.pack(nonlinear_batch(3200, [1024, 1024]))
    with cme.Plan(p, 0.004, integrator=cme.CME_RK4IP) as plan:
        A = plan.state(p.a0)
        ck = torch.zeros((3, p.total), dtype=A.dtype, device=A.device)
        plan.run(A, 12, step0=2, ckpt_every=4, ckpt=ck)
        B = plan.state(p.a0)
        mids = []
        for s in range(3):
            plan.run(B, 4, step0=2 + 4 * s)
            mids.append(B.clone())
        torch.cuda.synchronize()
        assert torch.equal(A, B)
        for s in range(3):
            assert torch.equal(ck[s], mids[s])


@pytest.mark.gpu
@pytest.mark.parametrize("n,steps,h", [(1024, 300, 2e-3), (4096, 100, 2e-3), (16384, 10, 5e-3)])
def test_gpu_rk4ip_longer_runs_match_oracle(cme, orc, n, steps, h):
    """Longer RK4IP runs against the oracle (the default kernel of each size:
    wave, lean, staged), with checkpoints."""
    batch = 2 if n <= 4096 else 1
    p = W.pack(nonlinear_batch(3300 + n, [n] * batch))
    y, ck, st, name = gpu_ip(cme, p, h, steps, ckpt_every=steps // 2)
    ref = orc.rk4ip_run(p, h, steps)
    mid = orc.rk4ip_run(p, h, steps // 2)
    for b in range(batch):
        err = rel_err(y[p.slice(b)], ref[p.slice(b)])
        cerr = rel_err(ck[0][p.slice(b)], mid[p.slice(b)])
        moved = rel_err(p.a0[p.slice(b)], ref[p.slice(b)])
        print(f"{name} N={n} instance {b}: {err:.2e}, checkpoint {cerr:.2e} (moved {moved:.2e})")
        assert err <= 1e-11 and cerr <= 1e-11 and moved > 0.1
    assert not st.any()
