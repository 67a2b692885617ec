"""GPU edge cases of the boundary: empty and short runs, checkpoint
intervals that do not divide the run, the stability refusal and its
override, non-finite parameters, the zero state under every integrator,
the smallest and largest sizes in one ragged plan, many tiny instances,
and a caller-chosen stream."""
import math

import numpy as np
import pytest

from paper_1307_3428_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cme():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1307_3428_amd import cme as C
    C.load_library()
    return C


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def moderate_batch(seed, sizes):
    insts = W.random_batch(seed, sizes, noise=1.0)
    for inst in insts:
        inst.a0 = inst.a0 / math.sqrt(inst.n_modes)
        inst.a0[inst.n_modes // 2] += 0.5
    return insts


def test_zero_steps_and_short_checkpointed_runs(cme):
    import torch
    p = W.pack(moderate_batch(1, [256, 2048]))
    with cme.Plan(p, 0.005) as plan:
        A = plan.state(p.a0)
        A0 = A.clone()
        plan.run(A, 0)
        torch.cuda.synchronize()
        assert torch.equal(A, A0)
        # fewer steps than the checkpoint interval: no row written
        ck = torch.full((1, p.total), 7.0 + 7.0j, dtype=A.dtype, device=A.device)
        plan.run(A, 3, ckpt_every=5, ckpt=ck)
        # an interval that does not divide the run: rows after 4 and 8 steps
        B = A0.clone()
        ck2 = torch.zeros((2, p.total), dtype=A.dtype, device=A.device)
        plan.run(B, 10, ckpt_every=4, ckpt=ck2)
        C_ = A0.clone()
        plan.run(C_, 4)
        r1 = C_.clone()
        plan.run(C_, 4, step0=4)
        r2 = C_.clone()
        plan.run(C_, 2, step0=8)
        torch.cuda.synchronize()
        assert torch.equal(ck2[0], r1) and torch.equal(ck2[1], r2) and torch.equal(B, C_)
        assert torch.all(ck == 7.0 + 7.0j)


def test_step_equals_one_step_run(cme):
    import torch
    p = W.pack(moderate_batch(2, [512, 1024]))
    with cme.Plan(p, 0.005) as plan:
        A = plan.state(p.a0)
        B = A.clone()
        for s in range(3):
            plan.step(A, 7 + s)
        plan.run(B, 3, step0=7)
        torch.cuda.synchronize()
        assert torch.equal(A, B)


def test_stability_refusal_and_override(cme):
    inst = W.random_batch(3, [1024])[0]
    p = W.pack([inst])
    h_bad = 4.0 / np.abs(inst.omega).max()      # h max |omega'| = 4 > 2 sqrt 2
    with pytest.raises(cme.CmeError) as e:
        cme.Plan(p, h_bad)
    assert e.value.code == cme.CME_EUNSTABLE
    with cme.Plan(p, h_bad, flags=cme.CME_INIT_SKIP_STABILITY):
        pass
    # the exact-linear integrators have no such bound
    with cme.Plan(p, h_bad, integrator=cme.CME_RK4IP):
        pass
    with cme.Plan(p, h_bad, integrator=cme.CME_SPLIT_STEP):
        pass


@pytest.mark.parametrize("field", ["kappa", "omega"])
def test_nonfinite_parameters_are_refused(cme, field):
    inst = W.random_batch(4, [256])[0]
    getattr(inst, field)[17] = float("nan")
    with pytest.raises(cme.CmeError) as e:
        cme.Plan(W.pack([inst]), 0.005)
    assert e.value.code == cme.CME_ENONFINITE


@pytest.mark.parametrize("mode", ["rk4", "rk4ip", "split", "padded", "staged"])
def test_zero_state_without_pump_stays_zero(cme, mode):
    import torch
    n = {"staged": 16384, "padded": 512}.get(mode, 1024)
    insts = W.random_batch(5, [n, n])
    for inst in insts:
        inst.a0[:] = 0
        inst.a_in = 0j
    p = W.pack(insts)
    kw = {"rk4ip": {"integrator": cme.CME_RK4IP}, "split": {"integrator": cme.CME_SPLIT_STEP},
          "padded": {"fwm": cme.CME_FWM_PADDED}}.get(mode, {})
    with cme.Plan(p, 1e-3, **kw) as plan:
        A = plan.state(p.a0)
        plan.run(A, 20)
        torch.cuda.synchronize()
        assert torch.count_nonzero(A).item() == 0
        assert not plan.status().any()


def test_smallest_and_largest_sizes_in_one_ragged_plan(cme, orc):
    """N = 16 (several instances per workgroup, a ragged count), 256 (four
    wavefront-sized instances per workgroup, ragged) and 65536 (staged) side
    by side, one step against the oracle."""
    sizes = [16] * 7 + [256] * 5 + [65536]
    p = W.pack(moderate_batch(6, sizes))
    with cme.Plan(p, 0.005) as plan:
        import torch
        A = plan.state(p.a0)
        plan.run(A, 1, step0=3)
        torch.cuda.synchronize()
        y = A.cpu().numpy()
        names = {n: plan.kernel(n)["name"] for n in (16, 256, 65536)}
    ref, _ = orc.run(p, 0.005, 1, step0=3)
    errs = [rel_err(y[p.slice(b)], ref[p.slice(b)]) for b in range(p.batch)]
    print(names, max(errs))
    assert max(errs) <= 1e-13


def test_thousands_of_tiny_instances(cme, orc):
    import torch
    p = W.pack(moderate_batch(7, [16] * 4099))
    with cme.Plan(p, 0.005) as plan:
        A = plan.state(p.a0)
        plan.run(A, 5)
        torch.cuda.synchronize()
        y = A.cpu().numpy()
    ref, _ = orc.run(p, 0.005, 5)
    errs = [rel_err(y[p.slice(b)], ref[p.slice(b)]) for b in range(0, p.batch, 97)]
    assert max(errs) <= 1e-13


def test_caller_stream_gives_the_same_result(cme):
    import torch
    p = W.pack(moderate_batch(8, [2048, 1024, 2048]))
    with cme.Plan(p, 0.005) as plan:
        A = plan.state(p.a0)
        B = A.clone()
        plan.run(A, 20)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())   # B's copy comes first
        plan.set_stream(s)
        with torch.cuda.stream(s):
            plan.run(B, 20)
        s.synchronize()
        plan.set_stream(None)
        torch.cuda.synchronize()
        assert torch.equal(A, B)
