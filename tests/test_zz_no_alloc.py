"""cme_adjoint_noalloc (the allocation-free variant of cme_adjoint) against
cme_adjoint, through the C ABI.

Both run the same kernels on the same inputs; the allocation-free variant
works in the library's fixed device scratch array and runs each segment's
recompute and reverse sweep one after the other.  Bar: the FP64 parity bar
(relative error <= 1e-10), asserted here far tighter (<= 1e-13), on two calls
in a row, the second with a smaller input so that it reuses scratch the
first one left behind; requests larger than the scratch are refused with
CME_ESCRATCH before anything runs."""
import math

import numpy as np
import pytest

from paper_1307_3428_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-13


@pytest.fixture(scope="module")
def cme():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1307_3428_amd import cme as C
    C.load_library()
    return C


def batch(seed, sizes):
    insts = W.random_batch(seed, sizes, noise=1.0)
    for inst in insts:
        inst.a0 = inst.a0 / math.sqrt(inst.n_modes)
        inst.a0[inst.n_modes // 2] += 0.5
    return W.pack(insts)


def rel(a, b):
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


def both_adjoints(C, p, h, steps, K, with_ckpt):
    """gA_0, g_omega, g_kappa, g_ain from cme_adjoint and cme_adjoint_noalloc."""
    import torch
    out = []
    with C.Plan(p, h) as plan:
        A0 = plan.state(p.a0)
        rng = np.random.default_rng(len(p.a0))
        gT = plan.state(rng.standard_normal(p.total) + 1j * rng.standard_normal(p.total))
        ck = None
        if with_ckpt:
            ck = torch.zeros((steps // K, p.total), dtype=A0.dtype, device=A0.device)
            plan.run(A0.clone(), steps, ckpt_every=K, ckpt=ck)
        for fn in (C.cme_adjoint, C.cme_adjoint_noalloc):
            gA0 = torch.full_like(A0, float("nan"))
            g_om = torch.zeros(p.total, dtype=torch.float64, device=A0.device)
            g_ka = torch.zeros(p.total, dtype=torch.float64, device=A0.device)
            g_ai = torch.zeros(2 * p.batch, dtype=torch.float64, device=A0.device)
            print(f"{fn.__name__}: sizes {sorted(set(p.n_modes.tolist()))} steps {steps} K {K} "
                  f"ckpt {with_ckpt}", flush=True)
            fn(plan.handle, A0, ck, 0, steps, K, gT, gA0, g_om, g_ka, g_ai)
            torch.cuda.synchronize()
            out.append([t.cpu().numpy() for t in (gA0, g_om, g_ka, g_ai)])
        assert torch.equal(A0, plan.state(p.a0))
    return out


@pytest.mark.parametrize("with_ckpt_first", [True, False])
def test_noalloc_adjoint_matches_adjoint_twice(cme, with_ckpt_first):
    # first call: two size classes, several segments
    p1 = batch(31, [2048, 1024, 2048])
    ref, got = both_adjoints(cme, p1, 2e-3, 120, 40, with_ckpt_first)
    for r, g in zip(ref, got):
        assert np.isfinite(g).all()
        assert rel(g, r) <= TOL, rel(g, r)
    # second call, smaller: one instance of 512 modes, no caller checkpoints
    # (the forward pass's segment starts live in the scratch too)
    p2 = batch(32, [512])
    ref, got = both_adjoints(cme, p2, 2e-3, 50, 20, not with_ckpt_first)
    for r, g in zip(ref, got):
        assert np.isfinite(g).all()
        assert rel(g, r) <= TOL, rel(g, r)


def test_noalloc_adjoint_refuses_oversized_requests(cme):
    import torch
    p = batch(33, [4096, 4096])
    with cme.Plan(p, 1e-3) as plan:
        A0 = plan.state(p.a0)
        gA0 = torch.zeros_like(A0)
        # 8 * K * total complex values of stage records alone exceed the scratch
        K = cme.CME_NOALLOC_SCRATCH_BYTES // (16 * 8 * p.total) + 1
        with pytest.raises(cme.CmeError) as e:
            cme.cme_adjoint_noalloc(plan.handle, A0, None, 0, K, K, A0, gA0)
        assert e.value.code == cme.CME_ESCRATCH
        # a request that fits still runs after the refusal
        cme.cme_adjoint_noalloc(plan.handle, A0, None, 0, 4, 2, A0, gA0)
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(gA0)).all()
