"""GPU tests of the staged path: four-step transforms whose transpose goes
through global memory, for FP64 N = 8192 (a selectable alternative) and
N = 16384 ... 65536 (the only kernels there).

Parity with the FP64 oracle at full size over a few steps (the oracle's
O(N^2) sum costs seconds per step at N = 65536), a property that holds over
long runs at the largest size (the single-mode steady state is a fixed point
of Eq. (1)), agreement with the LDS-resident kernel over a longer horizon,
and the integer bookkeeping (split runs, checkpoints, graph replay) bitwise.
"""
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
    """Random per-mode kappa / omega', complex pump, ramp, and a full-support
    state of total power ~1 (every mode takes part in the mixing)."""
    insts = W.random_batch(seed, sizes, noise=1.0)
    for inst in insts:
        inst.a0 = inst.a0 / math.sqrt(inst.n_modes)
        inst.a0[inst.n_modes // 2] += 0.5
    return insts


def staged_ids(C, n):
    return [k for k in C.cme_list_kernels(C.CME_F64, n) if C.cme_kernel_info(k)["kind"] == 6]


def run(C, p, h, steps, step0=0, select=None, ckpt_every=0):
    import torch
    with C.Plan(p, h) as plan:
        for n, kid in (select or {}).items():
            plan.select(n, kid)
        A = plan.state(p.a0)
        ck = None
        if ckpt_every:
            ck = torch.zeros((steps // ckpt_every, p.total), dtype=A.dtype, device=A.device)
        plan.run(A, steps, step0=step0, ckpt_every=ckpt_every, ckpt=ck)
        torch.cuda.synchronize()
        st = plan.status()
        names = {int(n): plan.kernel(int(n))["name"] for n in set(p.n_modes.tolist())}
        return A.cpu().numpy(), (ck.cpu().numpy() if ck is not None else None), st, names


def _staged_params():
    try:
        from paper_1307_3428_amd import cme as C
        return [(n, k) for n in (8192, 16384, 32768, 65536) for k in staged_ids(C, n)]
    except Exception:
        return [(16384, 0)]


@pytest.mark.parametrize("n,kid", _staged_params())
def test_staged_variant_matches_oracle(cme, orc, n, kid):
    batch, steps = {8192: (3, 3), 16384: (2, 3), 32768: (2, 2), 65536: (1, 2)}[n]
    p = W.pack(moderate_batch(2000 + n + kid, [n] * batch))
    h = 0.01
    y, _, st, names = run(cme, p, h, steps, step0=5, select={n: kid})
    print(f"N={n} {names[n]}", flush=True)
    ref, _ = orc.run(p, h, steps, step0=5)
    for b in range(batch):
        err = rel_err(y[p.slice(b)], ref[p.slice(b)])
        moved = rel_err(p.a0[p.slice(b)], ref[p.slice(b)])
        print(f"  instance {b}: GPU vs oracle {err:.2e} (state moved {moved:.2e})", flush=True)
        assert err <= 1e-13 and moved > 1e-3
    assert not st.any()


def _staged_f32_params():
    try:
        from paper_1307_3428_amd import cme as C
        return [(n, k) for n in (8192, 16384, 32768, 65536)
                for k in C.cme_list_kernels(C.CME_F32, n) if C.cme_kernel_info(k)["kind"] == 6]
    except Exception:
        return [(16384, 0)]


@pytest.mark.parametrize("n,kid", _staged_f32_params())
def test_staged_fp32_variant_matches_fp64_oracle(cme, orc, n, kid):
    """FP32 state and transforms (FP64 stage arithmetic) against the FP64 oracle."""
    import torch
    batch, steps = {8192: (3, 3), 16384: (2, 3), 32768: (1, 2), 65536: (1, 2)}[n]
    p = W.pack(moderate_batch(2100 + n, [n] * batch))
    h = 0.01
    with cme.Plan(p, h, precision=cme.CME_F32) as plan:
        plan.select(n, kid)
        A = plan.state(p.a0)
        assert A.dtype == torch.complex64
        plan.run(A, steps, step0=5)
        torch.cuda.synchronize()
        y = A.cpu().numpy().astype(np.complex128)
        assert not plan.status().any()
        name = plan.kernel(n)["name"]
    ref, _ = orc.run(p, h, steps, step0=5)
    errs = [rel_err(y[p.slice(b)], ref[p.slice(b)]) for b in range(batch)]
    print(f"N={n} {name}: {errs}", flush=True)
    assert max(errs) <= 2e-6


def test_staged_mixed_plan_matches_oracle(cme, orc):
    """Staged and LDS-resident classes in one plan (concurrent launches)."""
    sizes = [16384, 2048, 512, 16384, 8192]
    p = W.pack(moderate_batch(31, sizes))
    y, _, st, names = run(cme, p, 0.005, 3)
    assert names[16384].startswith("rk4_staged")
    ref, _ = orc.run(p, 0.005, 3)
    errs = [rel_err(y[p.slice(b)], ref[p.slice(b)]) for b in range(p.batch)]
    print(names, errs)
    assert max(errs) <= 1e-13
    assert not st.any()


def test_staged_cw_fixed_point_at_full_size(cme):
    """The homogeneous single-mode steady state is an exact fixed point of
    Eq. (1) (every four-wave-mixing term but |A0|^2 A0 vanishes); 300 RK4
    steps at N = 65536 must keep it to rounding and the other modes at zero."""
    insts = []
    for j, (s0, m) in enumerate([(1.0, 2.0), (3.0, 4.0)]):
        inst = W.make_instance(65536, d2=1e-6, pump_multiple=m, sigma0=s0, start="cw")
        insts.append(inst)
    p = W.pack(insts)
    y, _, st, names = run(cme, p, 1e-3, 300)
    for b in range(p.batch):
        a0, yb = p.a0[p.slice(b)], y[p.slice(b)]
        side = np.abs(np.delete(yb, 65536 // 2)).max()
        err = abs(yb[65536 // 2] - a0[65536 // 2]) / abs(a0[65536 // 2])
        print(f"{names[65536]}: pump mode drift {err:.2e}, max sideband {side:.2e}")
        assert err <= 1e-12 and side <= 1e-12 * abs(a0[65536 // 2])
    assert not st.any()


def test_staged_agrees_with_lds_kernel_over_a_longer_run(cme):
    """N = 8192: the staged variants and the LDS-resident kernel
    over 400 steps with checkpoints.  Kernel-against-kernel: both are held
    to the oracle over short runs above; this bounds the drift between the
    two evaluation orders."""
    p = W.pack(moderate_batch(47, [8192] * 3))
    wave = [k for k in cme.cme_list_kernels(cme.CME_F64, 8192) if cme.cme_kernel_info(k)["kind"] == 1][0]
    base, ck0, _, names0 = run(cme, p, 2e-3, 400, select={8192: wave}, ckpt_every=100)
    assert names0[8192].startswith("rk4_wave")
    for kid in staged_ids(cme, 8192):
        y, ck, st, names = run(cme, p, 2e-3, 400, select={8192: kid}, ckpt_every=100)
        errs = [rel_err(y[p.slice(b)], base[p.slice(b)]) for b in range(3)]
        cerr = float(np.abs(ck - ck0).max() / np.abs(ck0).max())
        print(f"{names[8192]} vs {names0[8192]}: {errs}, checkpoints {cerr:.2e}")
        assert max(errs) <= 1e-12 and cerr <= 1e-12
        assert not st.any()


def test_staged_longer_horizon_matches_oracle(cme, orc):
    """N = 8192 on the staged kernels for 100 steps (the state moves by tens
    of percent) against the oracle, checkpoints included."""
    p = W.pack(moderate_batch(71, [8192]))
    kid = staged_ids(cme, 8192)[0]
    y, ck, st, names = run(cme, p, 2e-3, 100, select={8192: kid}, ckpt_every=50)
    ref, ref_ck = orc.run(p, 2e-3, 100, ckpt_every=50)
    err = rel_err(y, ref)
    moved = rel_err(p.a0, ref)
    cerr = max(rel_err(ck[j], ref_ck[j]) for j in range(2))
    print(f"{names[8192]}: {err:.2e} (moved {moved:.2e}), checkpoints {cerr:.2e}")
    assert err <= 1e-11 and cerr <= 1e-11 and moved > 0.1
    assert not st.any()


def test_staged_split_runs_and_checkpoints_are_bitwise(cme):
    import torch
    p = W.pack(moderate_batch(53, [16384, 16384]))
    h = 0.004
    with cme.Plan(p, h) as plan:
        A = plan.state(p.a0)
        ck = torch.zeros((4, p.total), dtype=A.dtype, device=A.device)
        plan.run(A, 12, step0=3, ckpt_every=3, ckpt=ck)
        B = plan.state(p.a0)
        mids = []
        for s in range(4):
            plan.run(B, 3, step0=3 + 3 * s)
            mids.append(B.clone())
        torch.cuda.synchronize()
        assert torch.equal(A, B)
        for s in range(4):
            assert torch.equal(ck[s], mids[s])
        assert not plan.status().any()


def test_staged_graph_replays_match_eager(cme):
    import torch
    p = W.pack(moderate_batch(59, [16384, 1024]))
    with cme.Plan(p, 0.005) as plan:
        A = plan.state(p.a0)
        B = A.clone()
        s = torch.cuda.Stream()
        plan.set_stream(s)
        with torch.cuda.stream(s):
            warm = A.clone()
            plan.run(warm, 2)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            plan.run(A, 5)
        plan.set_stream(None)
        for _ in range(3):
            g.replay()
            torch.cuda.synchronize()
            plan.run(B, 5)
            torch.cuda.synchronize()
            assert torch.equal(A, B)
        assert not plan.status().any()


def test_adjoint_with_staged_forward_uses_a_reverse_capable_kernel(cme):
    """With the staged kernel selected at N = 8192 the adjoint recomputes and
    reverses with a kernel of that size that has a reverse sweep: the result
    equals the adjoint of a plan on its default kernel, and the forward
    selection is kept afterwards."""
    import torch
    p = W.pack(moderate_batch(61, [8192, 8192]))
    h, steps = 2e-3, 20
    rng = np.random.default_rng(5)
    gT = (rng.standard_normal(p.total) + 1j * rng.standard_normal(p.total)) * 1e-2
    outs = []
    for select in (False, True):
        with cme.Plan(p, h) as plan:
            if select:
                plan.select(8192, staged_ids(cme, 8192)[0])
            A0 = plan.state(p.a0)
            g = plan.adjoint(A0, plan.state(gT), steps, ckpt_every=10)
            torch.cuda.synchronize()
            outs.append({k: v.cpu().numpy() for k, v in g.items()})
            if select:
                assert plan.kernel(8192)["name"].startswith("rk4_staged")
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_staged_rejects_unsupported_requests(cme):
    """Above 8192 points: no FP32 split-step, no adjoint, no FP32
    four-wave-mixing sum alone."""
    p = W.pack(moderate_batch(67, [16384]))
    with pytest.raises(cme.CmeError) as e:
        cme.Plan(p, 0.01, precision=cme.CME_F32, integrator=cme.CME_SPLIT_STEP)
    assert e.value.code == cme.CME_EUNSUPPORTED
    with cme.Plan(p, 0.01) as plan:
        A0 = plan.state(p.a0)
        with pytest.raises(cme.CmeError):
            plan.adjoint(A0, A0.clone(), 2)
    with cme.Plan(p, 0.01, precision=cme.CME_F32) as plan:
        A0 = plan.state(p.a0)
        with pytest.raises(cme.CmeError):
            plan.fwm(A0)


def test_staged_padded_and_split_longer_runs_match_oracle(cme, orc):
    """The padded sum (8192 modes on 16384-point staged transforms, 20 RK4
    steps) and the split-step map (N = 16384, 30 steps) against the oracle,
    checkpoints included."""
    import torch
    for kind, n, steps, h in (("padded", 8192, 20, 5e-3), ("split", 16384, 30, 5e-3)):
        p = W.pack(moderate_batch(2200 + n, [n]))
        kw = {"fwm": cme.CME_FWM_PADDED} if kind == "padded" else {"integrator": cme.CME_SPLIT_STEP}
        with cme.Plan(p, h, **kw) as plan:
            A = plan.state(p.a0)
            ck = torch.zeros((2, p.total), dtype=A.dtype, device=A.device)
            plan.run(A, steps, ckpt_every=steps // 2, ckpt=ck)
            torch.cuda.synchronize()
            y, ck = A.cpu().numpy(), ck.cpu().numpy()
            name = plan.kernel(n)["name"]
            assert not plan.status().any()
        if kind == "padded":
            ref, _ = orc.run(p, h, steps, truncated=True)
            mid, _ = orc.run(p, h, steps // 2, truncated=True)
        else:
            ref = orc.split_step_run(p, h, steps)
            mid = orc.split_step_run(p, h, steps // 2)
        err, cerr, moved = rel_err(y, ref), rel_err(ck[0], mid), rel_err(p.a0, ref)
        print(f"{name}: {err:.2e}, checkpoint {cerr:.2e} (moved {moved:.2e})", flush=True)
        assert err <= 1e-11 and cerr <= 1e-11 and moved > 0.05
