"""The discrete adjoint behind torch.autograd (cme.evolve): torch's gradcheck
on tiny sizes, and central finite differences on the N = 2048 gradient
workload (5000 RK4 steps, checkpoints every 100) along 32 seeded directions,
the 64 perturbed forward runs batched in one launch."""
import numpy as np
import pytest

from paper_1307_3428_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1307_3428_amd import cme
    cme.load_library()
    return cme


def meta_of(p, h, n_steps, K):
    return dict(n_modes=p.n_modes, offsets=p.offsets, kappa_ext=p.kappa_ext, g0=p.g0,
                sigma0=p.sigma0, sigma1=p.sigma1, tau_ramp=p.tau_ramp, h=h, n_steps=n_steps,
                ckpt_every=K)


def test_gradcheck_tiny(C):
    import torch
    insts = W.random_batch(21, [16, 16], noise=0.3, max_detuning=5)
    p = W.pack(insts)
    dev = "cuda"
    A0 = torch.tensor(p.a0, device=dev, requires_grad=True)
    om = torch.tensor(p.omega, device=dev, requires_grad=True)
    ka = torch.tensor(p.kappa, device=dev, requires_grad=True)
    ai = torch.tensor(p.a_in, dtype=torch.complex128, device=dev, requires_grad=True)
    meta = meta_of(p, 0.01, 6, 2)

    def f(A0, om, ka, ai):
        return C.evolve(A0, om, ka, ai, **meta)

    assert torch.autograd.gradcheck(f, (A0, om, ka, ai), eps=1e-6, atol=1e-7, rtol=1e-6)


def test_finite_differences_gradient_workload(C):
    import torch
    wl = W.adjoint_n2048()
    inst = wl.instances[0]
    n, h, steps, K = inst.n_modes, wl.h, wl.n_steps, wl.extra["ckpt_every"]
    target = torch.tensor(wl.extra["target"], device="cuda")
    p = W.pack([inst])
    A0 = torch.tensor(p.a0, device="cuda")
    om = torch.tensor(p.omega, device="cuda", requires_grad=True)
    ka = torch.tensor(p.kappa, device="cuda")
    ai = torch.tensor(p.a_in, dtype=torch.complex128, device="cuda", requires_grad=True)
    AT = C.evolve(A0, om, ka, ai, **meta_of(p, h, steps, K))
    loss = ((AT.abs() ** 2 - target) ** 2).sum()
    loss.backward()
    g = np.concatenate([om.grad.cpu().numpy(), [ai.grad.real.item(), ai.grad.imag.item()]])

    # 32 unit directions in R^(N+2): (delta omega'_mu, Re A_in, Im A_in)
    rng = np.random.default_rng(W.seed_for(4, 1))
    dirs = rng.standard_normal((32, n + 2))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    eps = 1e-6
    pert = []
    for v in dirs:
        for sgn in (1.0, -1.0):
            x = inst.copy()
            x.omega = inst.omega + sgn * eps * v[:n]
            x.a_in = inst.a_in + sgn * eps * complex(v[n], v[n + 1])
            pert.append(x)
    q = W.pack(pert)
    with C.Plan(q, h) as plan:            # the 64 perturbed runs: one launch
        A = plan.state(q.a0)
        plan.run(A, steps)
        torch.cuda.synchronize()
        A = A.view(64, n)
        Lq = ((A.abs() ** 2 - target) ** 2).sum(dim=1).cpu().numpy()
    fd = (Lq[0::2] - Lq[1::2]) / (2 * eps)
    ad = dirs @ g
    # "relative" is taken against the size of the directional derivatives:
    # a central difference carries a cancellation error of about
    # u |L| / eps (u = 2^-53), which swamps directions whose derivative is
    # close to zero, so those are held to the same absolute scale.
    scale = np.abs(fd).max()
    agg = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    floor = np.finfo(np.float64).eps * np.abs(Lq).max() / eps
    print("adjoint vs FD: aggregate rel %.2e, max |diff|/max|d| %.2e, FD rounding floor %.1e, "
          "|d| in %.2e..%.2e" % (agg, np.abs(ad - fd).max() / scale, floor, np.abs(fd).min(),
                                 scale), flush=True)
    assert agg <= 1e-6
    assert np.all(np.abs(ad - fd) <= 1e-6 * scale)
