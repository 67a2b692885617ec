"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/cme.h, and rejects invalid arguments before touching a
device.  Also checks the seeded input generators."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1307_3428_amd import cme as C
from paper_1307_3428_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cme.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cme_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("cme_init", "cme_step", "cme_run", "cme_adjoint", "cme_destroy",
                     "cme_strerror", "cme_status"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = C.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(C.EXPORTED)


def test_strerror_and_version():
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        s = C.cme_strerror(code)
        assert s and s != "unknown status code"
    assert C.cme_strerror(-99) == "unknown status code"
    assert C.cme_version() >= 10000


def test_kernel_table_covers_every_size():
    seen = set()
    for n in (16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768, 65536):
        ids = C.cme_list_kernels(C.CME_F64, n)
        assert ids, n
        for k in ids:
            info = C.cme_kernel_info(k)
            assert info["n_modes"] == n and info["precision"] == C.CME_F64
            e = info["elems_per_thread"]
            assert e & (e - 1) == 0 and 2 <= e <= n
            assert info["threads"] <= 1024 and info["lds_bytes"] <= 160 * 1024
            if info["kind"] in (6, 8, 9, 10):
                # staged: rows of N1 and columns of N / N1 points, each a
                # team of whole lanes inside one wavefront
                n1 = info["sub_transforms"]
                assert n % n1 == 0 and 64 % (n1 // e) == 0 and 64 % (n // n1 // e) == 0
                assert info["threads"] % 64 == 0
            else:
                assert info["threads"] == info["instances_per_group"] * (n // e)
            if info["kind"] in (1, 2, 3, 4, 5, 7, 11, 12, 13, 14):  # two-level: whole wavefronts per instance
                assert (n // e) % 64 == 0
            seen.add(k)
        # above 8192 only the staged kernels
        assert n <= 8192 or all(C.cme_kernel_info(k)["kind"] in (6, 8, 9, 10) for k in ids)
        assert n <= 8192 or all(C.cme_kernel_info(k)["kind"] in (6, 8)
                                for k in C.cme_list_kernels(C.CME_F32, n))
    assert C.cme_list_kernels(C.CME_F64, 100) == []
    assert C.cme_list_kernels(C.CME_F64, 131072) == []
    with pytest.raises(C.CmeError):
        C.cme_kernel_info(10 ** 6)


def _inst(n=64, offset=0, **kw):
    d = dict(kappa_ext=0.5, g0=1.0, a_in=[0.5], sigma0=[1.0], sigma1=[1.0], tau_ramp=[0.0])
    d.update(kw)
    return C.make_instances([n], [offset], [d["kappa_ext"]], [d["g0"]], d["a_in"], d["sigma0"],
                            d["sigma1"], d["tau_ramp"])


def _init_raw(inst, kappa, omega, h=0.01, precision=0, flags=0, batch=None, plan=True,
              integrator=0, fwm=0):
    lib = C.load_library()
    handle = ctypes.c_void_p(12345)
    kp = kappa.ctypes.data_as(ctypes.c_void_p) if kappa is not None else None
    op = omega.ctypes.data_as(ctypes.c_void_p) if omega is not None else None
    rc = lib.cme_init(ctypes.byref(handle) if plan else None,
                      len(inst) if batch is None else batch, inst, kp, op, precision, integrator,
                      fwm, h, None, flags)
    return rc, handle.value


@pytest.mark.parametrize("case", ["null_plan", "batch0", "null_kappa", "bad_n", "n_too_big",
                                  "n_too_small", "neg_h", "nan_h", "bad_precision",
                                  "reserved", "neg_offset", "overlap", "bad_flags",
                                  "nan_sigma", "neg_kext", "bad_integrator",
                                  "bad_fwm", "padded_split", "large_fp32", "large_padded",
                                  "rk4ip_padded"])
def test_init_rejects_invalid_arguments_without_a_device(case):
    kappa = np.ones(256)
    omega = np.zeros(256)
    inst = _inst()
    kw = {}
    expect = C.CME_EINVAL
    if case == "null_plan":
        kw["plan"] = False
    elif case == "batch0":
        kw["batch"] = 0
    elif case == "null_kappa":
        kappa = None
    elif case == "bad_n":
        inst = _inst(n=48)
    elif case == "n_too_big":
        inst = _inst(n=131072)
    elif case == "n_too_small":
        inst = _inst(n=8)
    elif case == "neg_h":
        kw["h"] = -1.0
    elif case == "nan_h":
        kw["h"] = float("nan")
    elif case == "bad_precision":
        kw["precision"] = 7
    elif case == "reserved":
        inst[0].reserved = 1
    elif case == "neg_offset":
        inst = _inst(offset=-1)
    elif case == "overlap":
        inst = C.make_instances([64, 64], [0, 32], [0.5, 0.5], [1, 1], [0.5, 0.5], [1, 1], [1, 1],
                                [0, 0])
    elif case == "bad_flags":
        kw["flags"] = 1 << 7
    elif case == "nan_sigma":
        inst = _inst(sigma0=[float("nan")])
        expect = C.CME_ENONFINITE
    elif case == "neg_kext":
        inst = _inst(kappa_ext=-0.1)
    elif case == "bad_integrator":
        kw["integrator"] = 3
    elif case == "rk4ip_padded":
        kw["integrator"] = C.CME_RK4IP
        kw["fwm"] = C.CME_FWM_PADDED
        expect = C.CME_EUNSUPPORTED
    elif case == "bad_fwm":
        kw["fwm"] = 2
    elif case == "padded_split":
        kw["fwm"] = C.CME_FWM_PADDED
        kw["integrator"] = C.CME_SPLIT_STEP
        expect = C.CME_EUNSUPPORTED
    elif case in ("large_fp32", "large_padded"):
        # no FP32 split-step (at any size); at most 65536 transform points
        # (32768 modes with the padded sum)
        inst = _inst(n=16384 if case != "large_padded" else 65536)
        kw.update({"large_fp32": {"precision": C.CME_F32, "integrator": C.CME_SPLIT_STEP},
                   "large_padded": {"fwm": C.CME_FWM_PADDED}}[case])
        expect = C.CME_EUNSUPPORTED
    rc, handle = _init_raw(inst, kappa, omega, **kw)
    assert rc == expect, (case, rc)
    if kw.get("plan", True):
        assert handle is None  # *plan cleared on error


def test_calls_on_null_plan():
    lib = C.load_library()
    assert lib.cme_run(None, None, 0, 1, 0, None) == C.CME_EINVAL
    assert lib.cme_step(None, None, 0) == C.CME_EINVAL
    assert lib.cme_fwm(None, None, None) == C.CME_EINVAL
    assert lib.cme_adjoint(None, None, None, 0, 1, 0, None, None, None, None, None) == C.CME_EINVAL
    flags = np.zeros(1, np.int32)
    assert lib.cme_status(None, flags.ctypes.data_as(ctypes.c_void_p)) == C.CME_EINVAL
    assert lib.cme_destroy(None) == C.CME_OK
    assert lib.cme_plan_kernel(None, 64, None) == C.CME_EINVAL
    assert lib.cme_plan_select(None, 64, 4) == C.CME_EINVAL
    assert lib.cme_set_stream(None, None) == C.CME_EINVAL


def test_binding_refuses_cpu_tensors():
    import torch
    with pytest.raises(ValueError):
        C._dptr(torch.zeros(4, dtype=torch.complex128))


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(C, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        C.load_library(str(tmp_path / "missing.so"))


def test_oracle_library_exports():
    import oracle
    lib = oracle.load()
    for name in ("orc_fwm", "orc_kerr_vjp", "orc_rhs", "orc_run", "orc_adjoint",
                 "orc_split_step_run", "orc_sigma"):
        assert hasattr(lib, name)


# ---------------------------------------------------------------------------
# Seeded input generators
# ---------------------------------------------------------------------------

def test_workloads_are_seeded_and_shaped():
    a = W.plain_n128().instances[0]
    b = W.plain_n128().instances[0]
    assert np.array_equal(a.a0, b.a0)
    assert a.n_modes == 128 and a.kappa.shape == (128,)
    mu = W.mu_grid(128)
    assert mu[0] == -64 and mu[-1] == 63 and mu[64] == 0
    assert np.allclose(a.omega, -0.02 * mu ** 2)
    assert abs(abs(a.a_in) ** 2 - 0.75) < 1e-15      # 3x threshold of 0.25
    wl = W.sweep_n2048(batch=256, n_steps=1)
    assert wl.batch == 256 and wl.total_modes == 256 * 2048
    assert wl.instances[0].sigma0 == -2.0 and abs(wl.instances[255].sigma0 - 10.0) < 1e-12
    sub = W.sweep_n2048(indices=[7])
    assert np.array_equal(sub.instances[0].a0, wl.instances[7].a0)
    u = W.uneven_octave(batch=64, n_steps=1)
    assert set(x.n_modes for x in u.instances) <= {1024, 2048, 4096, 8192}


def test_pack_offsets():
    insts = W.random_batch(3, [16, 64, 32])
    p = W.pack(insts)
    assert list(p.offsets) == [0, 16, 80] and p.total == 112
    assert np.array_equal(p.a0[p.slice(1)], insts[1].a0)


def test_cw_state_solves_the_single_mode_balance():
    for sigma, m in [(2.0, 3.0), (-2.0, 4.0), (0.5, 3.0), (6.0, 4.0)]:
        a_in = W.pump_for_multiple(m, 1.0, 1.0, 0.5)
        A = W.cw_state(a_in, sigma, 0.0, 1.0, 1.0, 0.5)
        # stationarity of dA/dt = (-1/2 - i sigma) A + sqrt(0.5) A_in + i |A|^2 A
        res = (-0.5 - 1j * sigma) * A + np.sqrt(0.5) * a_in + 1j * abs(A) ** 2 * A
        assert abs(res) < 1e-14


def test_one_hip_runtime_after_load():
    """load_library() imports torch before it opens libcme.so, so the HIP
    runtime libcme.so needs resolves to the one torch already mapped: a second
    libamdhip64 in the process (device pointers and streams of one runtime
    handed to the other) crashed a GPU run once.  Checked in a fresh process
    from /proc/self/maps."""
    import subprocess
    import sys
    code = (
        "from paper_1307_3428_amd import cme\n"
        "cme.load_library()\n"
        "paths = set()\n"
        "for line in open('/proc/self/maps'):\n"
        "    f = line.split()\n"
        "    if len(f) >= 6 and 'libamdhip64' in f[5]:\n"
        "        paths.add(f[5])\n"
        "print(len(paths), sorted(paths))\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split()[0] == "1", r.stdout
