"""Index maps of the lane-exchange transform layouts, modelled in numpy.

The N = 2048 paired kernel (8 x 256 layout), the N = 8192 stream kernels
(16 x 512 layout) and the N = 512 / 1024 paired kernels (last exchange in
registers) move data between lanes with v_permlane32_swap / v_permlane16_swap
and rename registers afterwards.  These tests model the threads, their slots,
the LDS regions and the two swap instructions in numpy, run the same sequence
of passes the kernels run, and compare with numpy's FFT, so that a wrong
position formula, swap pairing or renaming fails on the CPU.  They check the
layouts' arithmetic, not the HIP code; the GPU parity tests check that.
"""
import numpy as np
import pytest

LANES = np.arange(64)


def dft(z, S):
    """DFT of sign S over the last axis (natural order)."""
    R = z.shape[-1]
    r = np.arange(R)
    return z @ np.exp(S * 2j * np.pi * np.outer(r, r) / R)


def rot(x, S):
    return np.exp(S * 2j * np.pi * x)


def swap32(x, y):
    """v_permlane32_swap: the upper 32 lanes of x trade with the lower 32 of y."""
    x2, y2 = x.copy(), y.copy()
    x2[..., 32:] = y[..., :32]
    y2[..., :32] = x[..., 32:]
    return x2, y2


def swap16(x, y):
    """v_permlane16_swap: the odd rows (16 lanes) of x trade with the even rows of y."""
    x2, y2 = x.copy(), y.copy()
    for r0 in (0, 32):
        x2[..., r0 + 16:r0 + 32] = y[..., r0:r0 + 16]
        y2[..., r0:r0 + 16] = x[..., r0 + 16:r0 + 32]
    return x2, y2


def reference(y, S):
    n = y.size
    return np.fft.ifft(y) * n if S > 0 else np.fft.fft(y)


# ---------------------------------------------------------------------------
# N = 2048 as 8 x 256: 4 waves, slot m of thread c = 64 w + l holds mode c + 256 m

def sub256(V, S):
    """Two 256-point sub-transforms per wave on alternate lanes (lane = 2t + s):
    radix 8, exchange through the region, radix 8, lane-swap exchange, radix 4."""
    V = V.copy()
    t = LANES >> 1
    V = dft(V, S)
    reg = np.zeros((V.shape[0], 2, 256), complex)
    for s in (0, 1):
        for r in range(8):
            reg[:, s, 8 * t[s::2] + r] = V[:, s::2, r]
    for s in (0, 1):
        for m in range(8):
            V[:, s::2, m] = reg[:, s, t[s::2] + 32 * m]
    k = (t & 7)[None, :, None]
    V = dft(V * rot(k * np.arange(8)[None, None, :] / 64, S), S)
    for r in (0, 1, 4, 5):
        V[:, :, r], V[:, :, r ^ 2] = swap32(V[:, :, r], V[:, :, r ^ 2])
    for r in (0, 2, 4, 6):
        V[:, :, r], V[:, :, r ^ 1] = swap16(V[:, :, r], V[:, :, r ^ 1])
    V = V[:, :, [4 * (m & 1) + 2 * (m >> 2) + ((m >> 1) & 1) for m in range(8)]]
    out = V.copy()
    for q in (0, 1):
        j = (t + 32 * q)[None, :, None]
        z = V[:, :, [q + 2 * s for s in range(4)]] * rot(j * np.arange(4)[None, None, :] / 256, S)
        Z = dft(z, S)
        for r in range(4):
            out[:, :, q + 2 * r] = Z[:, :, r]
    return out


def d8_inverse(y, S):
    c = np.arange(256)
    V = dft(y[c[:, None] + 256 * np.arange(8)[None, :]], S) * rot(c[:, None] * np.arange(8)[None, :] / 2048, S)
    T = np.zeros((4, 64, 8), complex)
    for w in range(4):
        for s in (0, 1):
            tt = LANES[s::2] >> 1
            for m in range(8):
                T[w, s::2, m] = V[tt + 32 * m, 2 * w + s]
    return sub256(T, S)


def d8_forward(T, S):
    U = sub256(T, S)
    X = np.zeros((8, 256), complex)
    for w in range(4):
        for s in (0, 1):
            tt = LANES[s::2] >> 1
            for m in range(8):
                X[2 * w + s, tt + 32 * m] = U[w, s::2, m]
    c = np.arange(256)
    V = dft(X.T * rot(c[:, None] * np.arange(8)[None, :] / 2048, S), S)
    out = np.zeros(2048, complex)
    out[c[:, None] + 256 * np.arange(8)[None, :]] = V
    return out


def d8_time_index():
    w = np.arange(4)[:, None, None]
    l = LANES[None, :, None]
    m = np.arange(8)[None, None, :]
    return 2 * w + (l & 1) + 8 * ((l >> 1) + 32 * m)


@pytest.mark.parametrize("S", [+1, -1])
def test_8x256_layout(S):
    rng = np.random.default_rng(5)
    y = rng.standard_normal(2048) + 1j * rng.standard_normal(2048)
    ti = d8_time_index()
    assert sorted(ti.ravel().tolist()) == list(range(2048))
    T = d8_inverse(y, S)
    ref = reference(y, S)
    assert np.abs(T - ref[ti]).max() <= 1e-12 * np.abs(ref).max()
    back = d8_forward(T, -S)
    assert np.abs(back - 2048 * y).max() <= 1e-12 * 2048 * np.abs(y).max()


# ---------------------------------------------------------------------------
# N = 8192 as 16 x 512: 8 waves, slot m of thread c = 64 w + l holds mode c + 512 m

def sub512(V, S):
    """Two 512-point sub-transforms per wave on alternate lanes: radix 16,
    exchange through the region, radix 16, one lane-bit-5 swap stage, radix 2."""
    V = V.copy()
    t = LANES >> 1
    V = dft(V, S)
    reg = np.zeros((V.shape[0], 2, 512), complex)
    for s in (0, 1):
        for r in range(16):
            reg[:, s, 16 * t[s::2] + r] = V[:, s::2, r]
    for s in (0, 1):
        for m in range(16):
            V[:, s::2, m] = reg[:, s, t[s::2] + 32 * m]
    k = (t & 15)[None, :, None]
    V = dft(V * rot(k * np.arange(16)[None, None, :] / 256, S), S)
    for r in range(0, 16, 2):
        V[:, :, r], V[:, :, r + 1] = swap32(V[:, :, r], V[:, :, r + 1])
    V = V[:, :, [2 * (m & 7) + (m >> 3) for m in range(16)]]
    out = V.copy()
    for q in range(8):
        a = V[:, :, q]
        b = V[:, :, q + 8] * rot((t[None, :] + 32 * q) / 512, S)
        out[:, :, q], out[:, :, q + 8] = a + b, a - b
    return out


def s16_inverse(y, S):
    c = np.arange(512)
    V = dft(y[c[:, None] + 512 * np.arange(16)[None, :]], S) * rot(c[:, None] * np.arange(16)[None, :] / 8192, S)
    T = np.zeros((8, 64, 16), complex)
    for w in range(8):
        for s in (0, 1):
            tt = LANES[s::2] >> 1
            for m in range(16):
                T[w, s::2, m] = V[tt + 32 * m, 2 * w + s]
    return sub512(T, S)


def s16_forward(T, S):
    U = sub512(T, S)
    X = np.zeros((16, 512), complex)
    for w in range(8):
        for s in (0, 1):
            tt = LANES[s::2] >> 1
            for m in range(16):
                X[2 * w + s, tt + 32 * m] = U[w, s::2, m]
    c = np.arange(512)
    V = dft(X.T * rot(c[:, None] * np.arange(16)[None, :] / 8192, S), S)
    out = np.zeros(8192, complex)
    out[c[:, None] + 512 * np.arange(16)[None, :]] = V
    return out


@pytest.mark.parametrize("S", [+1, -1])
def test_16x512_layout(S):
    rng = np.random.default_rng(6)
    y = rng.standard_normal(8192) + 1j * rng.standard_normal(8192)
    w = np.arange(8)[:, None, None]
    l = LANES[None, :, None]
    m = np.arange(16)[None, None, :]
    ti = 2 * w + (l & 1) + 16 * ((l >> 1) + 32 * m)
    assert sorted(ti.ravel().tolist()) == list(range(8192))
    T = s16_inverse(y, S)
    ref = reference(y, S)
    assert np.abs(T - ref[ti]).max() <= 1e-12 * np.abs(ref).max()
    back = s16_forward(T, -S)
    assert np.abs(back - 8192 * y).max() <= 1e-12 * 8192 * np.abs(y).max()


# ---------------------------------------------------------------------------
# the last exchange of a 256-point sub-transform at four modes per thread

def test_lane_exchange4_is_the_last_stockham_exchange():
    """After the third radix-4 pass element r of lane t belongs at position
    64 (t >> 4) + 16 r + (t & 15); the last pass gathers position t' + 64 m
    into slot m.  Two swap stages must deliver exactly that."""
    pos = np.zeros((64, 4), int)
    for t in range(64):
        for r in range(4):
            pos[t, r] = 64 * (t >> 4) + 16 * r + (t & 15)
    v = pos.T.astype(complex).copy()             # v[r][lane]
    for r in (0, 1):
        v[r], v[r + 2] = swap32(v[r], v[r + 2])
    for r in (0, 2):
        v[r], v[r + 1] = swap16(v[r], v[r + 1])
    want = np.array([[t + 64 * m for t in range(64)] for m in range(4)])
    assert np.array_equal(v.real.astype(int), want)
