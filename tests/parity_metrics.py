"""Error metrics of the parity tests (spectra stored in centred order: index
i holds mode mu = i - N/2, the pump mode mu = 0 at N/2).

On the workloads that start from the pumped single-mode state plus noise,
the pump mode carries almost all of ||A||: a relative L2 error over the whole
vector then bounds the sidebands only loosely.  Every check that runs such a
workload therefore also looks at the sidebands alone (mu != 0) and at the
power spectrum |A_mu|^2."""
from __future__ import annotations

import numpy as np


def _rel(d, ref) -> float:
    nr = float(np.linalg.norm(ref))
    nd = float(np.linalg.norm(d))
    if nr == 0.0:
        return 0.0 if nd == 0.0 else float("inf")
    return nd / nr


def sideband_mask(n: int) -> np.ndarray:
    m = np.ones(n, dtype=bool)
    m[n // 2] = False
    return m


def errors(y, ref) -> dict:
    """Relative L2 errors of one instance's spectrum y against ref:
    whole     ||y - ref|| / ||ref||
    side      the same over mu != 0
    power     || |y|^2 - |ref|^2 || / || |ref|^2 ||
    power_side the power error over mu != 0
    side_frac ||ref over mu != 0|| / ||ref|| (how much of the state the
              sidebands hold)"""
    y = np.asarray(y)
    ref = np.asarray(ref)
    m = sideband_mask(ref.shape[0])
    py, pr = np.abs(y) ** 2, np.abs(ref) ** 2
    return {
        "whole": _rel(y - ref, ref),
        "side": _rel((y - ref)[m], ref[m]),
        "power": _rel(py - pr, pr),
        "power_side": _rel((py - pr)[m], pr[m]),
        "side_frac": _rel(ref[m], ref),
    }


def packed_errors(packed, y, ref, which=None) -> list:
    """errors() per instance of a packed batch (instances `which`, default all)."""
    idx = range(packed.batch) if which is None else which
    return [errors(y[packed.slice(b)], ref[packed.slice(b)]) for b in idx]


def worst(errs: list, key: str) -> float:
    return max(e[key] for e in errs) if errs else 0.0
