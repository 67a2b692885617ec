"""Write the oracle reference states for the long-horizon GPU parity tests.

Runs ONLY the FP64 CPU oracle (``oracle/``) on inputs drawn by the seeded
generators of ``paper_1307_3428_amd.workloads`` and stores what it computes in
``tests/golden/oracle_<case>.npz`` (plain arrays, no pickled objects).  Nothing
here calls the HIP library.

Every case runs each reference instance together with a perturbed twin,
A(0) + 1e-12 ||A(0)|| z/||z|| (z a seeded complex Gaussian), and records the
relative separation of the two oracle trajectories at every checkpoint: the
two-trajectory test that says whether parity at 1e-10 is meaningful at a
given horizon (a trajectory that amplifies a 1e-12 change past 1e-10 also
amplifies the rounding differences between any two correct FP64
implementations).

Cases (the workload recipes are those of the benchmark; each docstring of
``workloads`` states the parameters):
  c1_ramp     single soliton run: N = 1024, sigma ramped -2 -> 8 over
              tau in [0, 200], 4e5 RK4 steps of h = 5e-4 (states every 4e4)
  c1s_held    soliton held at sigma = 1.5 (zeta = 3), N = 1024, 4e4 steps
  c2_sweep    detuning sweep, N = 2048, 5e4 steps: instances 0 and 255 (both
              ends of sigma), 43 and 64 (inside the modulation-instability
              window), 128 (mid sweep)
  c3_uneven   uneven-octave batch: the first 8 instances of each size class
              that classic RK4 is stable for, 2e3 steps for every class and
              2e4 (the full horizon) for N = 1024 and 2048 (twins for every
              instance of N <= 2048 and two per class above)
  c3_uneven_ip interaction-picture RK4 on 2 instances per class, including
              N = 8192 instances that classic RK4 is unstable for, 2e3 steps
  c4_adjoint  gradient workload: N = 2048, sigma = 6, 5000 steps; the forward
              state and the oracle's adjoint for the cotangent of the loss
              L = sum_mu (|A_mu(T)|^2 - t_mu)^2 at the oracle's final state
  c4s_adjoint the same at sigma = 3 (zeta = 3, the soliton regime)

Usage: python tests/golden/make_oracle_goldens.py CASE [--threads T]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1307_3428_amd import workloads as W  # noqa: E402

PERTURB = 1e-12
DIV = 1          # --dry K: every step count divided by K (a quick check of the script)
OUT = HERE
PERTURB_SEED = W.SEED_BASE + 999


def twin(inst: W.Instance, i: int) -> W.Instance:
    """Copy of `inst` with A(0) moved by PERTURB relative to ||A(0)||."""
    rng = np.random.default_rng(PERTURB_SEED + i)
    z = rng.standard_normal(inst.n_modes) + 1j * rng.standard_normal(inst.n_modes)
    t = inst.copy()
    t.a0 = inst.a0 + PERTURB * np.linalg.norm(inst.a0) * z / np.linalg.norm(z)
    return t


def rk4_stable(inst: W.Instance, h: float) -> bool:
    """|R(h lambda_mu)| <= 1 for every mode at both ends of the detuning range,
    R the classic RK4 stability polynomial (the instances the classic
    integrator may run)."""
    ok = True
    for sg in (inst.sigma0, inst.sigma1):
        z = h * (-0.5 * inst.kappa + 1j * (inst.omega - sg))
        r = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
        ok &= bool(np.all(np.abs(r) <= 1 - 1e-9))
    return ok


def separations(refs, twins, n_modes):
    """Relative separation of each reference/twin pair: whole vector and
    sidebands (every mode but mu = 0)."""
    whole, side = [], []
    for r, t, n in zip(refs, twins, n_modes):
        m = np.ones(n, bool)
        m[n // 2] = False
        whole.append(np.linalg.norm(t - r) / np.linalg.norm(r))
        side.append(np.linalg.norm((t - r)[m]) / np.linalg.norm(r[m]))
    return whole, side


def run_pairs(insts, h, segments, step0=0, integrator="rk4", n_twin=None):
    """Run reference instances and the twins of the first `n_twin` of them
    (default: all) in one oracle batch over the consecutive segments (lengths
    in steps).  Returns the step counts at the end of each segment, the
    reference states there [seg][b] and the separations [seg][b < n_twin]."""
    n_twin = len(insts) if n_twin is None else n_twin
    tw = [twin(x, k) for k, x in enumerate(insts[:n_twin])]
    p = W.pack(list(insts) + tw)
    nb = len(insts)
    y = p.a0.copy()
    steps, states, sep_w, sep_s = [], [], [], []
    done = step0
    for seg in segments:
        t0 = time.time()
        if integrator == "rk4":
            y, _ = oracle.run(p, h, seg, step0=done, y0=y)
        else:
            y = oracle.rk4ip_run(p, h, seg, step0=done, y0=y)
        done += seg
        refs = [y[p.slice(b)].copy() for b in range(nb)]
        tws = [y[p.slice(nb + b)].copy() for b in range(n_twin)]
        w, s = separations(refs[:n_twin], tws, [x.n_modes for x in insts[:n_twin]])
        steps.append(done)
        states.append(refs)
        sep_w.append(w)
        sep_s.append(s)
        print(f"  step {done}: {time.time() - t0:.0f}s  max sep {max(w):.2e} "
              f"(sidebands {max(s):.2e})", flush=True)
    return steps, states, np.array(sep_w), np.array(sep_s)


def save(case: str, meta: dict, arrays: dict) -> None:
    meta = dict(meta, case=case, script=os.path.basename(__file__),
                perturbation=PERTURB, perturbation_seed=PERTURB_SEED,
                oracle_threads=oracle.max_threads())
    path = os.path.join(OUT, f"oracle_{case}.npz")
    np.savez(path, meta=np.array(json.dumps(meta, sort_keys=True)), **arrays)
    print(f"wrote {path}", flush=True)


def case_c1_ramp():
    wl = W.soliton_ramp_n1024(n_steps=400000 // DIV)
    every = 40000 // DIV
    steps, states, sw, ss = run_pairs(wl.instances, wl.h, [every] * (wl.n_steps // every))
    save("c1_ramp", {"workload": wl.name, "h": wl.h, "n_steps": wl.n_steps, "indices": [0]},
         {"steps": np.array(steps), "states": np.array([s[0] for s in states]),
          "sep_whole": sw, "sep_side": ss})


def case_c1s_held():
    wl = W.soliton_held_n1024(n_steps=40000 // DIV)
    every = 4000 // DIV
    steps, states, sw, ss = run_pairs(wl.instances, wl.h, [every] * (wl.n_steps // every))
    keep = [0, len(steps) - 1]
    save("c1s_held", {"workload": wl.name, "h": wl.h, "n_steps": wl.n_steps, "indices": [0]},
         {"steps": np.array(steps), "states_steps": np.array([steps[k] for k in keep]),
          "states": np.array([states[k][0] for k in keep]), "sep_whole": sw, "sep_side": ss})


C2_INDICES = [0, 43, 64, 128, 255]


def case_c2_sweep():
    wl = W.sweep_n2048(indices=C2_INDICES, n_steps=50000 // DIV)
    every = 5000 // DIV
    steps, states, sw, ss = run_pairs(wl.instances, wl.h, [every] * (wl.n_steps // every))
    keep = [0, len(steps) - 1]
    save("c2_sweep", {"workload": wl.name, "h": wl.h, "n_steps": wl.n_steps,
                      "indices": C2_INDICES,
                      "sigma": [x.sigma0 for x in wl.instances]},
         {"steps": np.array(steps), "states_steps": np.array([steps[k] for k in keep]),
          "states": np.array([[states[k][b] for b in range(len(C2_INDICES))] for k in keep]),
          "sep_whole": sw, "sep_side": ss})


def uneven_picks(per_class=8, stable=True):
    wl = W.uneven_octave(n_steps=20000 // DIV)
    by_n = {}
    for i, x in enumerate(wl.instances):
        if rk4_stable(x, wl.h) == stable:
            by_n.setdefault(x.n_modes, []).append(i)
    return wl, {n: v[:per_class] for n, v in sorted(by_n.items())}


def case_c3_uneven():
    wl, picks = uneven_picks()
    short = 2000 // DIV
    small = [i for n in (1024, 2048) for i in picks[n]]
    # the larger classes run the short horizon only; twins for two per class
    large = ([i for n in (4096, 8192) for i in picks[n][:2]]
             + [i for n in (4096, 8192) for i in picks[n][2:]])
    print(f"c3: {len(small)} instances N <= 2048 to {wl.n_steps} steps", flush=True)
    steps_s, st_s, sw_s, ss_s = run_pairs([wl.instances[i] for i in small], wl.h,
                                          [short] * (wl.n_steps // short))
    print(f"c3: {len(large)} instances N >= 4096 to {short} steps", flush=True)
    _, st_l, sw_l, ss_l = run_pairs([wl.instances[i] for i in large], wl.h, [short], n_twin=4)
    save("c3_uneven", {"workload": wl.name, "h": wl.h, "n_steps": wl.n_steps, "short": short,
                       "indices_short": small + large, "indices_full": small,
                       "indices_large_twinned": large[:4]},
         {"states_short": np.concatenate(st_s[0] + st_l[0]),
          "states_full": np.concatenate(st_s[-1]),
          "steps_small": np.array(steps_s), "sep_whole_small": sw_s, "sep_side_small": ss_s,
          "sep_whole_large": sw_l[0], "sep_side_large": ss_l[0]})


def case_c3_uneven_ip():
    wl, stable = uneven_picks(per_class=2, stable=True)
    _, unstable = uneven_picks(per_class=2, stable=False)
    idx = sorted({i for d in (stable, unstable) for v in d.values() for i in v})
    insts = [wl.instances[i] for i in idx]
    short = 2000 // DIV
    print(f"c3 rk4ip: {len(idx)} instances, {short} steps", flush=True)
    _, st, sw, ss = run_pairs(insts, wl.h, [short], integrator="rk4ip")
    save("c3_uneven_ip", {"workload": wl.name, "h": wl.h, "n_steps": short, "indices": idx,
                          "rk4_unstable": [i for i in idx if not rk4_stable(wl.instances[i], wl.h)],
                          "n_modes": [wl.instances[i].n_modes for i in idx]},
         {"states": np.concatenate(st[0]), "sep_whole": sw[0], "sep_side": ss[0]})


def adjoint_case(case: str, wl: W.Workload):
    inst = wl.instances[0]
    p = W.pack([inst])
    t0 = time.time()
    yT, _ = oracle.run(p, wl.h, wl.n_steps)
    target = np.asarray(wl.extra["target"])
    loss = float(np.sum((np.abs(yT) ** 2 - target) ** 2))
    # cotangent dL/dRe A + i dL/dIm A of L = sum (|A|^2 - t)^2
    gT = 4.0 * (np.abs(yT) ** 2 - target) * yT
    g = oracle.adjoint(p, wl.h, wl.n_steps, gT)
    print(f"  forward + adjoint {time.time() - t0:.0f}s", flush=True)
    every = 500 // DIV
    _, _, sw, ss = run_pairs([inst], wl.h, [every] * (wl.n_steps // every))
    save(case, {"workload": wl.name, "h": wl.h, "n_steps": wl.n_steps, "sigma": inst.sigma0,
                "loss": loss, "ckpt_every": int(wl.extra["ckpt_every"])},
         {"yT": yT, "gT": gT, "gy0": g["gy0"], "g_omega": g["g_omega"], "g_kappa": g["g_kappa"],
          "g_ain": g["g_ain"], "sep_whole": sw[:, 0], "sep_side": ss[:, 0]})


def case_c4_adjoint():
    adjoint_case("c4_adjoint", W.adjoint_n2048(n_steps=5000 // DIV))


def case_c4s_adjoint():
    adjoint_case("c4s_adjoint", W.adjoint_soliton_n2048(n_steps=5000 // DIV))


CASES = {name[5:]: fn for name, fn in globals().items() if name.startswith("case_")}


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=sorted(CASES))
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--dry", type=int, default=0, metavar="K",
                    help="divide every step count by K and write into --out")
    ap.add_argument("--out", default=HERE)
    args = ap.parse_args()
    global DIV, OUT
    if args.dry:
        DIV, OUT = args.dry, args.out
    oracle.build(force=False)
    if args.threads:
        oracle.set_threads(args.threads)
    t0 = time.time()
    CASES[args.case]()
    print(f"{args.case}: {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
