"""Write the oracle's results for the full-size workloads to tests/golden/*.json.

Calls only the FP64 CPU oracle (and the shared input generators).  The GPU parity tests compare
against these files at sizes where running the oracle inline would take minutes.

    python tests/golden/make_golden.py [name ...]
"""

from __future__ import annotations

import json
import os
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import hotrg as O  # noqa: E402
from paper_1912_02780_amd import inputs as I  # noqa: E402

# name -> (input description, builder, chi, n_steps)
CASES = {
    "ising_b0.30_chi32_n30": ("ising", 0.30, 32, 30),
    "ising_b0.4406868_chi32_n30": ("ising", 0.4406868, 32, 30),
    "ising_b0.50_chi32_n30": ("ising", 0.50, 32, 30),
    "random_d4_seed0_chi48_n24": ("random_d4", 0, 48, 24),
    "ising_b0.4406868_chi24_n24": ("ising", 0.4406868, 24, 24),
    "ising_b0.4406868_chi64_n30": ("ising", 0.4406868, 64, 30),
}

# Cases too large for a second (perturbed) oracle pass within a few hours, and large enough that
# each step's record is kept on disk (memory maps) rather than in RAM.
LARGE = {"ising_b0.4406868_chi64_n30"}


def rounding_sensitivity(T0, chi, n, L_ref, g_ref, seed=1234):
    rng = np.random.default_rng(seed)
    orig = O.gram

    def noisy_gram(A, B):
        G = orig(A, B)
        E = rng.standard_normal(G.shape)
        return G * (1.0 + 2.0 ** -52 * 0.5 * (E + E.T))

    O.gram = noisy_gram
    try:
        fwd = O.hotrg_forward(T0, chi, n)
        g = O.hotrg_backward(fwd, 1.0, O.DEFAULT_BROADENING)
    finally:
        O.gram = orig
    return (abs(fwd.lnZ_per_site / L_ref - 1.0),
            float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)))


def run(name):
    kind, param, chi, n = CASES[name]
    if kind == "ising":
        T0 = I.ising_T0(param)
        dT0 = I.ising_dT0_dbeta(param)
    else:
        T0 = I.random_d4_T0(int(param))
        dT0 = None
    large = name in LARGE
    spill = None
    if large:
        # the step records go to GOLDEN_SPILL_DIR (else a fresh temporary directory); delete it after
        spill = os.environ.get("GOLDEN_SPILL_DIR") or tempfile.mkdtemp(prefix="oracle_spill_")
        os.makedirs(spill, exist_ok=True)
    t0 = time.time()

    def progress(phase, k):
        print(f"  {name}: {phase} step {k} at {time.time() - t0:.0f}s", flush=True)

    fwd = O.hotrg_forward(T0, chi, n, spill_dir=spill, progress=progress)
    t1 = time.time()
    g = O.hotrg_backward(fwd, 1.0, O.DEFAULT_BROADENING, progress=progress)
    t2 = time.time()
    inv = O.step_invariants(fwd)
    # Rounding sensitivity of the oracle itself: repeat with every Gram perturbed entrywise by a
    # symmetric relative noise of 2^-52 (the size of FP64 rounding) and record how far ln Z / N
    # and T0bar move.  Parity between two correct FP64 implementations cannot be finer than this.
    # (Not run for the largest cases: it would double hours of oracle time.)
    sens = (None, None) if large else rounding_sensitivity(T0, chi, n, fwd.lnZ_per_site, g)
    out = {
        "name": name, "input": kind, "param": param, "chi": chi, "n_steps": n,
        "broadening": O.DEFAULT_BROADENING,
        "lnZ_per_site": fwd.lnZ_per_site,
        "T0bar": g.reshape(-1).tolist(),
        "T0bar_shape": list(g.shape),
        "dlnZ_dbeta": float(np.sum(g * dT0)) if dT0 is not None else None,
        "euler": float(np.sum(g * T0)),
        "c": [r["c"] for r in inv],
        "lam_last_kept": [float(r["lam_kept"][-1]) for r in inv],
        "cut_gap": [r["cut_gap"] for r in inv],
        "trunc_weight": [r["trunc_weight"] for r in inv],
        "rounding_sensitivity_lnZ": sens[0],
        "rounding_sensitivity_T0bar": sens[1],
        "oracle_seconds_forward": t1 - t0,
        "oracle_seconds_backward": t2 - t1,
        "generated_by": "tests/golden/make_golden.py (FP64 NumPy oracle)",
    }
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: lnZ/N={fwd.lnZ_per_site:.16f} fwd {t1 - t0:.1f}s bwd {t2 - t1:.1f}s", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for nm in names:
        run(nm)
