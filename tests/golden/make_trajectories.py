"""Writes the stored oracle trajectories that the full-size GPU tests compare
with.  Calls only the oracle and the seeded input generators.

  large_fp64_10steps.json  128^3 jittered lattice (periodic, Wendland C4, 200
                           neighbours): the FP64 oracle's reductions and pair
                           counts after init and after each of 10 global
                           steps, and the state of 400 sampled particles
                           after init and after the 10 steps.
  two_phase_fp64_3steps.json  128^3 lattice with a slab of density 10 in
                           density 1 (pressure equilibrium, shear flow): the
                           same record after init and three steps.
  spheres_1step.json       two spheres in vacuum (12 000 000 + 4 800 000
                           particles, stiffened gas): reductions and pair
                           counts after init and one step, and the state of
                           400 sampled particles after init and after the
                           step.

Usage: python tests/golden/make_trajectories.py [large|two_phase|spheres]...
(all-thread oracle; the large case takes minutes, the spheres tens of them)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import sph_inputs as si  # noqa: E402

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u", "rho", "H", "ax", "ay", "az", "dudt")


def sample(s, rows):
    return {k: [float(v) for v in s[k][rows]] for k in FIELDS}


def rms_a(s):
    """rms of |a| over all particles (the scale of the acceleration bars)."""
    return float(np.sqrt(np.mean(s["ax"] ** 2 + s["ay"] ** 2 + s["az"] ** 2)))


def record(rep, s):
    return {"momentum": list(rep["momentum"]), "e_kin": rep["e_kin"], "e_int": rep["e_int"],
            "dt": rep.get("dt"), "n_d": s["n_d"], "n_f": s["n_f"], "rms_a": rms_a(s),
            "rms_dudt": float(np.sqrt(np.mean(s["dudt"] ** 2)))}


def trajectory(case, steps, nsample, seed, out):
    st, p = case["state"], case["params"]
    n = len(st["x"])
    rows = np.sort(np.random.default_rng(seed).choice(n, size=nsample, replace=False))
    t0 = time.time()
    s = oracle.init(p, st)
    print(f"init {time.time() - t0:.0f} s", flush=True)
    recs = [record(dict(oracle.reductions(s), dt=None), s)]
    first = sample(s, rows)
    for k in range(steps):
        rep = oracle.step(p, s)
        recs.append(record(rep, s))
        print(f"step {k + 1} dt {rep['dt']:.6e} {time.time() - t0:.0f} s", flush=True)
    doc = {"workload": case["name"], "n": n, "rows": [int(r) for r in rows], "steps": steps,
           "records": recs, "after_init": first, "final": sample(s, rows)}
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(doc, f)


def main():
    which = sys.argv[1:] or ["large", "two_phase", "spheres"]
    if "large" in which:
        trajectory(si.config_large(), 10, 400, 2024, "large_fp64_10steps.json")
    if "two_phase" in which:
        trajectory(si.config_two_phase(), 3, 400, 2026, "two_phase_fp64_3steps.json")
    if "spheres" in which:
        trajectory(si.config_spheres(), 1, 400, 2025, "spheres_1step.json")


if __name__ == "__main__":
    main()
