"""Pins of the oracle's kick-drift-kick step with the predictor (Sec. 2.3.6).

  * a perfect lattice in uniform motion feels no force, so every step moves it
    by dt V exactly (wrapped) and leaves u, H, rho unchanged;
  * total momentum is conserved over several steps to round-off;
  * the total energy error over a fixed time falls as dt^2 (second order);
  * the global step is the minimum of the per-particle limits.
The size of the energy drift itself is "parity unpinned": the paper quotes
only whole-run conservation levels for its own tests (Sec. 3.3, 3.4).
"""
import numpy as np
import pytest

import sph_inputs as si


def test_uniform_motion_is_exact(orc):
    c = si.perfect_lattice(12, "m4", 64, u=1.0)
    s, p = c["state"], c["params"]
    V = (0.125, -0.25, 0.0625)
    s["vx"][:] = V[0]; s["vy"][:] = V[1]; s["vz"][:] = V[2]
    st = orc.init(p, s)
    x0 = st["x"].copy()
    H0, rho0 = st["H"].copy(), st["rho"].copy()
    dt = 0.0078125
    for k in range(1, 4):
        rep = orc.step(p, st, dt)
        assert rep["dt"] == dt
        expect = np.mod(x0 + k * dt * V[0], 1.0)
        assert np.max(np.abs(st["x"] - expect)) < 1e-14
        np.testing.assert_allclose(st["u"], 1.0, rtol=1e-12)
        np.testing.assert_allclose(st["vx"], V[0], rtol=1e-12)
    np.testing.assert_allclose(st["H"], H0, rtol=1e-12)
    np.testing.assert_allclose(st["rho"], rho0, rtol=1e-12)


def test_momentum_conserved(orc):
    c = si.uniform_box(8, 12, "wc4", 100, vsig=0.3)
    s, p = c["state"], c["params"]
    st = orc.init(p, s)
    r0 = orc.reductions(st)
    scale = np.sum(st["m"] * np.abs(st["vx"]))
    for _ in range(5):
        r = orc.step(p, st)
    for a in range(3):
        assert abs(r["momentum"][a] - r0["momentum"][a]) < 1e-14 * scale


def test_global_dt_is_min_of_limits(orc):
    c = si.uniform_box(9, 10, "m4", 64, vsig=0.3)
    s, p = c["state"], c["params"]
    st = orc.init(p, s)
    dtp = st["dt"].copy()
    rep = orc.step(p, st)
    assert rep["dt"] == min(dtp.min(), p["dt_max"])


def test_energy_error_second_order(orc):
    c = si.uniform_box(10, 10, "wc4", 100, vsig=0.2, jitter=0.2)
    s, p = c["state"], c["params"]
    p = dict(p, alpha=0.0, beta=0.0)
    T = 0.04
    errs = []
    for nsteps in (4, 8, 16):
        st = orc.init(p, s)
        e0 = orc.reductions(st)["e_tot"]
        for _ in range(nsteps):
            r = orc.step(p, st, T / nsteps)
        errs.append(abs(r["e_tot"] - e0))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
