"""Pins of the oracle's force pass (Sec. 2.3.5: symmetrised pressure force,
PdV du/dt, Monaghan viscosity with eq:AV_heating; Sec. 2.3.6 time-step limits).

Pins, each of which a plausible slip (dropped gather or scatter term, wrong
sign, wrong factor 1/2, transposed x_ij) breaks:
  * pairwise antisymmetry: total momentum change is zero to round-off;
  * the semi-discrete energy identity sum m (v.a + du/dt) = 0, viscosity on;
  * angular momentum conservation in an open box (central pair forces);
  * the variational identity m_i a_i = -dE_int/dx_i at fixed entropy with H
    re-solved (no viscosity), which fixes Omega and both kernel terms;
  * a perfect lattice at rest has a = 0, du/dt = 0 and the closed-form
    signal-velocity time step;
  * Galilean invariance; viscosity only heats.
"""
import numpy as np
import pytest

import sph_inputs as si


def prepare(orc, c, u=None):
    s, p = c["state"], c["params"]
    d = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    uu = s["u"] if u is None else u
    P, cs = orc.eos(p, d["rho"], uu)
    return s, p, d, P, cs


def run_forces(orc, s, p, d, P, cs, vx=None, vy=None, vz=None):
    return orc.forces(p, s["x"], s["y"], s["z"],
                      s["vx"] if vx is None else vx, s["vy"] if vy is None else vy,
                      s["vz"] if vz is None else vz,
                      s["m"], d["H"], d["rho"], d["omega"], P, cs)


@pytest.mark.parametrize("periodic,kernel", [(True, "m4"), (True, "wc4"), (False, "wc2"), (False, "wc6")])
def test_momentum_and_energy_identities(orc, periodic, kernel):
    c = si.random_cloud(31, 1500, kernel=kernel, n_ngb=60, periodic=periodic, clumped=True, vsig=0.5)
    s, p, d, P, cs = prepare(orc, c)
    f = run_forces(orc, s, p, d, P, cs)
    m = s["m"]
    for ax, v in (("ax", "vx"), ("ay", "vy"), ("az", "vz")):
        scale = np.sum(m * np.abs(f[ax]))
        assert abs(np.sum(m * f[ax])) < 1e-13 * scale
    power = m * (s["vx"] * f["ax"] + s["vy"] * f["ay"] + s["vz"] * f["az"])
    scale = np.sum(np.abs(power)) + np.sum(np.abs(m * f["dudt"]))
    assert abs(np.sum(power + m * f["dudt"])) < 1e-13 * scale
    # the viscosity was active in this case
    assert np.any(f["dudt"] != 0)


def test_angular_momentum_open(orc):
    c = si.random_cloud(32, 1200, kernel="wc4", n_ngb=80, periodic=False, clumped=True, vsig=0.5)
    s, p, d, P, cs = prepare(orc, c)
    f = run_forces(orc, s, p, d, P, cs)
    m = s["m"]
    x, y, z = s["x"], s["y"], s["z"]
    tx = np.sum(m * (y * f["az"] - z * f["ay"]))
    ty = np.sum(m * (z * f["ax"] - x * f["az"]))
    tz = np.sum(m * (x * f["ay"] - y * f["ax"]))
    scale = np.sum(m * np.sqrt(x * x + y * y + z * z) * np.sqrt(f["ax"] ** 2 + f["ay"] ** 2 + f["az"] ** 2))
    assert max(abs(tx), abs(ty), abs(tz)) < 1e-13 * scale


@pytest.mark.parametrize("kernel", ["m4", "wc4"])
def test_variational_force(orc, kernel):
    # E_int = sum_j m_j K_j rho_j^(gamma-1) / (gamma-1): the hydro force is -grad E_int
    c = si.random_cloud(33, 400, kernel=kernel, n_ngb=40, periodic=True, clumped=True,
                        alpha=0.0, beta=0.0)
    s, p = c["state"], c["params"]
    p = dict(p, alpha=0.0, beta=0.0)
    gam = p["gamma"]
    d = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    K = np.random.default_rng(5).uniform(0.5, 1.5, len(s["m"]))
    u = K * d["rho"] ** (gam - 1) / (gam - 1)
    P, cs = orc.eos(p, d["rho"], u)
    f = orc.forces(p, s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"], d["H"],
                   d["rho"], d["omega"], P, cs)

    def energy(x, y, z):
        dd = orc.solve_h(p, x, y, z, s["m"], d["H"])
        return np.sum(s["m"] * K * dd["rho"] ** (gam - 1) / (gam - 1))

    e = 2e-7
    rng = np.random.default_rng(6)
    amax = np.max(np.abs(s["m"] * f["ax"]))
    for i in rng.choice(len(s["m"]), 6, replace=False):
        for comp, key in ((0, "ax"), (1, "ay"), (2, "az")):
            xyz = [s["x"].copy(), s["y"].copy(), s["z"].copy()]
            xyz[comp][i] += e
            Ep = energy(*xyz)
            xyz[comp][i] -= 2 * e
            Em = energy(*xyz)
            fd = -(Ep - Em) / (2 * e)
            assert abs(fd - s["m"][i] * f[key][i]) < 2e-5 * amax, (i, comp)


@pytest.mark.parametrize("kernel,n_ngb", [("m4", 64), ("wc4", 200)])
def test_lattice_at_rest(orc, kernel, n_ngb):
    c = si.perfect_lattice(16, kernel, n_ngb, u=1.3)
    s, p, d, P, cs = prepare(orc, c)
    f = run_forces(orc, s, p, d, P, cs)
    # one pair term for scale
    A = P[0] / (d["omega"][0] * d["rho"][0] ** 2)
    scale = s["m"][0] * A * d["H"][0] ** -3 * 10
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(f[k])) < 1e-12 * scale
    assert np.max(np.abs(f["dudt"])) == 0.0
    gam = p["gamma"]
    c0 = np.sqrt(gam * (gam - 1) * 1.3)
    dt_cfl = p["eta_c"] * 0.5 * d["H"] / ((1 + 0.6 * p["alpha"]) * c0)
    np.testing.assert_allclose(f["dt"], np.minimum(dt_cfl, p["dt_max"]), rtol=1e-14)


def test_galilean_invariance(orc):
    c = si.random_cloud(34, 1000, kernel="wc2", n_ngb=50, clumped=True, vsig=0.4)
    s, p, d, P, cs = prepare(orc, c)
    f = run_forces(orc, s, p, d, P, cs)
    V = (0.75, -0.5, 0.25)
    g = run_forces(orc, s, p, d, P, cs, s["vx"] + V[0], s["vy"] + V[1], s["vz"] + V[2])
    for k in ("ax", "ay", "az", "dudt"):
        sc = np.max(np.abs(f[k]))
        assert np.max(np.abs(f[k] - g[k])) < 1e-12 * sc


def test_viscosity_only_heats(orc):
    # cold gas (u = 0: P = 0, c = 0) so only the beta term of the viscosity acts
    c = si.random_cloud(35, 1000, kernel="m4", n_ngb=50, clumped=True, vsig=1.0)
    s = c["state"]
    s, p, d, P, cs = prepare(orc, c, u=np.zeros_like(s["u"]))
    f = run_forces(orc, s, p, d, P, cs)
    assert np.all(f["dudt"] >= 0.0) and np.any(f["dudt"] > 0.0)
    m = s["m"]
    assert np.sum(m * (s["vx"] * f["ax"] + s["vy"] * f["ay"] + s["vz"] * f["az"])) < 0.0
    # without any approaching pair there is no viscosity: expanding flow v = x - centre
    p2 = dict(p, periodic=False)
    x0, y0, z0 = s["x"] - 0.5, s["y"] - 0.5, s["z"] - 0.5
    d2 = orc.solve_h(p2, x0, y0, z0, m, d["H"])
    P2, c2 = orc.eos(p2, d2["rho"], np.zeros_like(m))
    g = orc.forces(p2, x0, y0, z0, x0, y0, z0, m, d2["H"], d2["rho"], d2["omega"], P2, c2)
    assert np.all(g["dudt"] == 0.0) and np.all(g["ax"] == 0.0)


def test_scatter_only_pair(orc):
    # j reaches i (H_j > r) but not vice versa (H_i < r): only the scatter term acts
    p = si.params(kernel="m4", n_ngb=64, periodic=False, alpha=0.0, beta=0.0,
                  box_lo=(-1, -1, -1), box_hi=(1, 1, 1))
    x = np.array([0.0, 0.3]); y = np.zeros(2); z = np.zeros(2)
    H = np.array([0.2, 0.5]); m = np.array([1.0, 2.0])
    rho = np.array([1.0, 1.5]); om = np.array([0.9, 0.95]); P = np.array([2.0, 3.0])
    c = np.array([1.0, 1.0]); v = np.zeros(2)
    f = orc.forces(p, x, y, z, v, v, v, m, H, rho, om, P, c)
    assert f["count"].tolist() == [1, 1]
    assert f["ax"][0] != 0.0
    np.testing.assert_allclose(m[0] * f["ax"][0], -m[1] * f["ax"][1], rtol=1e-15)
    # j's own pressure pushes i away from j (i is at smaller x)
    assert f["ax"][0] < 0.0
