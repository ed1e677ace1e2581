"""Pins of the oracle's entropy-conserving update and evolved density
(Sec. 2.3.5, Sec. 2.3.3), against physics the paper's equations must obey:

  * the isentrope u(rho_new, s(rho_old, u_old)) solves the adiabatic first
    law du/d rho = P(rho, u)/rho^2 (integrated numerically here), for the
    ideal and the stiffened gas, in compression and expansion, P < 0 included;
  * under uniform compression v = -k (x - x0) the continuity equation's SPH
    rate is exactly d rho_i/dt = 3 k rho_i for every particle of any cloud
    (grad-h form: -sum m_j r W'(r) = 3 rho_i Omega_i), and the PdV heating is
    exactly 3 k P_i/rho_i (the first law); under a rigid rotation both vanish;
  * with the entropy flag, du/dt is the viscous heating alone: zero without
    viscosity, and for a pressureless gas the viscous energy identity
    sum m (v.a + du/dt) = 0 holds;
  * KDK steps without viscosity keep the entropy function (u - P0/rho) /
    rho^(gamma-1) of every particle to round-off;
  * a pressureless cloud in free uniform compression has the summed density
    rho0 / (1 - k t)^3 (self-similar); the evolved density follows it with an
    error of second order in the step.
"""
import numpy as np
import pytest

import sph_inputs as si


def first_law_u(eos, gamma, P0, rho0, u0, rho1, nsteps=4000):
    """RK4 integration of du/d rho = P(rho, u) / rho^2 from (rho0, u0) to rho1."""
    def P(r, u):
        return (gamma - 1.0) * r * u - (gamma * P0 if eos == "stiffened" else 0.0)

    def f(r, u):
        return P(r, u) / (r * r)

    h = (rho1 - rho0) / nsteps
    r, u = rho0, u0
    for _ in range(nsteps):
        k1 = f(r, u)
        k2 = f(r + 0.5 * h, u + 0.5 * h * k1)
        k3 = f(r + 0.5 * h, u + 0.5 * h * k2)
        k4 = f(r + h, u + h * k3)
        u += h * (k1 + 2 * k2 + 2 * k3 + k4) / 6.0
        r += h
    return u


@pytest.mark.parametrize("eos,gamma,P0", [("ideal", 5.0 / 3.0, 0.0), ("ideal", 1.4, 0.0),
                                          ("stiffened", 2.0, 1.0), ("stiffened", 7.0, 3.0)])
def test_isentrope_solves_the_adiabatic_first_law(orc, eos, gamma, P0):
    p = si.params(kernel="m4", n_ngb=64, eos=eos, gamma=gamma, P0=P0)
    rho_old = np.array([1.0, 1.0, 2.5, 0.4, 1.3])
    u_old = np.array([1.0, 0.3, 2.0, 5.0, 0.9])   # (the stiffened states include P < 0)
    rho_new = np.array([1.7, 0.6, 2.2, 0.5, 1.3])
    got = orc.isentrope(p, rho_old, u_old, rho_new)
    for k in range(len(got)):
        ref = first_law_u(eos, gamma, P0, rho_old[k], u_old[k], rho_new[k])
        assert abs(got[k] - ref) <= 1e-10 * max(1.0, abs(ref)), (k, got[k], ref)


def compress_cloud(seed, k=0.7, rotate=False, periodic=False):
    c = si.random_cloud(seed, 1500, kernel="wc4", n_ngb=80, periodic=periodic, clumped=True)
    s, p = c["state"], c["params"]
    d = orc_solve(c)
    x0 = np.array([0.5, 0.45, 0.55])
    X = np.stack([s["x"], s["y"], s["z"]]) - x0[:, None]
    if rotate:
        w = np.array([0.3, -1.1, 0.7])
        V = np.cross(w, X.T).T
    else:
        V = -k * X
    V = V + np.array([0.2, -0.1, 0.05])[:, None]   # a uniform drift cancels in v_ij
    return s, p, d, V


def orc_solve(c):
    import oracle
    s, p = c["state"], c["params"]
    return oracle.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])


@pytest.mark.parametrize("seed", [3, 4])
def test_continuity_rate_under_uniform_compression(orc, seed):
    k = 0.7
    s, p, d, V = compress_cloud(seed, k)
    P, c = orc.eos(p, d["rho"], s["u"])
    f = orc.forces(dict(p, evolved=True), s["x"], s["y"], s["z"], V[0], V[1], V[2], s["m"],
                   d["H"], d["rho"], d["omega"], P, c)
    assert np.max(np.abs(f["drho"] - 3 * k * d["rho"]) / d["rho"]) < 1e-11
    # the PdV part of du/dt is the first law's (P/rho^2) d rho/dt = 3 k P/rho
    f0 = orc.forces(dict(p, alpha=0.0, beta=0.0), s["x"], s["y"], s["z"], V[0], V[1], V[2],
                    s["m"], d["H"], d["rho"], d["omega"], P, c)
    assert np.max(np.abs(f0["dudt"] - 3 * k * P / d["rho"]) / (3 * k * P / d["rho"])) < 1e-11


def test_continuity_rate_vanishes_for_rotation(orc):
    s, p, d, V = compress_cloud(5, rotate=True)
    P, c = orc.eos(p, d["rho"], s["u"])
    f = orc.forces(dict(p, evolved=True), s["x"], s["y"], s["z"], V[0], V[1], V[2], s["m"],
                   d["H"], d["rho"], d["omega"], P, c)
    scale = np.max(np.abs(d["rho"])) * 1.3
    assert np.max(np.abs(f["drho"])) < 1e-12 * scale


def test_entropy_flag_leaves_only_viscous_heating(orc):
    c = si.random_cloud(6, 1200, kernel="m4", n_ngb=50, periodic=True, clumped=False)
    s, p = c["state"], c["params"]
    d = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    P, cs = orc.eos(p, d["rho"], s["u"])
    args = (s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"], d["H"], d["rho"],
            d["omega"])
    # no viscosity: no heating at all, although the PdV term is far from zero
    f_e = orc.forces(dict(p, alpha=0.0, beta=0.0, entropy=True), *args, P, cs)
    f_u = orc.forces(dict(p, alpha=0.0, beta=0.0), *args, P, cs)
    assert np.all(f_e["dudt"] == 0.0) and np.max(np.abs(f_u["dudt"])) > 0.0
    np.testing.assert_array_equal(f_e["ax"], f_u["ax"])
    # a pressureless gas (u = 0, so P = c = 0): the viscous force and heating
    # conserve energy, sum m (v.a + du/dt) = 0
    P0, c0 = orc.eos(p, d["rho"], np.zeros_like(s["u"]))
    f = orc.forces(dict(p, entropy=True), *args, P0, c0)
    m = s["m"]
    work = np.sum(m * (s["vx"] * f["ax"] + s["vy"] * f["ay"] + s["vz"] * f["az"]))
    heat = np.sum(m * f["dudt"])
    assert heat > 0.0
    assert abs(work + heat) < 1e-12 * heat


@pytest.mark.parametrize("eos,gamma,P0,u0", [("ideal", 5.0 / 3.0, 0.0, 1.0),
                                              ("stiffened", 2.0, 1.0, 2.5)])
def test_entropy_steps_keep_the_entropy_function(orc, eos, gamma, P0, u0):
    c = si.random_cloud(7, 1500, kernel="wc2", n_ngb=60, periodic=True, clumped=True)
    s, p = c["state"], dict(c["params"], eos=eos, gamma=gamma, P0=P0, alpha=0.0, beta=0.0,
                            entropy=True)
    s = dict(s, u=np.full(len(s["x"]), u0))
    st = orc.init(p, s)

    def S(state):
        return (state["u"] - P0 / state["rho"]) / state["rho"] ** (gamma - 1.0)

    S0 = S(st)
    rho_init = st["rho"].copy()
    for _ in range(5):
        orc.step(p, st)
    assert np.max(np.abs(S(st) - S0) / np.abs(S0)) < 1e-12
    # the densities did change, so the check is not vacuous
    assert np.max(np.abs(st["rho"] - rho_init) / rho_init) > 1e-4


def free_compression(nsteps, t_end=0.2, k=1.0):
    c = si.random_cloud(8, 1000, kernel="wc4", n_ngb=80, periodic=False, clumped=False)
    s = c["state"]
    p = dict(c["params"], alpha=0.0, beta=0.0, evolved=True)
    x0 = np.array([0.5, 0.5, 0.5])
    s = dict(s, u=np.zeros(len(s["x"])))
    for a, key in enumerate(("x", "y", "z")):
        s["v" + key] = -k * (s[key] - x0[a])
    return s, p, t_end / nsteps, k


@pytest.mark.slow
def test_evolved_density_follows_self_similar_compression(orc):
    errs = []
    for nsteps in (10, 20):
        s, p, dt, k = free_compression(nsteps)
        st = orc.init(p, s)
        rho0 = st["rho"].copy()
        for _ in range(nsteps):
            orc.step(p, st, dt)
        t = dt * nsteps
        exact = rho0 / (1.0 - k * t) ** 3
        # the summed density of the compressed cloud is self-similar too
        d = orc.solve_h(dict(p, evolved=False), st["x"], st["y"], st["z"], st["m"], st["H"])
        assert np.max(np.abs(d["rho"] - exact) / exact) < 1e-9
        errs.append(np.max(np.abs(st["rho"] - exact) / exact))
    assert errs[0] < 2e-3
    assert 3.0 < errs[0] / errs[1] < 5.0   # second order in the step


# ---- each pin above rejects a planted mistake (a compiled copy of the oracle
# with one textual substitution; the oracle's own source and library are not
# touched)

def _isentrope_error(orc, eos, gamma, P0):
    p = si.params(kernel="m4", n_ngb=64, eos=eos, gamma=gamma, P0=P0)
    ro, uo, rn = np.array([1.0, 2.5]), np.array([1.0, 2.0]), np.array([1.7, 2.2])
    got = orc.isentrope(p, ro, uo, rn)
    return max(abs(got[k] - first_law_u(eos, gamma, P0, ro[k], uo[k], rn[k])) for k in range(2))


def _continuity_error(orc):
    k = 0.7
    s, p, d, V = compress_cloud(3, k)
    P, c = orc.eos(p, d["rho"], s["u"])
    f = orc.forces(dict(p, evolved=True), s["x"], s["y"], s["z"], V[0], V[1], V[2], s["m"],
                   d["H"], d["rho"], d["omega"], P, c)
    return np.max(np.abs(f["drho"] - 3 * k * d["rho"]) / d["rho"])


def _entropy_heating(orc):
    c = si.random_cloud(6, 600, kernel="m4", n_ngb=50, periodic=True, clumped=False)
    s, p = c["state"], c["params"]
    d = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    P, cs = orc.eos(p, d["rho"], s["u"])
    f = orc.forces(dict(p, alpha=0.0, beta=0.0, entropy=True), s["x"], s["y"], s["z"], s["vx"],
                   s["vy"], s["vz"], s["m"], d["H"], d["rho"], d["omega"], P, cs)
    return np.max(np.abs(f["dudt"]))


F4_MUTANTS = {
    "isentrope_exponent_gamma": (
        "const double ratio = pow(rho_new[i] / rho_old[i], gm - 1.0);",
        "const double ratio = pow(rho_new[i] / rho_old[i], gm);",
        lambda orc: _isentrope_error(orc, "ideal", 5.0 / 3.0, 0.0)),
    "stiffened_isentrope_like_ideal": (
        "u_new[i] = (u_old[i] - p->P0 / rho_old[i]) * ratio + p->P0 / rho_new[i];",
        "u_new[i] = u_old[i] * ratio;",
        lambda orc: _isentrope_error(orc, "stiffened", 2.0, 1.0)),
    "continuity_without_omega": (
        "if (drho) drho[k] = spdv / omega[i];", "if (drho) drho[k] = spdv;", _continuity_error),
    "entropy_flag_keeps_pdv": (
        "dudt[k] = (p->flags & ORC_ENTROPY) ? heat : A[i] * spdv + heat;",
        "dudt[k] = A[i] * spdv + heat;", _entropy_heating),
}


@pytest.mark.parametrize("name", sorted(F4_MUTANTS))
def test_f4_pins_reject_planted_mistakes(orc, tmp_path, name):
    old, new, measure = F4_MUTANTS[name]
    src = orc.source_text()
    assert src.count(old) == 1, name
    assert measure(orc) < 1e-10   # the oracle itself
    lib = orc.compile_variant(src.replace(old, new), str(tmp_path / f"mut_{name}.so"))
    saved = orc._lib
    orc._lib = lib
    try:
        assert measure(orc) > 1e-3, name
    finally:
        orc._lib = saved
