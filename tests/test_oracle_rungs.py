"""Pins of the oracle's individual time steps (Sec. 2.3.6: power-of-two rungs,
the rung criterion after eq:courant_condition, the Saitoh-Makino limiter,
moving to a longer step only at its boundary, the predictor inside a
hierarchical kick-drift-kick).

  * the desired rung of closed-form step limits (exact powers of two, values
    between, a limit below the finest rung, NaN);
  * the predictor weight at hand-placed times inside a step;
  * every particle on one rung r: 2^r substeps equal 2^r global steps of
    dt0 2^-r bit for bit (the hierarchical scheme reduces to the global one);
  * the limiter: at T = 0 and after every rung update, the new step of an
    updated particle is at most four times the step of every particle of its
    force set (rungs before the update; at T = 0 the desired rungs), checked
    pair by pair on brute-force sets;
  * alignment: a particle that wants a longer step at a time that is not a
    boundary of it waits; every updated particle's new step divides the time
    of the update;
  * timing: the substeps of one base step add up to dt0, and at its end
    every particle is at a step boundary; particles without neighbours drift
    in straight lines;
  * second order: against the same system integrated with every particle on
    the finest rung, the difference falls about 4x when the step-limit
    parameters are halved.
Each composed pin rejects a planted mistake (the oracle's step function
replaced in the test).
"""
import copy

import numpy as np
import pytest

import sph_inputs as si


def hot_lattice(n_side=12, seed=7, hot=30.0, vsig=0.05):
    """Jittered periodic lattice with a hot sphere (u 30x) in the middle: its
    sound speed, hence its rung, is higher."""
    rng = np.random.default_rng(seed)
    x, y, z, a = si.jittered_lattice(rng, n_side)
    n = x.size
    r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
    u = np.where(r2 < 0.15 ** 2, hot, 1.0)
    st = dict(x=x, y=y, z=z, vx=rng.normal(0, vsig, n), vy=rng.normal(0, vsig, n),
              vz=rng.normal(0, vsig, n), m=np.full(n, 1.0 / n), u=u,
              H=np.full(n, si._h_guess(a, 60)))
    return st, si.params(kernel="wc2", n_ngb=60.0)


@pytest.fixture(scope="module")
def hot(orc):
    st, p = hot_lattice()
    s0 = orc.init(p, st)
    p = dict(p, dt_max=float(1.5 * s0["dt"].max()), rung_max=6)
    return st, p


@pytest.fixture(scope="module")
def hotter(orc):
    """u 300x in the hot sphere: five populated rungs, and the limiter changes
    rung updates inside the base step, not only at T = 0."""
    st, p = hot_lattice(hot=300.0)
    s0 = orc.init(p, st)
    p = dict(p, dt_max=float(1.5 * s0["dt"].max()), rung_max=7)
    return st, p


def run_base_step(orc, p, s, check=None):
    s = copy.deepcopy(s)
    reps = []
    while s["T"] < (1 << p["rung_max"]):
        before = copy.deepcopy(s)
        reps.append(orc.substep(p, s))
        if check:
            check(before, s, reps[-1])
    return s, reps


def test_desired_rung_closed_form(orc):
    p = {"rung_max": 5, "dt_max": 1.0}
    got = orc.desired_rung(p, [2.0, 1.0, 0.75, 0.5, 0.3, 1 / 32, 1 / 64, np.nan])
    assert got.tolist() == [0, 0, 1, 1, 2, 5, 5, 5]
    p = {"rung_max": 3, "dt_max": 0.1}
    assert orc.desired_rung(p, [0.1, 0.05, 0.0499, 0.0125]).tolist() == [0, 1, 2, 3]


def test_predict_coeff_values(orc):
    # steps of 8, 8, 2 and 4 units seen at T = 10 (delta = 1): the first two
    # started at 8 (middle 12), the third ends at 10 (started at 8, middle 9),
    # the fourth started at 8 (middle 10)
    got = orc.predict_coeff(np.int64(10), np.array([8, 8, 2, 4]), 1.0)
    assert got.tolist() == [-2.0, -2.0, 1.0, 0.0]
    assert orc.predict_coeff(np.int64(16), np.array([16]), 0.25).tolist() == [2.0]


@pytest.mark.parametrize("rung", [0, 2])
def test_one_rung_equals_global_steps(orc, rung):
    st, p = hot_lattice(hot=1.0, vsig=0.02)
    s0 = orc.init(p, st)
    lo, hi = s0["dt"].min(), s0["dt"].max()
    assert hi < 1.6 * lo
    dt0 = 0.9 * lo * 2 ** rung
    p = dict(p, dt_max=float(dt0), rung_max=4)
    s = orc.rung_init(p, st)
    assert np.all(s["rung"] == rung)
    ref = copy.deepcopy(s)
    for _ in range(2 ** rung):
        rep = orc.substep(p, s)
        assert rep["n_active"] == len(s["x"])
        orc.step(p, ref, dt=dt0 / 2 ** rung)
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "rho", "H", "ax", "dudt"):
        assert np.array_equal(s[k], ref[k]), k


def limiter_violations(orc, p, before, after, rep):
    """Updated particles whose new step exceeds four times a neighbour's step
    (rungs before the update), on the force sets at the update time."""
    L_old = orc.step_units(p, before["rung"])
    act = np.nonzero(rep["T"] % L_old == 0)[0]
    off, idx = orc.neighbors(p, after["x"], after["y"], after["z"], after["H"], mode=1)
    L_new = orc.step_units(p, after["rung"])
    bad = 0
    for i in act:
        nb = idx[off[i]:off[i + 1]]
        if nb.size and L_new[i] > 4 * np.min(orc.step_units(p, before["rung"][nb])):
            bad += 1
    return bad, act.size


def limiter_check(orc, hot):
    st, p = hot
    s = orc.rung_init(p, st)
    rd = orc.desired_rung(p, s["dt"])
    raised = int(np.sum(s["rung"] > rd))
    # at T = 0 the rungs the limiter looks at are the desired ones
    b0, _ = limiter_violations(orc, p, dict(s, rung=rd), s, {"T": 0})
    tally = {"bad": b0, "updated": 0, "changed": 0}

    def check(before, after, rep):
        b, n = limiter_violations(orc, p, before, after, rep)
        tally["bad"] += b
        tally["updated"] += n
        # updates whose result the limiter changed (against the desired rung
        # moved down as far as the update time allows)
        old = before["rung"]
        rows = np.nonzero(rep["T"] % orc.step_units(p, old) == 0)[0]
        rd_ = orc.desired_rung(p, after["dt"][rows])
        free = orc.align_down(p, old[rows], np.minimum(rd_, p["rung_max"]), rep["T"])
        tally["changed"] += int(np.sum(after["rung"][rows] != free))
    run_base_step(orc, p, s, check)
    return raised, tally


def test_limiter_holds_at_every_update(orc, hotter):
    raised, tally = limiter_check(orc, hotter)
    assert raised > 0             # the limiter acts at T = 0 ...
    assert tally["changed"] > 10  # ... and in the substeps
    assert tally["updated"] > 1000
    assert tally["bad"] == 0


def alignment_check(orc, hot):
    """Particles put on the finest rung at T = 0 want longer steps at their
    first update (T = 1 unit), which is no boundary of any longer step: they
    may only move down as far as the update time allows."""
    st, p = hot
    s = orc.rung_init(p, st)
    s["rung"][: len(s["rung"]) // 3] = p["rung_max"]
    bad = {"n": 0, "moved": 0}

    def check(before, after, rep):
        L_old = orc.step_units(p, before["rung"])
        act = rep["T"] % L_old == 0
        L_new = orc.step_units(p, after["rung"])
        bad["n"] += int(np.sum(act & (rep["T"] % L_new != 0)))
        bad["moved"] += int(np.sum(act & (after["rung"] < before["rung"])))
    run_base_step(orc, p, s, check)
    return bad


def test_longer_steps_only_at_their_boundaries(orc, hot):
    bad = alignment_check(orc, hot)
    assert bad["moved"] > 100
    assert bad["n"] == 0


def test_base_step_timing_and_free_drift(orc, hot):
    st, p = hot
    s = orc.rung_init(p, st)
    assert len(np.unique(s["rung"])) >= 3
    out, reps = run_base_step(orc, p, s)
    assert sum(r["dt"] for r in reps) == pytest.approx(p["dt_max"], rel=1e-15)
    assert np.all(out["T"] % orc.step_units(p, out["rung"]) == 0)
    # isolated particles: no neighbours, no force; straight lines over the step
    rng = np.random.default_rng(5)
    n = 64
    g = (np.arange(4) + 0.5) / 4
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    iso = dict(x=X.ravel(), y=Y.ravel(), z=Z.ravel(), vx=rng.normal(0, 0.3, n),
               vy=rng.normal(0, 0.3, n), vz=rng.normal(0, 0.3, n), m=np.full(n, 1.0 / n),
               u=rng.uniform(0.1, 20.0, n), H=np.full(n, 0.05))
    # (no neighbour within h_max: every H stops there)
    pi = si.params(kernel="m4", n_ngb=20.0, h_max=0.05, dt_max=0.02, rung_max=4)
    s = orc.rung_init(pi, iso)
    assert len(np.unique(s["rung"])) >= 2
    out, reps = run_base_step(orc, pi, s)
    for k in ("x", "y", "z"):
        want = orc._wrap(pi, iso[k] + 0.02 * iso["v" + k], "xyz".index(k))
        assert np.max(np.abs(out[k] - want)) < 1e-15


def convergence_ratio(orc, hot):
    """max|mixed rungs - finest rung| at step parameters eta and eta/2."""
    st, p0 = hot
    res = []
    for f in (1.0, 0.5):
        p = dict(p0, eta_c=0.3 * f, eta_a=0.2 * f, rung_max=8)
        s = orc.rung_init(p, st)
        rmax = int(s["rung"].max())
        a, _ = run_base_step(orc, p, s)
        b = copy.deepcopy(s)
        b["rung"][:] = rmax
        keep = orc.desired_rung
        orc.desired_rung = lambda prm, dt: np.full(np.shape(dt), rmax, dtype=np.int64)
        try:
            b, _ = run_base_step(orc, p, b)
        finally:
            orc.desired_rung = keep
        res.append({k: np.max(np.abs(a[k] - b[k])) / np.max(np.abs(b[k])) for k in ("x", "u")})
    return {k: res[0][k] / res[1][k] for k in ("x", "u")}


def test_second_order_against_finest_rung(orc, hot):
    r = convergence_ratio(orc, hot)
    print(f"error ratios at eta / (eta/2): {r}")
    assert r["x"] > 3.2 and r["u"] > 3.2


# ---- planted mistakes -----------------------------------------------------------

MUTANTS = {
    "limiter_off": ("limit_rungs", lambda orc: (lambda r_des, nb: r_des),
                    lambda orc, hot: limiter_check(orc, hot)[1]["bad"] > 0),
    "limiter_only_at_start": ("_assign_rungs", None,
                              lambda orc, hot: limiter_check(orc, hot)[1]["bad"] > 0),
    "down_anytime": ("align_down", lambda orc: (lambda p, r_old, r_new, T: np.asarray(r_new)),
                     lambda orc, hot: alignment_check(orc, hot)["n"] > 0),
    "predict_to_step_end": ("predict_coeff",
                            lambda orc: (lambda T, L, d: 0.5 * L.astype(np.float64) * d),
                            lambda orc, hot: min(convergence_ratio(orc, hot).values()) < 3.2),
}


def _limiter_only_at_start(orc):
    """Rung updates inside the base step skip the limiter (T = 0 keeps it)."""
    keep = orc._assign_rungs

    def assign(params, s, rows, old):
        if len(rows) == len(s["x"]) and s["T"] == 0:
            return keep(params, s, rows, old)
        R = int(params.get("rung_max", 8))
        return np.minimum(orc.desired_rung(params, s["dt"][rows]), R)
    return assign


MUTANTS["limiter_only_at_start"] = ("_assign_rungs", _limiter_only_at_start,
                                    MUTANTS["limiter_only_at_start"][2])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_rung_pins_reject_planted_mistakes(orc, hot, hotter, name):
    fn, make, caught = MUTANTS[name]
    keep = getattr(orc, fn)
    setattr(orc, fn, make(orc))
    try:
        assert caught(orc, hotter if name.startswith("limiter") else hot), name
    finally:
        setattr(orc, fn, keep)
