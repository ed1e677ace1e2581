"""Ten kick-drift-kick steps on the GPU against ten oracle steps (Sec. 2.3.6).

A step feeds its H, densities and forces into the next one, so agreement after
ten steps checks the whole loop (drift with periodic wrap, density with the
previous H as the first guess, prediction, EOS, forces, kicks, global time
step) and that differences do not grow from step to step.

  * FP64: positions, velocities, u and H of every particle within 1e-10 of the
    oracle's trajectory (absolute for positions in a unit box, relative to the
    rms for velocities, relative for u and H); the time step of every step
    within 1e-12 relative; momentum conserved to 1e-13 of sum m|v| (the pair
    terms are antisymmetric bit for bit, only the summation order differs).
  * Mixed: the per-step bar on accelerations is 1e-4 of rms |a|; over ten
    steps the velocity error may grow to 1e-3 of the rms velocity change the
    oracle's accelerations produce, and positions to that times the elapsed
    time.
"""
import numpy as np
import pytest

import sph_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STEPS = 10


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_11425_amd as m
    return m


def min_image(d):
    return d - np.round(d)


def trajectories(sph, orc, c, precision):
    s, p = c["state"], c["params"]
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(dict(p, precision=precision))
    print(f"trajectory {c['name']} {precision}", flush=True)
    ctx.init(P)
    ref = orc.init(p, s)
    dts = []
    for _ in range(STEPS):
        ctx.step(P)
        rep = orc.step(p, ref)
        dts.append((ctx.stats()["dt_used"], rep["dt"]))
    return P.numpy(), ref, ctx.stats(), np.array(dts)


CASES = [
    dict(seed=11, n=3000, kernel="wc4", n_ngb=100, clumped=True),
    dict(seed=12, n=2500, kernel="m4", n_ngb=50, clumped=False),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c['n']}-{c['kernel']}")
def test_ten_steps_fp64(sph, orc, case):
    c = si.random_cloud(case["seed"], case["n"], kernel=case["kernel"], n_ngb=case["n_ngb"],
                        periodic=True, clumped=case["clumped"])
    got, ref, st, dts = trajectories(sph, orc, c, "fp64")
    assert np.all(np.abs(dts[:, 0] - dts[:, 1]) <= 1e-12 * dts[:, 1])
    for k in ("x", "y", "z"):
        assert np.max(np.abs(min_image(got[k] - ref[k]))) < 1e-10, k
    vrms = np.sqrt(np.mean(ref["vx"] ** 2 + ref["vy"] ** 2 + ref["vz"] ** 2))
    for k in ("vx", "vy", "vz"):
        assert np.max(np.abs(got[k] - ref[k])) < 1e-10 * vrms, k
    for k in ("u", "H"):
        assert np.max(np.abs(got[k] - ref[k]) / np.abs(ref[k])) < 1e-10, k
    s0 = c["state"]
    m = s0["m"]
    scale = np.sum(m * (np.abs(s0["vx"]) + np.abs(s0["vy"]) + np.abs(s0["vz"])))
    p0 = [np.sum(m * s0[k]) for k in ("vx", "vy", "vz")]
    for a in range(3):
        assert abs(st["momentum"][a] - p0[a]) < 1e-13 * scale
    rep = orc.reductions(ref)
    assert abs(st["e_kin"] + st["e_int"] - rep["e_tot"]) < 1e-12 * rep["e_tot"]


def test_ten_steps_mixed(sph, orc):
    case = CASES[0]
    c = si.random_cloud(case["seed"], case["n"], kernel=case["kernel"], n_ngb=case["n_ngb"],
                        periodic=True, clumped=case["clumped"])
    got, ref, st, dts = trajectories(sph, orc, c, "mixed")
    s0 = c["state"]
    dv = np.sqrt(np.mean((ref["vx"] - s0["vx"]) ** 2 + (ref["vy"] - s0["vy"]) ** 2 +
                         (ref["vz"] - s0["vz"]) ** 2))
    t = float(np.sum(dts[:, 1]))
    verr = max(np.max(np.abs(got[k] - ref[k])) for k in ("vx", "vy", "vz"))
    xerr = max(np.max(np.abs(min_image(got[k] - ref[k]))) for k in ("x", "y", "z"))
    print(f"mixed: velocity error {verr / dv:.2e} of rms dv, position error "
          f"{xerr / (dv * t):.2e} of rms dv * t, dt {np.max(np.abs(dts[:, 0] / dts[:, 1] - 1)):.2e}")
    assert verr < 1e-3 * dv
    assert xerr < 1e-3 * dv * t
    assert np.all(np.abs(dts[:, 0] - dts[:, 1]) <= 1e-3 * dts[:, 1])


def test_step_after_caller_changes_h(sph, orc):
    """The first guess of the smoothing-length iteration is the last step's H
    extrapolated by its change; when the caller rescales H between steps the
    guess is far off, and the step must still reach the oracle's result (the
    root does not depend on the guess)."""
    case = CASES[0]
    c = si.random_cloud(case["seed"], case["n"], kernel=case["kernel"], n_ngb=case["n_ngb"],
                        periodic=True, clumped=case["clumped"])
    s, p = c["state"], c["params"]
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(p)
    print("step after a caller change of H", flush=True)
    ctx.init(P)
    ref = orc.init(p, s)
    ctx.step(P)
    orc.step(p, ref)
    P["H"].mul_(1.7)           # caller rescales H between steps
    ref["H"] = ref["H"] * 1.7
    ctx.step(P)
    rep = orc.step(p, ref)
    got = P.numpy()
    assert abs(ctx.stats()["dt_used"] - rep["dt"]) <= 1e-12 * rep["dt"]
    for k in ("H", "rho", "omega"):
        assert np.max(np.abs(got[k] - ref[k]) / np.abs(ref[k])) < 1e-11, k
    arms = np.sqrt(np.mean(ref["ax"] ** 2 + ref["ay"] ** 2 + ref["az"] ** 2))
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(got[k] - ref[k])) < 1e-10 * arms, k
