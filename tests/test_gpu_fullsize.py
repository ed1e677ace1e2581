"""Full-size checks at 128^3 = 2 097 152 particles (the benchmarked workloads),
in the launch configuration the benchmark times.

The oracle cannot finish 2M particles within a test, so it is evaluated on a
sample of rows (its row-subset mode) and compared element by element there;
properties that hold at any size (total momentum change, symmetric pair
counts) are checked on the whole output.  Force inputs (H, rho, Omega) are
generated, never taken from the GPU, so both sides see the same inputs.
"""
import numpy as np
import pytest

import sph_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_11425_amd as m
    return m


def rows_sample(n, k=1500, seed=99):
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False))


def perturbed_force_inputs(s, seed=5):
    """Generated H, rho, Omega for the force pass (a few per cent of scatter)."""
    rng = np.random.default_rng(seed)
    n = len(s["x"])
    H = s["H"] * rng.uniform(0.97, 1.03, n)
    rho = (s["m"] * n) * rng.uniform(0.95, 1.05, n)
    om = rng.uniform(0.95, 1.0, n)
    return dict(s, H=H, rho=rho, omega=om)


@pytest.mark.parametrize("cfg,precision", [("large", "fp64"), ("large", "mixed"),
                                           ("two_phase", "mixed"), ("two_phase", "fp64")])
def test_fullsize_density_sampled(sph, orc, cfg, precision):
    c = si.config_large() if cfg == "large" else si.config_two_phase()
    s, p = c["state"], c["params"]
    n = len(s["x"])
    print(f"full-size density {c['name']} {precision}", flush=True)
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(dict(p, precision=precision))
    ctx.build_tree(P)
    ctx.density(P)
    st = ctx.stats()
    assert st["n_overflow"] == 0 and st["n_noconv"] == 0
    got = P.numpy()
    rows = rows_sample(n)
    ref = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"], rows=rows)
    tol = 1e-12 if precision == "fp64" else 1e-5
    for k, r in (("H", ref["H"]), ("rho", ref["rho"]), ("omega", ref["omega"])):
        err = np.max(np.abs(got[k][rows] - r) / np.abs(r))
        print(f"  {k} max rel err {err:.3e}", flush=True)
        if k != "omega" or precision == "fp64":
            assert err < tol, k
    if precision == "mixed":
        err = np.max(np.abs(got["omega"][rows] - ref["omega"]) / np.abs(ref["omega"]))
        assert err < 1e-4


@pytest.mark.parametrize("cfg,precision", [("large", "fp64"), ("large", "mixed"),
                                           ("two_phase", "mixed"), ("two_phase", "fp64")])
def test_fullsize_forces_sampled(sph, orc, cfg, precision):
    c = si.config_large() if cfg == "large" else si.config_two_phase()
    s, p = c["state"], c["params"]
    n = len(s["x"])
    print(f"full-size forces {c['name']} {precision}", flush=True)
    st = perturbed_force_inputs(s)
    P = sph.ParticleArrays.from_state(st)
    ctx = sph.Context(dict(p, precision=precision))
    ctx.build_tree(P)
    ctx.forces(P)
    got = P.numpy()
    rows = rows_sample(n)
    Pp, cs = orc.eos(p, st["rho"], st["u"])
    ref = orc.forces(p, st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["m"], st["H"],
                     st["rho"], st["omega"], Pp, cs, rows=rows)
    arms = np.sqrt(np.mean(ref["ax"] ** 2 + ref["ay"] ** 2 + ref["az"] ** 2))
    tol = 1e-12 if precision == "fp64" else 1e-4
    for k in ("ax", "ay", "az"):
        err = np.max(np.abs(got[k][rows] - ref[k])) / arms
        print(f"  {k} max err / rms {err:.3e}", flush=True)
        assert err < tol, k
    # du/dt has no stated bar for the mixed path (reported like a); 10x the
    # acceleration bar guards against gross errors
    durms = np.sqrt(np.mean(ref["dudt"] ** 2))
    du_err = np.max(np.abs(got["dudt"][rows] - ref["dudt"])) / durms
    print(f"  dudt max err / rms {du_err:.3e}", flush=True)
    assert du_err < (tol if precision == "fp64" else 1e-3)
    if precision == "fp64":
        np.testing.assert_allclose(got["dt"][rows], ref["dt"], rtol=1e-12)
    # whole output: pairwise antisymmetry keeps the total momentum change at round-off
    m = st["m"]
    for k in ("ax", "ay", "az"):
        scale = np.sum(m * np.abs(got[k]))
        lim = 1e-12 if precision == "fp64" else 1e-5
        assert abs(np.sum(m * got[k])) < lim * scale, k


def test_fullsize_neighbor_sets_symmetric(sph):
    """Force sets are symmetric (j in F_i <=> i in F_j): the multiset of pairs
    equals its transpose, checked on the whole 2M output through two
    order-independent fingerprints (sums of a non-symmetric hash)."""
    c = si.config_large()
    s, p = c["state"], c["params"]
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(p)
    ctx.build_tree(P)
    off, idx = ctx.neighbors(P, 1)
    n = len(s["x"])
    cnt = off[1:] - off[:-1]
    rowid = torch.repeat_interleave(torch.arange(n, device=off.device), cnt)
    j = idx.to(torch.int64)
    assert int(cnt.sum()) == idx.numel()
    for A, B in ((1000003, 7919), (2654435761, 40503)):
        f = (rowid * A + j * B) % 1000000007
        g = (j * A + rowid * B) % 1000000007
        assert int(f.sum()) == int(g.sum())
    assert ctx.stats()["n_overflow"] == 0


@pytest.fixture(scope="module")
def spheres():
    return si.config_spheres()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_spheres_16m_density_sampled(sph, orc, spheres, precision):
    """The 16.8M-particle open-boundary workload (two spheres, stiffened gas):
    smoothing lengths, densities and Omega of sampled rows against the
    oracle's row-subset solve, in the launch configuration the benchmark
    times."""
    c = spheres
    s, p = c["state"], c["params"]
    n = len(s["x"])
    print(f"spheres density {n} {precision}", flush=True)
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(dict(p, precision=precision))
    ctx.build_tree(P)
    ctx.density(P)
    st = ctx.stats()
    assert st["n_overflow"] == 0
    got = P.numpy()
    rows = rows_sample(n, k=1000, seed=7)
    ref = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"], rows=rows)
    tol = 1e-12 if precision == "fp64" else 1e-5
    for k in ("H", "rho"):
        err = np.max(np.abs(got[k][rows] - ref[k]) / np.abs(ref[k]))
        print(f"  {k} max rel err {err:.3e}", flush=True)
        assert err < tol, k
    err = np.max(np.abs(got["omega"][rows] - ref["omega"]) / np.abs(ref["omega"]))
    assert err < (1e-12 if precision == "fp64" else 1e-4)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_spheres_16m_forces_sampled(sph, orc, spheres, precision):
    """Forces of the 16.8M-particle open-boundary workload (stiffened gas,
    pressure of either sign) on sampled rows against the oracle's row-subset
    force loop, from generated H, rho and Omega."""
    c = spheres
    s, p = c["state"], c["params"]
    n = len(s["x"])
    print(f"spheres forces {n} {precision}", flush=True)
    rng = np.random.default_rng(11)
    st = dict(s, H=s["H"] * rng.uniform(0.97, 1.03, n), rho=rng.uniform(0.95, 1.05, n),
              omega=rng.uniform(0.95, 1.0, n))
    P = sph.ParticleArrays.from_state(st)
    ctx = sph.Context(dict(p, precision=precision))
    ctx.build_tree(P)
    ctx.forces(P)
    assert ctx.stats()["n_overflow"] == 0
    got = P.numpy()
    rows = rows_sample(n, k=1000, seed=13)
    Pp, cs = orc.eos(p, st["rho"], st["u"])
    ref = orc.forces(p, st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["m"], st["H"],
                     st["rho"], st["omega"], Pp, cs, rows=rows)
    arms = np.sqrt(np.mean(ref["ax"] ** 2 + ref["ay"] ** 2 + ref["az"] ** 2))
    tol = 1e-12 if precision == "fp64" else 1e-4
    for k in ("ax", "ay", "az"):
        err = np.max(np.abs(got[k][rows] - ref[k])) / arms
        print(f"  {k} max err / rms {err:.3e}", flush=True)
        assert err < tol, k
    # each sphere moves as a whole (v_ij = 0 inside it, no pair across the gap
    # yet), so du/dt vanishes exactly on both sides
    np.testing.assert_array_equal(ref["dudt"], 0.0)
    np.testing.assert_array_equal(got["dudt"][rows], 0.0)
    if precision == "fp64":
        np.testing.assert_allclose(got["dt"][rows], ref["dt"], rtol=1e-12)
