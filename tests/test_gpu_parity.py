"""GPU path against the FP64 oracle, through the C interface.

Bars (stated for the sweep): neighbour sets bit-exact given the same H; FP64
path H, rho, Omega within 1e-12 relative per particle; a and du/dt within
1e-12 of their rms (per-particle relative error is ill-posed for nearly
cancelling sums); time-step limits within 1e-12 relative.  Mixed path: rho
within 1e-5 relative, a within 1e-4 of rms |a|.
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


def rel(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def rms_err(a, b, ref_rms):
    return np.max(np.abs(a - b)) / ref_rms


def csr_rows(off, idx, n):
    off = np.asarray(off)
    idx = np.asarray(idx)
    return [idx[off[i]:off[i + 1]] for i in range(n)]


CLOUDS = [
    dict(seed=1, n=3000, periodic=True, clumped=False, kernel="m4", n_ngb=50),
    dict(seed=2, n=5000, periodic=True, clumped=True, kernel="wc4", n_ngb=100),
    dict(seed=3, n=4001, periodic=False, clumped=True, kernel="wc2", n_ngb=60),
    dict(seed=4, n=777, periodic=False, clumped=False, kernel="wc6", n_ngb=120),
]


def cloud(case):
    return si.random_cloud(case["seed"], case["n"], kernel=case["kernel"], n_ngb=case["n_ngb"],
                           periodic=case["periodic"], clumped=case["clumped"])


@pytest.mark.parametrize("case", CLOUDS, ids=lambda c: f"n{c['n']}-{c['kernel']}")
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("bucket", [8, 16, 32, 64])
def test_neighbor_sets_bit_exact(sph, orc, case, mode, bucket):
    c = cloud(case)
    s, p = c["state"], c["params"]
    rng = np.random.default_rng(case["seed"] + 7)
    s = dict(s, H=s["H"] * rng.uniform(0.6, 1.6, s["H"].size))
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(dict(p, bucket=bucket))
    print(f"neighbors {c['name']} mode={mode} B={bucket}", flush=True)
    ctx.build_tree(P)
    off, idx = ctx.neighbors(P, mode)
    ro, ri = orc.neighbors(p, s["x"], s["y"], s["z"], s["H"], mode)
    np.testing.assert_array_equal(off.cpu().numpy(), ro)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), ri)
    assert ctx.stats()["n_overflow"] == 0


def test_neighbor_sets_config_small(sph, orc):
    c = si.config_small()
    s, p = c["state"], c["params"]
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(p)
    ctx.build_tree(P)
    for mode in (0, 1):
        off, idx = ctx.neighbors(P, mode)
        ro, ri = orc.neighbors(p, s["x"], s["y"], s["z"], s["H"], mode)
        np.testing.assert_array_equal(off.cpu().numpy(), ro)
        np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), ri)


@pytest.mark.parametrize("case", CLOUDS, ids=lambda c: f"n{c['n']}-{c['kernel']}")
def test_density_fp64(sph, orc, case):
    c = cloud(case)
    s, p = c["state"], c["params"]
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(p)
    print(f"density {c['name']}", flush=True)
    ctx.build_tree(P)
    ctx.density(P)
    st = ctx.stats()
    got = P.numpy()
    ref = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    assert st["n_noconv"] == ref["n_noconv"]
    assert rel(got["H"], ref["H"]) < 1e-12
    assert rel(got["rho"], ref["rho"]) < 1e-12
    assert rel(got["omega"], ref["omega"]) < 1e-12
    assert st["pairs_density"] == int(ref["count"].sum())
    assert st["n_overflow"] == 0


def force_inputs(orc, c):
    s, p = c["state"], c["params"]
    d = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    Pp, cs = orc.eos(p, d["rho"], s["u"])
    ref = orc.forces(p, s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"], d["H"],
                     d["rho"], d["omega"], Pp, cs)
    st = dict(s, H=d["H"], rho=d["rho"], omega=d["omega"])
    return st, ref, Pp, cs


@pytest.mark.parametrize("case", CLOUDS, ids=lambda c: f"n{c['n']}-{c['kernel']}")
def test_forces_fp64(sph, orc, case):
    c = cloud(case)
    s, p = c["state"], c["params"]
    st, ref, Pp, cs = force_inputs(orc, c)
    P = sph.ParticleArrays.from_state(st)
    ctx = sph.Context(p)
    print(f"forces {c['name']}", flush=True)
    ctx.build_tree(P)
    ctx.forces(P)
    got = P.numpy()
    arms = np.sqrt(np.mean(ref["ax"] ** 2 + ref["ay"] ** 2 + ref["az"] ** 2))
    for k in ("ax", "ay", "az"):
        assert rms_err(got[k], ref[k], arms) < 1e-12, k
    durms = np.sqrt(np.mean(ref["dudt"] ** 2))
    assert rms_err(got["dudt"], ref["dudt"], durms) < 1e-12
    assert rel(got["dt"], ref["dt"]) < 1e-12
    assert rel(got["P"], Pp) < 1e-14 and rel(got["c"] + 1e-300, cs + 1e-300) < 1e-14
    assert ctx.stats()["pairs_force"] == int(ref["count"].sum())


def test_init_and_step_config_small(sph, orc):
    c = si.config_small()
    s, p = c["state"], c["params"]
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(p)
    ctx.init(P)
    ref = orc.init(p, s)
    got = P.numpy()
    for k in ("H", "rho", "omega"):
        assert rel(got[k], ref[k]) < 1e-12, k
    arms = np.sqrt(np.mean(ref["ax"] ** 2 + ref["ay"] ** 2 + ref["az"] ** 2))
    for k in ("ax", "ay", "az"):
        assert rms_err(got[k], ref[k], arms) < 1e-11, k
    st0 = ctx.stats()
    assert st0["pairs_density"] == ref["n_d"] and st0["pairs_force"] == ref["n_f"]
    ctx.step(P)
    rep = orc.step(p, ref)
    got = P.numpy()
    st = ctx.stats()
    assert abs(st["dt_used"] - rep["dt"]) <= 1e-12 * rep["dt"]
    for k in ("x", "y", "z"):
        assert np.max(np.abs(got[k] - ref[k])) < 1e-13, k
    for k in ("H", "rho", "omega"):
        assert rel(got[k], ref[k]) < 1e-11, k
    arms = np.sqrt(np.mean(ref["ax"] ** 2 + ref["ay"] ** 2 + ref["az"] ** 2))
    for k in ("ax", "ay", "az"):
        assert rms_err(got[k], ref[k], arms) < 1e-10, k
    vrms = np.sqrt(np.mean(ref["vx"] ** 2))
    assert rms_err(got["vx"], ref["vx"], vrms) < 1e-12
    assert abs(st["e_kin"] + st["e_int"] - rep["e_tot"]) < 1e-12 * rep["e_tot"]
    for a in range(3):
        assert abs(st["momentum"][a] - rep["momentum"][a]) < 1e-15 * np.sum(ref["m"] * np.abs(ref["vx"]))


@pytest.mark.parametrize("case", CLOUDS[:2], ids=lambda c: f"n{c['n']}-{c['kernel']}")
def test_mixed_precision_bounds(sph, orc, case):
    c = cloud(case)
    s, p = c["state"], c["params"]
    st, ref, Pp, cs = force_inputs(orc, c)
    # density from the original guess
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(dict(p, precision="mixed"))
    ctx.build_tree(P)
    ctx.density(P)
    got = P.numpy()
    dref = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    assert rel(got["rho"], dref["rho"]) < 1e-5
    assert rel(got["H"], dref["H"]) < 1e-5
    # forces from the oracle's H, rho, Omega
    P2 = sph.ParticleArrays.from_state(st)
    ctx.build_tree(P2)
    ctx.forces(P2)
    g2 = P2.numpy()
    arms = np.sqrt(np.mean(ref["ax"] ** 2 + ref["ay"] ** 2 + ref["az"] ** 2))
    for k in ("ax", "ay", "az"):
        assert rms_err(g2[k], ref[k], arms) < 1e-4, k


def test_empty_and_single_particle(sph):
    p = si.params(kernel="m4", n_ngb=64)
    for n in (0, 1):
        s = {k: np.full(n, 0.5) for k in ("x", "y", "z", "m", "u")}
        s.update({k: np.zeros(n) for k in ("vx", "vy", "vz")})
        s["H"] = np.full(n, 0.1)
        P = sph.ParticleArrays.from_state(s) if n else None
        ctx = sph.Context(p)
        if n == 0:
            t = {f: torch.zeros(0, dtype=torch.float64, device="cuda") for f in sph.FIELDS}
            P = sph.ParticleArrays(t)
        ctx.init(P)
        torch.cuda.synchronize()
        st = ctx.stats()
        assert st["pairs_density"] == 0
        if n == 1:
            got = P.numpy()
            # lone particle: H grows to the cap, the cap is reported
            assert st["n_noconv"] == 1
            assert got["ax"][0] == 0.0


def test_determinism(sph):
    c = si.random_cloud(9, 6000, kernel="wc4", n_ngb=80, clumped=True)
    outs = []
    for _ in range(2):
        P = sph.ParticleArrays.from_state(c["state"])
        ctx = sph.Context(c["params"])
        ctx.init(P)
        ctx.step(P)
        outs.append(P.numpy())
    for k in ("x", "H", "rho", "ax", "dudt", "dt"):
        np.testing.assert_array_equal(outs[0][k], outs[1][k])


def test_walk_fallback_is_exact(sph, orc):
    """A tiny walk stack forces every group onto the linear bucket test; sets
    stay bit-exact and the density stays within the FP64 bar."""
    c = cloud(CLOUDS[1])
    s, p = c["state"], c["params"]
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(dict(p, stack_limit=2))
    ctx.build_tree(P)
    for mode in (0, 1):
        off, idx = ctx.neighbors(P, mode)
        assert ctx.stats()["n_overflow"] > 0
        ro, ri = orc.neighbors(p, s["x"], s["y"], s["z"], s["H"], mode)
        np.testing.assert_array_equal(off.cpu().numpy(), ro)
        np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), ri)
    ctx.density(P)
    assert ctx.stats()["n_overflow"] > 0
    got = P.numpy()
    ref = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    assert rel(got["rho"], ref["rho"]) < 1e-12
    st, fref, Pp, cs = force_inputs(orc, c)
    Q = sph.ParticleArrays.from_state(st)
    ctx.build_tree(Q)
    ctx.forces(Q)
    assert ctx.stats()["n_overflow"] > 0
    g = Q.numpy()
    arms = np.sqrt(np.mean(fref["ax"] ** 2 + fref["ay"] ** 2 + fref["az"] ** 2))
    assert rms_err(g["ax"], fref["ax"], arms) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_paused_walk_resumes(sph, orc, precision):
    """Small buckets and many neighbours: a group's candidate buckets exceed
    the candidate list, so the walk pauses, the tiles consume the list and
    the walk resumes (several times per scan).  Results meet the same bars."""
    c = si.random_cloud(11, 6000, kernel="wc4", n_ngb=300, periodic=True, clumped=True)
    s, p = c["state"], dict(c["params"], bucket=8, precision=precision)
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(p)
    print(f"paused walk {precision}", flush=True)
    ctx.build_tree(P)
    ctx.density(P)
    st = ctx.stats()
    assert st["n_overflow"] == 0
    # more candidate buckets per group than the list holds (256)
    assert st["cand_density"] / max(1, st["nr_scans"]) > 64 * 256 * 8
    got = P.numpy()
    ref = orc.solve_h(c["params"], s["x"], s["y"], s["z"], s["m"], s["H"])
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert rel(got["rho"], ref["rho"]) < tol
    assert rel(got["H"], ref["H"]) < tol
    if precision == "fp64":
        assert st["pairs_density"] == int(ref["count"].sum())
    st2, fref, Pp, cs = force_inputs(orc, c)
    Q = sph.ParticleArrays.from_state(st2)
    ctx.build_tree(Q)
    ctx.forces(Q)
    g = Q.numpy()
    arms = np.sqrt(np.mean(fref["ax"] ** 2 + fref["ay"] ** 2 + fref["az"] ** 2))
    for k in ("ax", "ay", "az"):
        assert rms_err(g[k], fref[k], arms) < (1e-12 if precision == "fp64" else 1e-4), k
    if precision == "fp64":
        assert ctx.stats()["pairs_force"] == int(fref["count"].sum())


def degenerate_cloud():
    """A clumped periodic cloud where 100 particles sit exactly on top of
    others (r = 0 pairs) and ten lie on the box faces (x = 0, y just below 1)."""
    c = si.random_cloud(21, 2000, kernel="wc4", n_ngb=80, periodic=True, clumped=True)
    s = c["state"]
    rng = np.random.default_rng(5)
    dup = rng.choice(2000, 100, replace=False)
    src = rng.choice(2000, 100, replace=False)
    for k in ("x", "y", "z"):
        s[k][dup] = s[k][src]
    s["x"][:5] = 0.0
    s["y"][5:10] = np.nextafter(1.0, 0.0)
    return c


def test_coincident_and_face_particles(sph, orc):
    """Pairs at r = 0 count as neighbours and exert neither force nor heating
    (Sec. 2.3.5 with x_ij = 0); particles on the box faces find their
    neighbours through the minimum image.  FP64 to the usual bars, the
    neighbour counts exactly; the mixed path finite and within its bars."""
    c = degenerate_cloud()
    s, p = c["state"], c["params"]
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(p)
    print("coincident and face particles fp64", flush=True)
    ctx.build_tree(P)
    ctx.density(P)
    got = P.numpy()
    ref = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    for k in ("H", "rho", "omega"):
        assert rel(got[k], ref[k]) < 1e-12, k
    assert ctx.stats()["pairs_density"] == int(ref["count"].sum())
    st, fref, Pp, cs = force_inputs(orc, c)
    P2 = sph.ParticleArrays.from_state(st)
    ctx.build_tree(P2)
    ctx.forces(P2)
    g2 = P2.numpy()
    arms = np.sqrt(np.mean(fref["ax"] ** 2 + fref["ay"] ** 2 + fref["az"] ** 2))
    for k in ("ax", "ay", "az"):
        assert rms_err(g2[k], fref[k], arms) < 1e-12, k
    durms = np.sqrt(np.mean(fref["dudt"] ** 2))
    assert rms_err(g2["dudt"], fref["dudt"], durms) < 1e-12
    assert ctx.stats()["pairs_force"] == int(fref["count"].sum())
    # mixed precision on the same inputs
    cm = sph.Context(dict(p, precision="mixed"))
    P3 = sph.ParticleArrays.from_state(st)
    cm.build_tree(P3)
    cm.forces(P3)
    g3 = P3.numpy()
    assert all(np.all(np.isfinite(g3[k])) for k in ("ax", "ay", "az", "dudt", "dt"))
    for k in ("ax", "ay", "az"):
        assert rms_err(g3[k], fref[k], arms) < 1e-4, k


@pytest.mark.parametrize("n,n_ngb", [(300, 150), (400, 100)])
def test_smoothing_length_at_the_cap(sph, orc, n, n_ngb):
    """Few particles, many neighbours: most (or some) smoothing lengths reach
    the cap of 0.45 of the periodic box, where every sink group's
    neighbourhood wraps the box.  The capped particles are counted and every
    result equals the oracle's (FP64) or stays within the mixed bars."""
    c = si.random_cloud(31, n, kernel="m4", n_ngb=n_ngb, periodic=True, clumped=False)
    s, p = c["state"], c["params"]
    ref = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    print(f"H at the cap n={n} n_ngb={n_ngb}: {ref['n_noconv']} capped", flush=True)
    for precision, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
        P = sph.ParticleArrays.from_state(s)
        ctx = sph.Context(dict(p, precision=precision))
        ctx.build_tree(P)
        ctx.density(P)
        got = P.numpy()
        st = ctx.stats()
        assert st["n_noconv"] == ref["n_noconv"], precision
        for k in ("H", "rho"):
            assert rel(got[k], ref[k]) < tol, (precision, k)
        if precision == "fp64":
            assert st["pairs_density"] == int(ref["count"].sum())
    st2, fref, Pp, cs = force_inputs(orc, c)
    P2 = sph.ParticleArrays.from_state(st2)
    ctx = sph.Context(p)
    ctx.build_tree(P2)
    ctx.forces(P2)
    g2 = P2.numpy()
    arms = np.sqrt(np.mean(fref["ax"] ** 2 + fref["ay"] ** 2 + fref["az"] ** 2))
    for k in ("ax", "ay", "az"):
        assert rms_err(g2[k], fref[k], arms) < 1e-12, k
    assert ctx.stats()["pairs_force"] == int(fref["count"].sum())
