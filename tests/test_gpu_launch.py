"""Launch shapes of the sweeps on the GPU, through the C interface.

Three shapes run the same per-group arithmetic: sweep kernels that walk the
tree themselves (one workgroup per sink group), and sweep kernels that read
each group's interaction list from a walk kernel run before them, either one
workgroup per group or a persistent grid taking groups from per-XCD queues.
Lists too long to store, and density groups whose root lies beyond the stored
list, go back to the walking kernel.  Every result must equal the walking
shape's bit for bit, and every counter exactly: single sets (clouds, clumped
with dynamic bucket sizing, the interface correction, the entropy update and
the evolved density), a batch of uneven sets, a replayed HIP graph (the
queue counters are cleared inside the graph), fewer groups than resident
workgroups, groups sent back to the walking kernel, and the autotuner's
choice.
"""
import numpy as np
import pytest

import sph_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u", "H", "rho", "omega", "P", "c", "ax", "ay", "az",
          "dudt", "dt")
COUNTERS = ("pairs_density", "pairs_force", "cand_density", "cand_force", "nr_scans",
            "nr_iter_max", "n_noconv", "n_rewalk", "n_overflow", "slots_density", "slots_force",
            "n_retest", "pairs_density_total", "pairs_force_total")


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_11425_amd as m
    return m


def concat_sets(sets):
    keys = sets[0].keys()
    st = {k: np.concatenate([s[k] for s in sets]) for k in keys}
    offs = np.concatenate([[0], np.cumsum([len(s["x"]) for s in sets])])
    return st, offs


def clumped(seed, n=6000):
    """A quarter of the particles in a tight clump inside a uniform box (open
    boundary): long lists next to the clump, short ones inside."""
    c = si.random_cloud(seed, n, kernel="wc4", n_ngb=100, periodic=False)
    s = dict(c["state"])
    rng = np.random.default_rng(seed + 1000)
    k = n // 4
    for key in ("x", "y", "z"):
        v = s[key].copy()
        v[:k] = 0.015 * rng.standard_normal(k)
        s[key] = v
    return s, c["params"]


def cases():
    c = si.random_cloud(21, 5000, kernel="wc4", n_ngb=100, periodic=True)
    yield "cloud", c["state"], c["params"], None
    s, p = clumped(22)
    yield "clumped-dynamic", s, dict(p, dynamic=True, bucket=32), None
    c = si.uniform_box(23, 16, "wc2", 60)
    yield "entropy", c["state"], dict(c["params"], entropy=True), None
    yield "evolved", c["state"], dict(c["params"], evolved=True), None
    c = si.config_two_phase(seed=24, n_side=16)
    yield "interface", c["state"], dict(c["params"], interface=True), None
    b = si.config_batch(seed=25, nsets=6, nmin=512, nmax=4096)
    st, offs = concat_sets(b["sets"])
    yield "batch", st, b["params"], offs.tolist()
    c = si.random_cloud(26, 100, kernel="m4", n_ngb=32, periodic=True)
    yield "two-groups", c["state"], c["params"], None


CASES = list(cases())


def run(sph, state, p, offs, launch, steps=3):
    P = sph.ParticleArrays.from_state(state)
    ctx = sph.Context(dict(p, launch=launch), set_offsets=offs)
    ctx.init(P)
    stats = [ctx.stats()]
    for _ in range(steps):
        ctx.step(P)
        stats.append(ctx.stats())
    out = P.numpy()
    ctx.close()
    return out, stats


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_persistent_equals_per_group(sph, case, precision):
    name, state, p, offs = case
    p = dict(p, precision=precision)
    print(f"launch shapes {name} {precision} n={len(state['x'])}", flush=True)
    w, sw = run(sph, state, p, offs, "walk")
    ngroups = sum((n + 63) // 64 for n in np.diff(offs)) if offs else (len(state["x"]) + 63) // 64
    for shape, code in (("groups", sph.LAUNCH_GROUPS), ("persistent", sph.LAUNCH_PERSISTENT)):
        b, sb = run(sph, state, p, offs, shape)
        for k in FIELDS:
            np.testing.assert_array_equal(w[k], b[k], err_msg=f"{shape} {k}")
        for k, (x, y) in enumerate(zip(sw, sb)):
            assert x["launch"] == sph.LAUNCH_WALK and y["launch"] == code
            for c in COUNTERS:
                assert x[c] == y[c], (shape, k, c)
        # the resident grid: at most one workgroup per sink group
        if shape == "persistent":
            assert 1 <= sb[-1]["workgroups_force"] <= ngroups
        else:
            assert sb[-1]["workgroups_force"] == ngroups
    assert sw[-1]["workgroups_force"] == ngroups


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_persistent_graph_replay(sph, precision):
    c = si.uniform_box(12, 16, "wc2", 100)
    p = dict(c["params"], precision=precision, launch="persistent")
    A = sph.ParticleArrays.from_state(c["state"])
    B = sph.ParticleArrays.from_state(c["state"])
    ca, cb = sph.Context(p), sph.Context(p)
    ca.init(A)
    cb.init(B)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        cb.graph_capture_step(B, 0.0, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        ca.step(A)
        with torch.cuda.stream(s):
            cb.graph_launch(stream=s)
        torch.cuda.synchronize()
        _ = (torch.arange(1000, device="cuda", dtype=torch.float64) ** 2).sum().item()
        a, b = A.numpy(), B.numpy()
        for k in ("x", "vx", "u", "H", "rho", "ax", "dudt", "dt"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"replay {rep} {k}")
        assert ca.stats()["pairs_force"] == cb.stats()["pairs_force"]


def test_autotune_chooses_a_shape(sph):
    c = si.uniform_box(27, 24, "wc4", 200)
    P = sph.ParticleArrays.from_state(c["state"])
    ref = sph.ParticleArrays.from_state(c["state"])
    ctx = sph.Context(dict(c["params"], bucket=0))
    ctx.build_tree(P)   # (the trials start from the generator's H, as sph_init below does)
    b = ctx.autotune(P)
    st = ctx.stats()
    print(f"autotune: bucket {b}, launch {st['launch']}, workgroups {st['workgroups_force']}",
          flush=True)
    assert b in (8, 16, 32, 64)
    assert st["launch"] in (sph.LAUNCH_GROUPS, sph.LAUNCH_PERSISTENT, sph.LAUNCH_WALK)
    # the state it leaves is sph_init's with the chosen shape
    c2 = sph.Context(dict(c["params"], bucket=b, launch=int(st["launch"])))
    c2.init(ref)
    got, want = P.numpy(), ref.numpy()
    for k in ("H", "rho", "ax", "dudt", "dt"):
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)


def test_launch_parameter_checked(sph):
    c = si.uniform_box(28, 8, "m4", 32)
    with pytest.raises(sph.SphError):
        sph.Context(dict(c["params"], launch=3))
    with pytest.raises(sph.SphError):
        sph.Context(dict(c["params"], launch="persistent", rungs=True, rung_max=4))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("guess", [0.5, 0.3], ids=["long-lists", "root-beyond-list"])
def test_groups_sent_back_to_the_walking_kernel(sph, precision, guess):
    """A first guess of H far from the root: at 0.5 (the cap with h_max 0.5)
    the density pass's stored lists would exceed 4096 buckets of 8, so the
    groups go back to the walking kernel; at 0.3 of the converged H the root
    lies beyond the stored list's radius, and the group leaves the listed
    kernel when its iteration wants a new walk.  Either way the results equal
    the walking shape's bit for bit."""
    c = si.random_cloud(31, 60000, kernel="wc4", n_ngb=100, periodic=True)
    s, p = dict(c["state"]), dict(c["params"], precision=precision, bucket=8, h_max=0.5)
    if guess == 0.3:
        s["H"] = 0.3 * s["H"]
    else:
        s["H"] = np.full_like(s["H"], guess)
    print(f"groups sent back: {precision}, H guess {guess}", flush=True)
    w, sw = run(sph, s, p, None, "walk", steps=1)
    assert sw[0]["groups_walked"] == 0
    for shape in ("groups", "persistent"):
        b, sb = run(sph, s, p, None, shape, steps=1)
        for k in FIELDS:
            np.testing.assert_array_equal(w[k], b[k], err_msg=f"{shape} {k}")
        for c_ in COUNTERS:
            assert sw[0][c_] == sb[0][c_], (shape, c_)
        print(f"  {shape} init: {sb[0]['groups_walked']} of {(60000 + 63) // 64} groups walked "
              f"again, {sb[0]['n_rewalk']} new walks", flush=True)
        assert sb[0]["groups_walked"] > 0
