"""Pins of the oracle's neighbour sets (Sec. 2.3.2, "smaller than the kernel size").

The oracle finds neighbours through a uniform cell list.  It is pinned against
an O(N^2) dense-matrix brute force on small sets (periodic, open, clumped),
against the shell counts of a perfect cubic lattice (sums of three squares,
tests/golden/lattice_shells.json), and against the set identities (gather
set inside the force set; the force set is symmetric).
"""
import json
import os

import numpy as np
import pytest

import sph_inputs as si

GOLD = os.path.join(os.path.dirname(__file__), "golden", "lattice_shells.json")


def brute_sets(params, x, y, z, H, mode):
    """Dense all-pairs distances with the same minimum-image convention."""
    P = np.stack([x, y, z])
    d = P[:, None, :] - P[:, :, None]  # d[a, i, j] = x_j - x_i
    if params.get("periodic", True):
        lo = np.array(params["box_lo"])[:, None, None]
        hi = np.array(params["box_hi"])[:, None, None]
        L = hi - lo
        half = 0.5 * L
        d = np.where(d > half, d - L, np.where(d < -half, d + L, d))
    r2 = d[0] * d[0] + d[1] * d[1]
    r2 = r2 + d[2] * d[2]
    Hi2 = (H * H)[:, None]
    if mode == 0:
        ok = r2 < Hi2
    else:
        Hs = np.maximum(H[:, None], H[None, :])
        ok = r2 < Hs * Hs
    np.fill_diagonal(ok, False)
    return [np.nonzero(row)[0] for row in ok]


@pytest.mark.parametrize("case", [
    dict(seed=1, n=600, periodic=True, clumped=False),
    dict(seed=2, n=900, periodic=True, clumped=True),
    dict(seed=3, n=700, periodic=False, clumped=True),
    dict(seed=4, n=1, periodic=True, clumped=False),
    dict(seed=5, n=2, periodic=False, clumped=False),
])
@pytest.mark.parametrize("mode", [0, 1])
def test_against_brute_force(orc, case, mode):
    c = si.random_cloud(case["seed"], case["n"], periodic=case["periodic"], clumped=case["clumped"])
    s, p = c["state"], c["params"]
    rng = np.random.default_rng(case["seed"] + 100)
    H = s["H"] * rng.uniform(0.5, 1.8, s["H"].size)
    off, idx = orc.neighbors(p, s["x"], s["y"], s["z"], H, mode)
    ref = brute_sets(p, s["x"], s["y"], s["z"], H, mode)
    for i in range(len(ref)):
        assert np.array_equal(idx[off[i]:off[i + 1]], ref[i]), i


def test_set_identities(orc):
    c = si.random_cloud(11, 800, clumped=True)
    s, p = c["state"], c["params"]
    H = s["H"] * np.random.default_rng(3).uniform(0.5, 2.0, s["H"].size)
    og, ig = orc.neighbors(p, s["x"], s["y"], s["z"], H, 0)
    of, if_ = orc.neighbors(p, s["x"], s["y"], s["z"], H, 1)
    n = len(H)
    F = [set(if_[of[i]:of[i + 1]].tolist()) for i in range(n)]
    for i in range(n):
        assert set(ig[og[i]:og[i + 1]].tolist()) <= F[i]
        for j in F[i]:
            assert i in F[j]


def test_golden_shells_are_sums_of_three_squares():
    r3 = json.load(open(GOLD))["r3"]
    v = np.arange(-5, 6)
    a, b, c = np.meshgrid(v, v, v, indexing="ij")
    k = (a * a + b * b + c * c).ravel()
    for kk in range(len(r3)):
        assert int(np.sum(k == kk)) == r3[kk]


@pytest.mark.parametrize("H_over_a,kmax", [(2.4823, 6), (3.6271, 13), (1.2, 1), (2.0, 3)])
def test_perfect_lattice_shell_counts(orc, H_over_a, kmax):
    r3 = json.load(open(GOLD))["r3"]
    n_side = 16
    c = si.perfect_lattice(n_side, "m4", 64, H=H_over_a / n_side)
    s, p = c["state"], c["params"]
    off, idx = orc.neighbors(p, s["x"], s["y"], s["z"], s["H"], 0)
    expect = sum(r3[1:kmax + 1])
    assert np.all(np.diff(off) == expect)
