"""GPU path on perfect cubic lattices against closed forms (no oracle involved).

On a periodic lattice of spacing a every particle sees the same neighbourhood,
so the quantities of Sec. 2.3.3 reduce to sums over lattice vectors n in Z^3:

  * density at fixed H: rho = m sigma / H^3 sum_{|n| a < H} f(|n| a / H), self
    term included (eq:Density_estimate);
  * the smoothing length solving (4 pi / 3) H^3 rho = n_ngb m: the root of a
    scalar function of H / a, found here by a library bracketing solver on the
    enumerated sum;
  * gather neighbour counts: the number of lattice vectors with 0 < |n|^2 <
    (H/a)^2, i.e. sums of the representation counts r3(k) of k as a sum of
    three squares (tests/golden/lattice_shells.json);
  * at rest with uniform u, every pair force has an opposite partner, so a and
    du/dt vanish to round-off, and the time step is the Courant limit of a
    particle with sound speed c and no approaching neighbours (Sec. 2.3.6).

Both precisions run; the FP64 path meets 1e-12 relative, the mixed path its
1e-5 density bar.
"""
import json
import os

import numpy as np
import pytest
from scipy import optimize

import sph_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lattice_shells.json")
SIGMA = {"m4": 8.0 / np.pi, "wc2": 21.0 / (2.0 * np.pi), "wc4": 495.0 / (32.0 * np.pi),
         "wc6": 1365.0 / (64.0 * np.pi)}


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_11425_amd as m
    return m


def shape(kernel, q):
    """Kernel shapes f(q) on 0 <= q < 1 (Monaghan's cubic spline; Wendland C2, C4, C6)."""
    s = 1.0 - q
    if kernel == "m4":
        return np.where(q < 0.5, 1.0 - 6.0 * q * q + 6.0 * q ** 3, 2.0 * s ** 3)
    if kernel == "wc2":
        return s ** 4 * (1.0 + 4.0 * q)
    if kernel == "wc4":
        return s ** 6 * (1.0 + 6.0 * q + 35.0 / 3.0 * q * q)
    return s ** 8 * (1.0 + 8.0 * q + 25.0 * q * q + 32.0 * q ** 3)


def lattice_sum(kernel, h, reach=8):
    v = np.arange(-reach, reach + 1)
    a, b, c = np.meshgrid(v, v, v, indexing="ij")
    r = np.sqrt((a * a + b * b + c * c).ravel().astype(np.float64))
    q = r[r < h] / h
    return float(np.sum(shape(kernel, q)))


def shell_count(h):
    r3 = json.load(open(GOLDEN))["r3"]
    return sum(r3[k] for k in range(1, len(r3)) if k < h * h)


CASES = [("m4", 2.5), ("wc2", 3.1), ("wc4", 3.63), ("wc6", 3.9)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kernel,h", CASES)
def test_lattice_density_at_fixed_H(sph, kernel, h, precision):
    n_side = 16
    c = si.perfect_lattice(n_side, kernel, 64, H=h / n_side)
    s, p = c["state"], c["params"]
    print(f"lattice density {kernel} H/a={h} {precision}", flush=True)
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(dict(p, precision=precision))
    ctx.build_tree(P)
    off, idx = ctx.neighbors(P, 0)
    counts = np.diff(off.cpu().numpy())
    assert np.all(counts == shell_count(h))
    # density at the given H: one scan with the target set to the lattice's
    # own kernel mass, so the iteration accepts H as it is
    nb = 4.0 * np.pi / 3.0 * SIGMA[kernel] * lattice_sum(kernel, h)
    ctx2 = sph.Context(dict(p, precision=precision, n_ngb=nb))
    ctx2.build_tree(P)
    ctx2.density(P)
    got = P.numpy()
    m = 1.0 / n_side ** 3
    H = h / n_side
    expect = m * SIGMA[kernel] / H ** 3 * lattice_sum(kernel, h)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.max(np.abs(got["rho"] / expect - 1.0)) < tol
    assert np.max(np.abs(got["H"] / H - 1.0)) < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kernel,n_ngb", [("m4", 64), ("wc4", 200)])
def test_lattice_root_and_rest(sph, kernel, n_ngb, precision):
    sig = SIGMA[kernel]
    root = optimize.brentq(lambda h: 4.0 * np.pi / 3.0 * sig * lattice_sum(kernel, h) - n_ngb,
                           1.0, 6.0, xtol=1e-15, rtol=1e-15)
    n_side = 16
    u = 1.3
    c = si.perfect_lattice(n_side, kernel, n_ngb, u=u)
    s, p = c["state"], c["params"]
    print(f"lattice root {kernel} n_ngb={n_ngb} {precision}", flush=True)
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(dict(p, precision=precision))
    ctx.init(P)
    got = P.numpy()
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.max(np.abs(got["H"] * n_side / root - 1.0)) < tol
    m = 1.0 / n_side ** 3
    H = root / n_side
    rho = m * sig / H ** 3 * lattice_sum(kernel, root)
    assert np.max(np.abs(got["rho"] / rho - 1.0)) < tol
    # at rest: the pair terms cancel in opposite pairs
    gam = p["gamma"]
    P0 = (gam - 1.0) * rho * u
    A = P0 / (got["omega"][0] * rho * rho)
    scale = m * A * H ** -4 * 100.0   # a pair term is of order m A |dW/dr| ~ m A / H^4
    eps = 1e-12 if precision == "fp64" else 1e-5
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(got[k])) < eps * scale, k
    assert np.max(np.abs(got["dudt"])) < eps * scale * 1e-3
    # time step: Courant limit with c = sqrt(gamma (gamma - 1) u), h = H / 2
    c0 = np.sqrt(gam * (gam - 1.0) * u)
    dt = min(p["eta_c"] * 0.5 * H / ((1.0 + 0.6 * p["alpha"]) * c0), p["dt_max"])
    assert np.max(np.abs(got["dt"] / dt - 1.0)) < (1e-12 if precision == "fp64" else 1e-5)
