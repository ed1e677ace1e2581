"""Pins of the oracle's density sum, grad-h term and smoothing-length solve
(Sec. 2.3.3: eq:Density_estimate, the Omega term, constant kernel mass).

Pins: the perfect-lattice density by direct enumeration of lattice vectors
(a different summation from the cell list); the continuum limit rho a^3 / m
-> 1 for large H/a (normalisation seen through the discrete sum, with the self
term); invariance under periodic translation and open-boundary rotation;
the scaling laws in mass and length; Omega against a finite difference of
rho(H); the solve's residual; and the lattice root found by a library
bracketing root finder.
"""
import numpy as np
import pytest
from scipy import optimize
from scipy.spatial.transform import Rotation

import sph_inputs as si


def lattice_sum(orc, kernel, H_over_a, reach=8):
    """sum_{n in Z^3, |n| < H/a} f(|n| a / H), self included."""
    v = np.arange(-reach, reach + 1)
    a, b, c = np.meshgrid(v, v, v, indexing="ij")
    r = np.sqrt((a * a + b * b + c * c).ravel().astype(np.float64))
    q = r / H_over_a
    q = q[q < 1.0]
    f, _ = orc.kernel_shape(kernel, q)
    return float(np.sum(f))


@pytest.mark.parametrize("kernel,H_over_a", [("m4", 2.5), ("wc2", 3.1), ("wc4", 3.63), ("wc6", 4.2)])
def test_perfect_lattice_density(orc, kernel, H_over_a):
    n_side = 16
    c = si.perfect_lattice(n_side, kernel, 64, H=H_over_a / n_side)
    s, p = c["state"], c["params"]
    rho, drho, om, cnt = orc.density(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    m = 1.0 / n_side ** 3
    H = H_over_a / n_side
    expect = m * orc.sigma(kernel) / H ** 3 * lattice_sum(orc, kernel, H_over_a)
    np.testing.assert_allclose(rho, expect, rtol=1e-12)


@pytest.mark.parametrize("kernel", ["m4", "wc2", "wc4", "wc6"])
def test_continuum_limit(orc, kernel):
    # rho a^3 / m -> 1 as H/a grows (Poisson summation of a normalised kernel)
    dev = [abs(orc.sigma(kernel) / h ** 3 * lattice_sum(orc, kernel, h, reach=int(h) + 2) - 1.0)
           for h in (4.0, 10.0)]
    assert dev[1] < 3e-6 and dev[1] < dev[0] / 30.0


def test_translation_and_scaling_invariance(orc):
    c = si.random_cloud(21, 700, kernel="wc4", n_ngb=50, clumped=True)
    s, p = c["state"], c["params"]
    x, y, z, m, H = s["x"], s["y"], s["z"], s["m"], s["H"] * 1.3
    rho, drho, om, cnt = orc.density(p, x, y, z, m, H)
    sh = np.array([0.3125, 0.6875, 0.1875])  # dyadic: the shift itself is exact
    xs = np.mod(x + sh[0], 1.0)
    ys = np.mod(y + sh[1], 1.0)
    zs = np.mod(z + sh[2], 1.0)
    rho2, _, om2, cnt2 = orc.density(p, xs, ys, zs, m, H)
    np.testing.assert_allclose(rho2, rho, rtol=1e-12)
    np.testing.assert_allclose(om2, om, rtol=1e-11)
    rho3, _, _, _ = orc.density(p, x, y, z, 3.0 * m, H)
    np.testing.assert_allclose(rho3, 3.0 * rho, rtol=1e-14)
    # length scaling: box and positions by 2 (exact in binary), H by 2 -> rho / 8
    p2 = dict(p, box_hi=(2.0, 2.0, 2.0), h_max=0.9)
    rho4, _, om4, _ = orc.density(p2, 2 * x, 2 * y, 2 * z, m, 2 * H)
    np.testing.assert_allclose(rho4 * 8.0, rho, rtol=1e-13)
    np.testing.assert_allclose(om4, om, rtol=1e-12)


def test_rotation_invariance_open(orc):
    c = si.random_cloud(22, 600, kernel="m4", n_ngb=40, periodic=False, clumped=True)
    s, p = c["state"], c["params"]
    R = Rotation.from_euler("xyz", [0.3, -1.1, 2.0]).as_matrix()
    P = np.stack([s["x"], s["y"], s["z"]])
    Q = R @ P
    rho, _, om, cnt = orc.density(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    rho2, _, om2, cnt2 = orc.density(p, Q[0], Q[1], Q[2], s["m"], s["H"])
    np.testing.assert_allclose(rho2, rho, rtol=1e-10)
    np.testing.assert_allclose(om2, om, rtol=1e-9)


@pytest.mark.parametrize("kernel", ["m4", "wc4"])
def test_omega_is_log_derivative(orc, kernel):
    c = si.random_cloud(23, 500, kernel=kernel, n_ngb=60, clumped=True)
    s, p = c["state"], c["params"]
    H = s["H"]
    e = 1e-6
    rho, drho, om, _ = orc.density(p, s["x"], s["y"], s["z"], s["m"], H)
    rp, _, _, _ = orc.density(p, s["x"], s["y"], s["z"], s["m"], H * (1 + e))
    rm, _, _, _ = orc.density(p, s["x"], s["y"], s["z"], s["m"], H * (1 - e))
    fd = (rp - rm) / (2 * e * H)
    np.testing.assert_allclose(drho, fd, rtol=1e-6, atol=1e-8 * np.max(np.abs(drho)))
    np.testing.assert_allclose(om, 1.0 + H * drho / (3.0 * rho), rtol=1e-14)


@pytest.mark.parametrize("kernel,n_ngb", [("m4", 64), ("wc2", 100), ("wc4", 200), ("wc6", 200)])
def test_solve_h_residual(orc, kernel, n_ngb):
    c = si.random_cloud(24, 3000, kernel=kernel, n_ngb=n_ngb, clumped=True)
    s, p = c["state"], c["params"]
    d = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"] * 0.7)
    assert d["n_noconv"] == 0
    res = 4.0 * np.pi / 3.0 * d["H"] ** 3 * d["rho"] / (n_ngb * s["m"]) - 1.0
    assert np.max(np.abs(res)) < 1e-12
    # a different starting guess converges to the same root
    d2 = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"] * 1.6)
    np.testing.assert_allclose(d2["H"], d["H"], rtol=1e-13)
    # re-evaluating the density at the returned H gives the returned rho and Omega
    rho, _, om, cnt = orc.density(p, s["x"], s["y"], s["z"], s["m"], d["H"])
    np.testing.assert_allclose(rho, d["rho"], rtol=1e-13)
    np.testing.assert_allclose(om, d["omega"], rtol=1e-12)
    np.testing.assert_array_equal(cnt, d["count"])


@pytest.mark.parametrize("kernel,n_ngb", [("m4", 64), ("wc4", 200)])
def test_lattice_root(orc, kernel, n_ngb):
    sig = orc.sigma(kernel)

    def F(h):  # h = H / a; (4 pi / 3) H^3 rho / m - n_ngb on the lattice
        return 4.0 * np.pi / 3.0 * sig * lattice_sum(orc, kernel, h) - n_ngb

    root = optimize.brentq(F, 1.0, 6.0, xtol=1e-15, rtol=1e-15)
    n_side = 16
    c = si.perfect_lattice(n_side, kernel, n_ngb)
    s, p = c["state"], c["params"]
    d = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    np.testing.assert_allclose(d["H"] * n_side, root, rtol=1e-12)


def test_capped_particles_are_counted(orc):
    c = si.random_cloud(25, 300, kernel="m4", n_ngb=64, periodic=False)
    s, p = c["state"], c["params"]
    p = dict(p, h_max=0.05)
    d = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    assert d["n_noconv"] > 0
    assert np.all(d["H"] <= 0.05)
