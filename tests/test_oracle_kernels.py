"""Pins of the oracle's kernel family (Sec. 2.3: cubic spline and Wendland C2/C4/C6).

The paper cites the kernels without printing them, so they are pinned by what
any normalised compact kernel must satisfy: unit integral over its support
(checked by adaptive quadrature, not by the closed-form sigma), f(0) = 1
(the self term), monotone decrease, vanishing value and slope at the edge,
continuity of the cubic spline's pieces, and derivatives that agree with
finite differences of the value.
"""
import numpy as np
import pytest
from scipy import integrate

KERNELS = ["m4", "wc2", "wc4", "wc6"]


@pytest.mark.parametrize("k", KERNELS)
def test_unit_normalisation(orc, k):
    sig = orc.sigma(k)

    def integrand(q):
        f, _ = orc.kernel_shape(k, np.array([q]))
        return 4.0 * np.pi * sig * f[0] * q * q

    val, err = integrate.quad(integrand, 0.0, 1.0, points=[0.5], epsabs=1e-14, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-12


@pytest.mark.parametrize("k", KERNELS)
def test_shape_edges_and_monotone(orc, k):
    q = np.linspace(0.0, 1.2, 12001)
    f, fp = orc.kernel_shape(k, q)
    assert f[0] == 1.0
    assert np.all(np.diff(f) <= 1e-15)
    assert np.all(f[q >= 1.0] == 0.0) and np.all(fp[q >= 1.0] == 0.0)
    ql = np.array([1.0 - 1e-6])
    fl, fpl = orc.kernel_shape(k, ql)
    assert abs(fl[0]) < 1e-11 and abs(fpl[0]) < 1e-5


@pytest.mark.parametrize("k", KERNELS)
def test_derivative_matches_finite_difference(orc, k):
    q = np.linspace(0.01, 0.99, 391)
    q = q[np.abs(q - 0.5) > 1e-3]
    e = 1e-6
    fp_, _ = orc.kernel_shape(k, q + e)
    fm_, _ = orc.kernel_shape(k, q - e)
    _, d = orc.kernel_shape(k, q)
    fd = (fp_ - fm_) / (2 * e)
    assert np.max(np.abs(fd - d)) < 2e-8


def test_cubic_spline_pieces_join(orc):
    q = np.array([0.5 - 1e-12, 0.5, 0.5 + 1e-12])
    f, fp = orc.kernel_shape("m4", q)
    assert np.ptp(f) < 1e-10 and np.ptp(fp) < 1e-10


@pytest.mark.parametrize("k", KERNELS)
def test_w_derivatives(orc, k):
    rng = np.random.default_rng(7)
    H = rng.uniform(0.5, 2.0, 200)
    r = H * rng.uniform(0.02, 0.98, 200)
    w, dwdr, dwdh = orc.kernel_w(k, r, H)
    e = 1e-6
    wr1, _, _ = orc.kernel_w(k, r + e, H)
    wr0, _, _ = orc.kernel_w(k, r - e, H)
    wh1, _, _ = orc.kernel_w(k, r, H + e)
    wh0, _, _ = orc.kernel_w(k, r, H - e)
    scale = np.max(np.abs(w)) + 1.0
    assert np.max(np.abs((wr1 - wr0) / (2 * e) - dwdr)) < 1e-7 * scale
    assert np.max(np.abs((wh1 - wh0) / (2 * e) - dwdh)) < 1e-7 * scale
    # W scales as H^-3 at fixed q
    w2, _, _ = orc.kernel_w(k, 2 * r, 2 * H)
    np.testing.assert_allclose(w2 * 8.0, w, rtol=1e-14)
