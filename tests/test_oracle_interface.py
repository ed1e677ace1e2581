"""Pins of the oracle's interface correction (Sec. 2.3.4, eq:Kernel_imbalance).

  * a perfect periodic lattice of one material has no imbalance (I = 0 to
    round-off) and its corrected fluid values equal the uncorrected ones;
  * on a perfect lattice split into two materials by planes, the imbalance of
    every layer equals the lattice sum 2 |sum_{n on the other side} n_x a
    f(|n| a/H)| / (h sum_n f(|n| a/H)) (the sum over all lattice vectors
    vanishes by symmetry, so the kappa = -1 part counts twice), enumerated
    here over lattice vectors, not particles;
  * at a free surface (an open lattice block) the imbalance of a face
    particle is the one-sided lattice sum over the vectors that stay inside;
  * the averages reproduce a constant field and, away from any interface, a
    linear one; the imbalance does not change under translation, rotation,
    swapping the material labels or scaling the masses;
  * at the free surface of a uniform body in vacuum, where the summed
    density falls to 30-80 % of the true one, the corrected density is
    within 15 % of it (normalisation alpha = 10, the default).
Each pin also rejects a planted mistake (a compiled copy of the oracle).
"""
import itertools

import numpy as np
import pytest

import sph_inputs as si


def lattice_vectors(R):
    k = int(np.ceil(R)) + 1
    r = np.arange(-k, k + 1)
    n = np.array(list(itertools.product(r, r, r)), dtype=np.float64)
    return n[np.einsum("ij,ij->i", n, n) < R * R]


def layer_imbalance(orc, kernel, H_over_a, layer, alpha=1.0):
    """Closed-form I of a particle `layer` lattice planes (0 = the last plane)
    before a material interface normal to x, lattice spacing 1."""
    n = lattice_vectors(H_over_a)
    q = np.sqrt(np.einsum("ij,ij->i", n, n)) / H_over_a
    f, _ = orc.kernel_shape(kernel, q)
    other = n[:, 0] >= layer + 1
    num = 2.0 * abs(np.sum(n[other, 0] * f[other]))
    return alpha * num / (0.5 * H_over_a * np.sum(f))


def slab_lattice(n_side=24, kernel="wc4", H_over_a=3.1):
    c = si.perfect_lattice(n_side, kernel, 100.0)
    s, p = c["state"], dict(c["params"], ic_alpha=1.0)
    a = 1.0 / n_side
    s["H"] = np.full(len(s["x"]), H_over_a * a)
    mat = np.where((s["x"] >= 0.25) & (s["x"] < 0.75), 1.0, 0.0)
    return s, p, mat, a


def test_one_material_lattice_has_no_imbalance(orc):
    s, p, _, a = slab_lattice()
    I = orc.imbalance(p, s["x"], s["y"], s["z"], s["m"], s["H"], None)
    assert np.max(np.abs(I)) < 1e-12
    rho, _, _, _ = orc.density(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    P, _ = orc.eos(p, rho, s["u"])
    ic = orc.interface_correct(p, s["x"], s["y"], s["z"], s["m"], s["H"], None, rho, s["u"], P)
    assert np.max(np.abs(ic["rho"] - rho) / rho) < 1e-12
    assert np.max(np.abs(ic["P"] - P) / P) < 1e-12


def imbalance_layer_error(orc, kernel="wc4", H_over_a=3.1):
    s, p, mat, a = slab_lattice(kernel=kernel, H_over_a=H_over_a)
    p = dict(p, kernel=kernel)
    I = orc.imbalance(p, s["x"], s["y"], s["z"], s["m"], s["H"], mat)
    # planes just below x = 0.25 (material 0) and just above (material 1)
    xs = (np.arange(24) + 0.5) * a
    err = 0.0
    for layer in range(4):
        for xv in (xs[5 - layer], xs[6 + layer]):
            sel = np.abs(s["x"] - xv) < 1e-12
            ref = layer_imbalance(orc, kernel, H_over_a, layer)
            err = max(err, np.max(np.abs(I[sel] - ref)) / max(ref, 1e-3))
    return err


@pytest.mark.parametrize("kernel", ["m4", "wc4"])
def test_two_material_lattice_layers(orc, kernel):
    assert imbalance_layer_error(orc, kernel, 3.1 if kernel == "wc4" else 2.2) < 1e-11


def surface_error(orc, kernel="wc2", H_over_a=2.6):
    n_side = 14
    c = si.perfect_lattice(n_side, kernel, 60.0)
    s, p = c["state"], dict(c["params"], periodic=False, ic_alpha=1.0)
    a = 1.0 / n_side
    s["H"] = np.full(len(s["x"]), H_over_a * a)
    I = orc.imbalance(p, s["x"], s["y"], s["z"], s["m"], s["H"], None)
    n = lattice_vectors(H_over_a)
    q = np.sqrt(np.einsum("ij,ij->i", n, n)) / H_over_a
    f, _ = orc.kernel_shape(kernel, q)
    err = 0.0
    for d in range(3):   # depth below the face x = 0 (planes 0, 1, 2)
        inside = n[:, 0] >= -d   # vectors that stay in the block
        num = abs(np.sum(n[inside, 0] * f[inside]))
        ref = num / (0.5 * H_over_a * np.sum(f[inside]))
        x0 = (d + 0.5) * a
        sel = (np.abs(s["x"] - x0) < 1e-12)
        sel &= (s["y"] > 4 * a) & (s["y"] < 1 - 4 * a) & (s["z"] > 4 * a) & (s["z"] < 1 - 4 * a)
        err = max(err, np.max(np.abs(I[sel] - ref)) / max(ref, 1e-3))
    return err


def test_free_surface_imbalance(orc):
    assert surface_error(orc) < 1e-11


def test_averages_of_constant_and_linear_fields(orc):
    n_side = 16
    c = si.perfect_lattice(n_side, "wc4", 100.0)
    s, p = c["state"], dict(c["params"], periodic=False)
    a = 1.0 / n_side
    s["H"] = np.full(len(s["x"]), 3.1 * a)
    I = orc.imbalance(p, s["x"], s["y"], s["z"], s["m"], s["H"], None)
    T = np.full(len(s["x"]), 2.5)
    Tb, Pb = orc.ic_average(p, s["x"], s["y"], s["z"], s["H"], I, T, 3.0 * T)
    assert np.max(np.abs(Tb - 2.5)) < 1e-14 and np.max(np.abs(Pb - 7.5)) < 1e-13
    lin = 1.0 + 0.7 * s["x"] - 0.3 * s["y"] + 0.2 * s["z"]
    Tb, _ = orc.ic_average(p, s["x"], s["y"], s["z"], s["H"], I, lin, lin)
    deep = np.ones(len(lin), bool)
    for key in ("x", "y", "z"):
        deep &= (s[key] > 7 * a) & (s[key] < 1 - 7 * a)   # neighbours of neighbours interior
    assert deep.sum() > 0
    assert np.max(np.abs(Tb[deep] - lin[deep])) < 1e-13


def test_imbalance_invariances(orc):
    c = si.random_cloud(91, 1500, kernel="wc4", n_ngb=80, periodic=False, clumped=True)
    s, p = c["state"], c["params"]
    rng = np.random.default_rng(3)
    mat = rng.integers(0, 3, len(s["x"])).astype(np.float64)
    I0 = orc.imbalance(p, s["x"], s["y"], s["z"], s["m"], s["H"], mat)
    assert np.max(I0) > 0.1
    # rotation about the cloud centre and a translation
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    X = R @ (np.stack([s["x"], s["y"], s["z"]]) - 0.5) + np.array([[0.3], [-0.2], [0.1]])
    I1 = orc.imbalance(p, X[0], X[1], X[2], s["m"], s["H"], mat)
    assert np.max(np.abs(I1 - I0)) < 1e-10
    # relabelled materials, scaled masses
    I2 = orc.imbalance(p, s["x"], s["y"], s["z"], 7.0 * s["m"], s["H"], (mat + 1) % 3 + 5)
    assert np.max(np.abs(I2 - I0)) < 1e-12


def surface_correction(orc, alpha=10.0):
    """A jittered lattice block in vacuum (uniform density 1, one material):
    the summed density falls short at the surface; the corrected one, with the
    default normalisation, is close to 1."""
    n_side = 16
    c = si.perfect_lattice(n_side, "wc4", 100.0)
    s, p = c["state"], dict(c["params"], periodic=False, h_max=1.0, ic_alpha=alpha)
    rng = np.random.default_rng(1)
    a = 1.0 / n_side
    for k in ("x", "y", "z"):
        s[k] = s[k] + rng.uniform(-0.1 * a, 0.1 * a, len(s[k]))
    d = orc.solve_h(p, s["x"], s["y"], s["z"], s["m"], s["H"])
    P, _ = orc.eos(p, d["rho"], s["u"])
    ic = orc.interface_correct(p, s["x"], s["y"], s["z"], s["m"], d["H"], None, d["rho"], s["u"], P)
    surf = np.zeros(len(s["x"]), bool)
    for k in ("x", "y", "z"):
        surf |= (s[k] < 1.5 * a) | (s[k] > 1 - 1.5 * a)
    return np.max(np.abs(d["rho"][surf] - 1.0)), np.max(np.abs(ic["rho"][surf] - 1.0))


def test_correction_restores_density_at_a_free_surface(orc):
    e_sum, e_ic = surface_correction(orc)
    print(f"density error at the surface: summed {e_sum:.3f}, corrected {e_ic:.3f}")
    assert e_sum > 0.5 and e_ic < 0.15


# ---- planted mistakes ---------------------------------------------------------

MUTANTS = {
    "kappa_ignored": (
        "double kappa = (mat && mat[j] != mat[i]) ? -1.0 : 1.0;", "double kappa = 1.0;",
        lambda orc: imbalance_layer_error(orc)),
    "support_for_smoothing_length": (
        "I[k] = alpha * sqrt(nx * nx + ny * ny + nz * nz) / (0.5 * H[i] * den);",
        "I[k] = alpha * sqrt(nx * nx + ny * ny + nz * nz) / (H[i] * den);",
        lambda orc: surface_error(orc)),
    "weights_without_self": (
        "double sw = w, st = w * T[i], sp = w * P[i];", "double sw = 0, st = 0, sp = 0;",
        lambda orc: _linear_average_error(orc)),
}


def _linear_average_error(orc):
    c = si.random_cloud(92, 1200, kernel="wc4", n_ngb=80, periodic=False, clumped=False)
    s, p = c["state"], c["params"]
    I = np.zeros(len(s["x"]))
    T = 1.0 + 30.0 * s["x"]
    Tb, _ = orc.ic_average(p, s["x"], s["y"], s["z"], s["H"], I, T, T)
    # the reference: the W-weighted mean of T over G_i and i, from the oracle's
    # own density sum of the field (rho[m T] / rho[m]) at the same H
    rho_T, _, _, _ = orc.density(p, s["x"], s["y"], s["z"], T, s["H"])
    rho_1, _, _, _ = orc.density(p, s["x"], s["y"], s["z"], np.ones_like(T), s["H"])
    return np.max(np.abs(Tb - rho_T / rho_1))


def test_average_equals_ratio_of_density_sums(orc):
    """With I = 0 the average is the W-weighted mean, i.e. the ratio of two
    density sums (masses T_j and 1)."""
    assert _linear_average_error(orc) < 1e-13


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_interface_pins_reject_planted_mistakes(orc, tmp_path, name):
    old, new, measure = MUTANTS[name]
    src = orc.source_text()
    assert src.count(old) == 1, name
    lib = orc.compile_variant(src.replace(old, new), str(tmp_path / f"mut_{name}.so"))
    saved = orc._lib
    orc._lib = lib
    try:
        assert measure(orc) > 1e-3, name
    finally:
        orc._lib = saved
