"""The closed-form pins of pins.py must reject plausible misreadings of the
paper.  Each case compiles a copy of the oracle's C source with one planted
mistake (a textual substitution), loads it in place of the oracle, and checks
that the pin's error exceeds the tolerance the real oracle meets.  Nothing
here touches the oracle's source file or its built library.

Planted mistakes:
  stiffened sound speed c^2 = gamma P / rho           (Sec. 2.3.1)
  viscosity with the mean support H in place of h = H/2 (Sec. 2.3.5)
  viscosity without eps hbar^2 in the denominator of mu
  harmonic instead of arithmetic mean density in Pi
  geometric instead of arithmetic mean sound speed in Pi
  full instead of half viscous heating in du/dt      (eq:AV_heating)
  alpha instead of beta in the signal term           (eq:courant_condition)
"""
import pytest

import pins

MUTANTS = {
    "stiffened_c2_gammaP_over_rho": (
        "c2 = gm * (Pi + p->P0) / rho[i];", "c2 = gm * Pi / rho[i];", "eos"),
    "hbar_from_H_not_h": (
        "double hbar = 0.5 * (hi_s + 0.5 * H[j]);", "double hbar = 0.5 * (H[i] + H[j]);", "visc"),
    "mu_without_eps": (
        "double mu = hbar * vdotx / (r2 + p->eps_av * hbar * hbar);",
        "double mu = hbar * vdotx / r2;", "visc"),
    "harmonic_rhobar": (
        "double rbar = 0.5 * (rho[i] + rho[j]);",
        "double rbar = 2.0 * rho[i] * rho[j] / (rho[i] + rho[j]);", "visc"),
    "geometric_cbar": (
        "double cbar = 0.5 * (c[i] + c[j]);", "double cbar = sqrt(c[i] * c[j]);", "visc"),
    "full_viscous_heating": (
        "const double heat = 0.5 * sav;", "const double heat = sav;", "visc"),
    "signal_term_alpha": (
        "double den = (1.0 + 0.6 * p->alpha) * c[i] + 0.6 * p->beta * mumax;",
        "double den = (1.0 + 0.6 * p->alpha) * c[i] + 0.6 * p->alpha * mumax;", "dt"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_rejects_planted_mistake(orc, tmp_path, name):
    old, new, which = MUTANTS[name]
    src = orc.source_text()
    assert src.count(old) == 1, f"pattern of {name} not unique in the oracle source"
    lib = orc.compile_variant(src.replace(old, new), str(tmp_path / f"mut_{name}.so"))
    saved = orc._lib
    orc._lib = lib
    try:
        if which == "eos":
            err = pins.sound_speed_error(orc, pins.STIFFENED, pins.STIFFENED_STATES)
            assert err > 1e-3, err
        else:
            e_du, e_dt, _ = pins.compression_errors(orc)
            if which == "visc":
                assert e_du > 1e-4, e_du
            else:
                assert e_dt > 1e-4, e_dt
    finally:
        orc._lib = saved
