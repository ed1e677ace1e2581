"""Pins of the oracle's equation of state, artificial viscosity and Courant
limit against closed forms (see pins.py for the derivations).

* Sound speed (Sec. 2.3.1): c^2 equals (dP/drho) along an adiabat for the
  ideal and the stiffened gas, including states under tension (P < 0), and is
  clamped to zero where that derivative is negative.
* Viscosity magnitude (Sec. 2.3.5, eq:AV_heating): du/dt of interior
  particles of an open lattice in uniform compression, whose two sublattices
  differ in rho, Omega, P and c, equals the sum over lattice vectors of the
  PdV term and half the viscous heating with mu = hbar v.x / (r^2 + eps hbar^2),
  hbar the mean of h = H/2, and arithmetic means of c and rho.
* Signal-velocity term of eq:courant_condition: the per-particle step equals
  eta_C h / ((1 + 0.6 alpha) c + 0.6 beta max |mu|) with mu over the same shells.
"""
import pytest

import pins


def test_stiffened_gas_sound_speed_is_adiabatic_derivative(orc):
    assert pins.sound_speed_error(orc, pins.STIFFENED, pins.STIFFENED_STATES) < 1e-9


def test_ideal_gas_sound_speed_is_adiabatic_derivative(orc):
    assert pins.sound_speed_error(orc, pins.IDEAL, pins.IDEAL_STATES) < 1e-9


@pytest.mark.parametrize("kernel,n_side,H_over_a", [("wc4", 12, 3.1), ("m4", 10, 2.3)])
def test_viscosity_and_signal_speed_on_compressed_lattice(orc, kernel, n_side, H_over_a):
    e_du, e_dt, e_a = pins.compression_errors(orc, kernel, n_side, H_over_a)
    assert e_du < 1e-12, e_du
    assert e_dt < 1e-13, e_dt
    assert e_a < 1e-12, e_a
