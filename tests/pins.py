"""Closed-form checks of the oracle's equation of state, viscosity and Courant
limit, shared by test_oracle_eos_viscosity.py (the oracle as built) and
test_oracle_mutants.py (copies of the oracle with a planted mistake, which the
same checks must reject).

Each check returns the largest relative error it finds.

* Sound speed (Sec. 2.3.1): c^2 is the derivative of P along an adiabat,
  (dP/drho)_s with du = (P / rho^2) drho.  Both equations of state are linear
  in the product rho u, so a central difference along the tangent of the
  adiabat is exact up to rounding.  Where that derivative is negative (a
  stiffened gas under strong tension) the sound speed is clamped to zero.

* Viscosity and signal speed (Sec. 2.3.5, eq:AV_heating; Sec. 2.3.6,
  eq:courant_condition): an open cubic lattice of spacing a in uniform
  compression, v = -k (x - x0), so v_ij . x_ij = -k r^2 < 0 for every pair.
  The two interpenetrating sublattices (parity of ix + iy + iz) carry
  different rho, Omega, P and c, so the means over a pair are tested.  For an
  interior particle every neighbour sits at x_i + a n for an integer vector n
  with 0 < a |n| < H, and du_i/dt and the Courant limit are sums over those
  vectors, enumerated here directly from the lattice (no neighbour search):
      mu_n  = hbar (-k r^2) / (r^2 + eps hbar^2),   hbar = (h_i + h_j)/2, h = H/2
      Pi_n  = (-alpha cbar mu_n + beta mu_n^2) / rhobar  (arithmetic means)
      du/dt = A_i sum m G(r) (-k r^2) + 1/2 sum m Pi_n G(r) (-k r^2)
      dt    = eta_C h_i / ((1 + 0.6 alpha) c_i + 0.6 beta max_n |mu_n|)
  with G(r) = (dW/dr)/r and A = P / (Omega rho^2).  The acceleration of an
  interior particle vanishes by the lattice's inversion symmetry.
"""
from __future__ import annotations

import numpy as np


def sound_speed_error(orc, params: dict, states) -> float:
    """Largest |c^2 - (dP/drho)_s| / scale over the (rho, u) states; a state
    whose adiabatic derivative is negative must give c = 0 exactly."""
    worst = 0.0
    for rho, u in states:
        P0, c0 = orc.eos(params, np.array([rho]), np.array([u]))
        P0, c0 = float(P0[0]), float(c0[0])
        d = 1e-4 * rho
        du = P0 / rho ** 2 * d
        Pp, _ = orc.eos(params, np.array([rho + d]), np.array([u + du]))
        Pm, _ = orc.eos(params, np.array([rho - d]), np.array([u - du]))
        dPdrho = (float(Pp[0]) - float(Pm[0])) / (2.0 * d)
        scale = abs(dPdrho) + abs(P0) / rho + 1e-300
        if dPdrho < 0.0:
            worst = max(worst, 0.0 if c0 == 0.0 else 1.0)
        else:
            worst = max(worst, abs(c0 * c0 - dPdrho) / scale)
    return worst


def compression_lattice(kernel: str, n_side: int, H_over_a: float, k: float = 5.0):
    """Inputs of the compression check: positions, velocities and per-particle
    rho, Omega, P, c on the two sublattices."""
    a = 1.0 / n_side
    g = (np.arange(n_side) + 0.5) * a
    iz, iy, ix = np.meshgrid(np.arange(n_side), np.arange(n_side), np.arange(n_side),
                             indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    x, y, z = g[ix], g[iy], g[iz]
    sub = (ix + iy + iz) % 2
    x0 = 0.5 + 0.1 * a
    n = x.size
    st = {
        "x": x, "y": y, "z": z,
        "vx": -k * (x - x0), "vy": -k * (y - x0), "vz": -k * (z - x0),
        "m": np.full(n, 1e-3), "H": np.full(n, H_over_a * a),
        "rho": np.where(sub == 0, 1.0, 1.7), "omega": np.where(sub == 0, 0.95, 1.05),
        "P": np.where(sub == 0, 0.9, 1.4), "c": np.where(sub == 0, 1.2, 0.8),
    }
    reach = int(np.ceil(H_over_a)) + 1
    interior = ((ix >= reach) & (ix < n_side - reach) & (iy >= reach) & (iy < n_side - reach) &
                (iz >= reach) & (iz < n_side - reach))
    return st, sub, np.nonzero(interior)[0], a


def lattice_expectation(orc, kernel, params, st, sub, i, a, k):
    """du_i/dt and the Courant limit of interior particle i by enumeration of
    the lattice vectors inside its kernel support."""
    H = float(st["H"][i])
    R = int(np.ceil(H / a))
    v = np.arange(-R, R + 1)
    n1, n2, n3 = (w.ravel() for w in np.meshgrid(v, v, v, indexing="ij"))
    r = a * np.sqrt((n1 * n1 + n2 * n2 + n3 * n3).astype(np.float64))
    keep = (r > 0) & (r < H)
    n1, n2, n3, r = n1[keep], n2[keep], n3[keep], r[keep]
    sj = (sub[i] + n1 + n2 + n3) % 2
    pick = lambda key: np.where(sj == 0, st[key][sub == 0][0], st[key][sub == 1][0])
    rho_j, c_j = pick("rho"), pick("c")
    m = st["m"][0]
    _, dWdr, _ = orc.kernel_w(kernel, r, H)
    G = dWdr / r
    A_i = st["P"][i] / (st["omega"][i] * st["rho"][i] ** 2)
    vx = -k * r * r
    hbar = 0.5 * (0.5 * H + 0.5 * H)
    mu = hbar * vx / (r * r + params["eps_av"] * hbar * hbar)
    cbar = 0.5 * (st["c"][i] + c_j)
    rbar = 0.5 * (st["rho"][i] + rho_j)
    Pi = (-params["alpha"] * cbar * mu + params["beta"] * mu * mu) / rbar
    du_terms = np.concatenate([A_i * m * G * vx, 0.5 * m * Pi * G * vx])
    du = float(np.sum(du_terms))
    du_scale = float(np.sum(np.abs(du_terms)))
    den = (1.0 + 0.6 * params["alpha"]) * st["c"][i] + 0.6 * params["beta"] * np.max(np.abs(mu))
    dt = min(params["eta_c"] * 0.5 * H / den, params["dt_max"])
    a_scale = float(np.sum(np.abs(m * (A_i + A_i + Pi) * G * r)))
    return du, du_scale, dt, a_scale


def compression_errors(orc, kernel: str = "wc4", n_side: int = 12, H_over_a: float = 3.1,
                       k: float = 5.0):
    """(du/dt error, dt error, |a| error), each relative, over the interior."""
    params = dict(kernel=kernel, n_ngb=100.0, periodic=False, alpha=1.0, beta=2.0,
                  eps_av=0.01, eta_c=0.3, eta_a=0.2, dt_max=1.0, gamma=5.0 / 3.0, P0=0.0)
    st, sub, interior, a = compression_lattice(kernel, n_side, H_over_a, k)
    f = orc.forces(params, st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["m"],
                   st["H"], st["rho"], st["omega"], st["P"], st["c"], rows=interior)
    e_du = e_dt = e_a = 0.0
    for t, i in enumerate(interior):
        du, du_s, dt, a_s = lattice_expectation(orc, kernel, params, st, sub, i, a, k)
        e_du = max(e_du, abs(f["dudt"][t] - du) / du_s)
        e_dt = max(e_dt, abs(f["dt"][t] / dt - 1.0))
        amag = np.sqrt(f["ax"][t] ** 2 + f["ay"][t] ** 2 + f["az"][t] ** 2)
        e_a = max(e_a, amag / a_s)
    return e_du, e_dt, e_a


STIFFENED = dict(kernel="m4", n_ngb=64.0, eos="stiffened", gamma=2.0, P0=1.0)
STIFFENED_STATES = [(1.0, 2.0), (1.0, 1.5), (1.3, 3.0), (0.7, 1.2), (2.0, 0.9), (1.0, 0.5)]
IDEAL = dict(kernel="m4", n_ngb=64.0, eos="ideal", gamma=5.0 / 3.0, P0=0.0)
IDEAL_STATES = [(1.0, 1.0), (0.3, 2.5), (10.0, 0.1)]
