"""Seeded synthetic particle sets shared by the oracle and the GPU path.

This module only builds initial conditions (positions, velocities, masses,
internal energies, a first guess of the support radius) and parameter dicts.
It holds none of the method's arithmetic: no kernel, no density, no force.

The workloads stand in for the paper's Mars-body benchmark (ballic planets
with M-ANEOS tables, not available here) at its per-device scale of a few
million particles (Sec. 4.3), and for its periodic hydrodynamic tests
(Sec. 3, numpy-made lattices).  Recipes:

  lattice    points at (i + 1/2) a of an n^3 cubic lattice in a periodic box,
             each component jittered by U(-0.1 a, 0.1 a) and wrapped back.
  velocities Gaussian, sigma 0.1 per component unless stated.
  H guess    the support radius holding n_ngb particles at the mean density
             of the set: H0 = a (3 n_ngb / (4 pi))^(1/3) (the solver refines it).

Parameter dicts use the names of the C interface; ``kernel`` is one of
"m4", "wc2", "wc4", "wc6" and ``eos`` one of "ideal", "stiffened".
"""
from __future__ import annotations

import math

import numpy as np

DEFAULTS = dict(alpha=1.0, beta=2.0, eps_av=0.01, eta_c=0.3, eta_a=0.2, dt_max=1.0,
                gamma=5.0 / 3.0, P0=0.0, eos="ideal", periodic=True,
                box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0), h_max=0.25)


def params(**kw) -> dict:
    p = dict(DEFAULTS)
    p.update(kw)
    return p


def _h_guess(a: float, n_ngb: float) -> float:
    return a * (3.0 * n_ngb / (4.0 * math.pi)) ** (1.0 / 3.0)


def jittered_lattice(rng, n_side: int, lo=(0.0, 0.0, 0.0), L=1.0, jitter=0.1):
    """n_side^3 points of a cubic lattice in [lo, lo+L)^3, jittered and wrapped."""
    a = L / n_side
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * a
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pos = [x.ravel(), y.ravel(), z.ravel()]
    out = []
    for c in range(3):
        v = pos[c] + rng.uniform(-jitter * a, jitter * a, size=pos[c].size)
        v = np.mod(v, L)
        v = np.where(v >= L, 0.0, v)
        out.append(v + lo[c])
    return out[0], out[1], out[2], a


def uniform_box(seed: int, n_side: int, kernel: str, n_ngb: float, rho=1.0, u=1.0,
                vsig=0.1, jitter=0.1, **kw) -> dict:
    """Jittered lattice in the periodic unit cube, equal masses, uniform rho and u."""
    rng = np.random.default_rng(seed)
    x, y, z, a = jittered_lattice(rng, n_side, jitter=jitter)
    n = x.size
    st = dict(x=x, y=y, z=z,
              vx=rng.normal(0.0, vsig, n), vy=rng.normal(0.0, vsig, n),
              vz=rng.normal(0.0, vsig, n),
              m=np.full(n, rho / n), u=np.full(n, float(u)),
              H=np.full(n, _h_guess(a, n_ngb)))
    p = params(kernel=kernel, n_ngb=float(n_ngb), **kw)
    return {"state": st, "params": p, "name": f"uniform{n_side}^3-{kernel}-{int(n_ngb)}"}


def config_small(seed: int = 1, n_side: int = 32) -> dict:
    """32^3 = 32768 particles, periodic unit cube, cubic spline, 64 neighbours."""
    return uniform_box(seed, n_side, "m4", 64)


def config_large(seed: int = 2, n_side: int = 128) -> dict:
    """128^3 = 2097152 particles, same setup, Wendland C4, 200 neighbours."""
    return uniform_box(seed, n_side, "wc4", 200)


def config_two_phase(seed: int = 3, n_side: int = 128) -> dict:
    """Slab 0.25 <= y < 0.75 of density 10 (10x particle mass on the same lattice)
    inside density 1; pressure equilibrium (u = 1 outside, 0.1 inside, gamma 5/3);
    shear v_x = 0.1 sin(2 pi y), no thermal velocity.  Wendland C4, 200 neighbours."""
    rng = np.random.default_rng(seed)
    x, y, z, a = jittered_lattice(rng, n_side)
    n = x.size
    slab = (y >= 0.25) & (y < 0.75)
    m0 = 1.0 / n
    m = np.where(slab, 10.0 * m0, m0)
    u = np.where(slab, 0.1, 1.0)
    st = dict(x=x, y=y, z=z, vx=0.1 * np.sin(2.0 * np.pi * y), vy=np.zeros(n), vz=np.zeros(n),
              m=m, u=u, H=np.full(n, _h_guess(a, 200)))
    p = params(kernel="wc4", n_ngb=200.0)
    return {"state": st, "params": p, "name": f"two-phase{n_side}^3-wc4-200"}


def config_batch(seed: int = 4, nsets: int = 256, nmin: int = 4096, nmax: int = 65536) -> dict:
    """Independent periodic unit boxes, sizes log-uniform in [nmin, nmax] rounded to a
    cube n_b^3; each box has rho ~ U(0.5, 2), u ~ U(0.5, 2), gamma 5/3, v ~ N(0, 0.1^2).
    Cubic spline, 64 neighbours."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(nsets + 1)
    top = np.random.default_rng(children[0])
    sets = []
    for b in range(nsets):
        rng = np.random.default_rng(children[b + 1])
        nb = math.exp(top.uniform(math.log(nmin), math.log(nmax)))
        ns = max(4, int(round(nb ** (1.0 / 3.0))))
        rho = top.uniform(0.5, 2.0)
        u = top.uniform(0.5, 2.0)
        x, y, z, a = jittered_lattice(rng, ns)
        n = x.size
        st = dict(x=x, y=y, z=z, vx=rng.normal(0, 0.1, n), vy=rng.normal(0, 0.1, n),
                  vz=rng.normal(0, 0.1, n), m=np.full(n, rho / n), u=np.full(n, u),
                  H=np.full(n, _h_guess(a, 64)))
        sets.append(st)
    p = params(kernel="m4", n_ngb=64.0, h_max=0.4)
    return {"sets": sets, "params": p, "name": f"batch{nsets}-m4-64"}


def config_spheres(seed: int = 5, n1: int = 12_000_000, n2: int = 4_800_000,
                   r1: float = 1.0, r2: float = 0.5, sep: float = 1.55, vrel: float = 2.0) -> dict:
    """Two uniform spheres (radius 1 and 0.5) of density 1 in vacuum, stiffened gas
    gamma = 2, P0 = 1, u = 2 (P = 0), approaching head-on along x at relative speed
    vrel in the centre-of-mass frame.  Each sphere is the innermost n_k points of a
    jittered cubic lattice of spacing (V_k / n_k)^(1/3).  Wendland C4, 200 neighbours."""
    rng = np.random.default_rng(seed)
    parts = []
    for (nk, rk) in ((n1, r1), (n2, r2)):
        vol = 4.0 / 3.0 * math.pi * rk ** 3
        a = (vol / nk) ** (1.0 / 3.0)
        ns = int(math.ceil(2.0 * rk / a)) + 4
        g = (np.arange(ns, dtype=np.float64) - 0.5 * (ns - 1)) * a
        pts = []
        for zc in g:  # slab by slab to bound memory
            yy, xx = np.meshgrid(g, g, indexing="ij")
            zz = np.full(xx.size, zc)
            pts.append(np.stack([xx.ravel(), yy.ravel(), zz]))
        P = np.concatenate(pts, axis=1)
        P += rng.uniform(-0.1 * a, 0.1 * a, size=P.shape)
        r2_ = np.einsum("ij,ij->j", P, P)
        keep = np.argpartition(r2_, nk - 1)[:nk]
        keep.sort()
        parts.append((P[:, keep], nk, vol, a))
    M1 = parts[0][2]
    M2 = parts[1][2]
    v1 = vrel * M2 / (M1 + M2)
    v2 = -vrel * M1 / (M1 + M2)
    xs, ys, zs, vx, m, H = [], [], [], [], [], []
    offsets = (-sep * M2 / (M1 + M2), sep * M1 / (M1 + M2))
    for k, (P, nk, vol, a) in enumerate(parts):
        xs.append(P[0] + offsets[k]); ys.append(P[1]); zs.append(P[2])
        vx.append(np.full(nk, v1 if k == 0 else v2))
        m.append(np.full(nk, vol / nk))
        H.append(np.full(nk, _h_guess(a, 200)))
    n = n1 + n2
    st = dict(x=np.concatenate(xs), y=np.concatenate(ys), z=np.concatenate(zs),
              vx=np.concatenate(vx), vy=np.zeros(n), vz=np.zeros(n), m=np.concatenate(m),
              u=np.full(n, 2.0), H=np.concatenate(H))
    p = params(kernel="wc4", n_ngb=200.0, periodic=False, eos="stiffened", gamma=2.0, P0=1.0,
               h_max=1.0, box_lo=(-4.0, -4.0, -4.0), box_hi=(4.0, 4.0, 4.0))
    return {"state": st, "params": p, "name": f"spheres{n}-wc4-200"}


def random_cloud(seed: int, n: int, kernel: str = "m4", n_ngb: float = 32, periodic: bool = True,
                 clumped: bool = False, L: float = 1.0, vsig: float = 0.3, **kw) -> dict:
    """Small irregular sets for fuzz-style cases: uniform random positions, optionally
    with half the particles in a dense Gaussian clump; random masses and u."""
    rng = np.random.default_rng(seed)
    if clumped:
        k = n // 2
        pos = np.concatenate([rng.uniform(0, L, (n - k, 3)),
                              np.mod(0.5 * L + 0.06 * L * rng.standard_normal((k, 3)), L)])
    else:
        pos = rng.uniform(0, L, (n, 3))
    if not periodic:
        pos = pos - 0.5 * L
    m = rng.uniform(0.5, 1.5, n) / n
    st = dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(),
              vx=rng.normal(0, vsig, n), vy=rng.normal(0, vsig, n), vz=rng.normal(0, vsig, n),
              m=m, u=rng.uniform(0.5, 1.5, n),
              H=np.full(n, _h_guess(L / n ** (1.0 / 3.0), n_ngb)))
    lo = (0.0, 0.0, 0.0) if periodic else (-L, -L, -L)
    hi = (L, L, L) if periodic else (L, L, L)
    p = params(kernel=kernel, n_ngb=float(n_ngb), periodic=periodic, box_lo=lo, box_hi=hi,
               h_max=0.45 * L if periodic else 2.0 * L, **kw)
    return {"state": st, "params": p, "name": f"cloud{n}-{kernel}-{int(n_ngb)}"}


def perfect_lattice(n_side: int, kernel: str, n_ngb: float, u=1.0, H=None) -> dict:
    """Unjittered lattice at rest (closed-form cases)."""
    a = 1.0 / n_side
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * a
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    n = n_side ** 3
    st = dict(x=x.ravel().copy(), y=y.ravel().copy(), z=z.ravel().copy(),
              vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n), m=np.full(n, 1.0 / n),
              u=np.full(n, float(u)), H=np.full(n, H if H is not None else _h_guess(a, n_ngb)))
    p = params(kernel=kernel, n_ngb=float(n_ngb))
    return {"state": st, "params": p, "name": f"lattice{n_side}^3-{kernel}"}
