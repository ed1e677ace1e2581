"""FP64 CPU oracle for the SPH neighbour-interaction sweep.

TEST INFRASTRUCTURE ONLY.  The product library never imports, links or runs
anything in this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` do.  The oracle shares no code with the GPU
path: the heavy loops are plain C in ``sph_oracle.c`` (built with gcc,
``-ffp-contract=off``), and this module only marshals numpy arrays and composes
the kick-drift-kick sequence.

Passages followed (section numbers of the paper):
  * kernels .......................... Sec. 2.3 (cubic spline, Wendland C2/C4/C6)
  * neighbour sets ................... Sec. 2.3.2 (gather / gather+scatter sets)
  * density, grad-h term, h solve .... Sec. 2.3.3 (eq:Density_estimate, constant kernel mass)
  * equation of state ................ Sec. 2.3.1
  * forces, du/dt, viscosity ......... Sec. 2.3.5 (eq:AV_heating)
  * time-step limits ................. Sec. 2.3.6 (eq:courant_condition, acceleration limit)
  * kick-drift-kick with predictor ... Sec. 2.3.6 (predictor, closing/opening kicks, drift)

Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` except the energy-drift level over several steps,
which is "parity unpinned" (the paper quotes only whole-run energy errors).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from ctypes import c_double, c_int, c_int32, c_int64, POINTER

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "libsph_oracle.so")

KERNELS = {"m4": 0, "wc2": 1, "wc4": 2, "wc6": 3}
EOS = {"ideal": 0, "stiffened": 1}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no FMA contraction, OpenMP for timing)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def configure(L):
    """Declare the C signatures on a loaded oracle library and check its layout."""
    dp = POINTER(c_double)
    ip = POINTER(c_int64)
    pp = POINTER(Params)
    L.orc_sigma.restype = c_double
    L.orc_sigma.argtypes = [c_int]
    L.orc_num_threads.restype = c_int
    L.orc_set_threads.argtypes = [c_int]
    L.orc_params_size.restype = c_int
    L.orc_kernel_shape.argtypes = [c_int, c_int64, dp, dp, dp]
    L.orc_kernel_w.argtypes = [c_int, c_int64, dp, dp, dp, dp, dp]
    L.orc_neighbors.argtypes = [pp, c_int64, dp, dp, dp, dp, c_int, ip, ip, ip]
    L.orc_neighbors.restype = c_int
    L.orc_density.argtypes = [pp, c_int64, dp, dp, dp, dp, dp, ip, c_int64, dp, dp, dp, ip]
    L.orc_density.restype = c_int
    L.orc_solve_h.argtypes = [pp, c_int64, dp, dp, dp, dp, dp, ip, c_int64, dp, dp, dp, ip,
                              POINTER(c_int32), POINTER(c_int64)]
    L.orc_solve_h.restype = c_int
    L.orc_eos.argtypes = [pp, c_int64, dp, dp, dp, dp]
    L.orc_forces.argtypes = [pp, c_int64] + [dp] * 12 + [ip, c_int64] + [dp] * 5 + [ip, dp]
    L.orc_forces.restype = c_int
    L.orc_isentrope.argtypes = [pp, c_int64, dp, dp, dp, dp]
    L.orc_imbalance.argtypes = [pp, c_int64, dp, dp, dp, dp, dp, dp, c_double, ip, c_int64, dp]
    L.orc_imbalance.restype = c_int
    L.orc_ic_average.argtypes = [pp, c_int64, dp, dp, dp, dp, dp, dp, dp, ip, c_int64, dp, dp]
    L.orc_ic_average.restype = c_int
    if L.orc_params_size() != ctypes.sizeof(Params):
        raise RuntimeError("oracle parameter layout mismatch")
    return L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = configure(ctypes.CDLL(_LIB))
    return _lib


def source_text() -> str:
    """The oracle's C source (tests compile altered copies of it to show that
    their checks catch a planted mistake)."""
    with open(_SRC) as f:
        return f.read()


def compile_variant(src: str, path: str):
    """Compile C source `src` with the oracle's flags into `path` and load it."""
    cpath = path + ".c"
    with open(cpath, "w") as f:
        f.write(src)
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", cpath, "-o", path, "-lm"]
    subprocess.check_call(cmd)
    return configure(ctypes.CDLL(path))


class Params(ctypes.Structure):
    _fields_ = [
        ("kernel", c_int32), ("periodic", c_int32), ("eos", c_int32), ("nr_maxit", c_int32),
        ("n_ngb", c_double), ("lo", c_double * 3), ("hi", c_double * 3),
        ("gamma", c_double), ("P0", c_double),
        ("alpha", c_double), ("beta", c_double), ("eps_av", c_double),
        ("eta_c", c_double), ("eta_a", c_double), ("dt_max", c_double),
        ("h_max", c_double), ("nr_tol", c_double), ("flags", c_int32), ("pad_", c_int32),
    ]


ENTROPY, EVOLVED = 1, 2


def make_params(p: dict) -> Params:
    """Build the C parameter block from the plain dict used by the input generators."""
    q = Params()
    k = p.get("kernel", "m4")
    q.kernel = KERNELS[k] if isinstance(k, str) else int(k)
    q.periodic = int(bool(p.get("periodic", True)))
    e = p.get("eos", "ideal")
    q.eos = EOS[e] if isinstance(e, str) else int(e)
    q.nr_maxit = int(p.get("oracle_nr_maxit", 200))
    q.n_ngb = float(p["n_ngb"])
    lo = p.get("box_lo", (0.0, 0.0, 0.0))
    hi = p.get("box_hi", (1.0, 1.0, 1.0))
    for a in range(3):
        q.lo[a] = float(lo[a])
        q.hi[a] = float(hi[a])
    q.gamma = float(p.get("gamma", 5.0 / 3.0))
    q.P0 = float(p.get("P0", 0.0))
    q.alpha = float(p.get("alpha", 1.0))
    q.beta = float(p.get("beta", 2.0))
    q.eps_av = float(p.get("eps_av", 0.01))
    q.eta_c = float(p.get("eta_c", 0.3))
    q.eta_a = float(p.get("eta_a", 0.2))
    q.dt_max = float(p.get("dt_max", 1.0))
    q.h_max = float(p.get("h_max", 0.25))
    q.nr_tol = float(p.get("oracle_nr_tol", 1e-14))
    q.flags = (ENTROPY if p.get("entropy") else 0) | (EVOLVED if p.get("evolved") else 0)
    return q


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(POINTER(c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(POINTER(c_int64))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's row loops (its results do not depend on it)."""
    lib().orc_set_threads(int(n))


def sigma(kernel) -> float:
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    return float(lib().orc_sigma(k))


def kernel_shape(kernel, q):
    """f(q) and f'(q) of the normalised shape function (support q < 1)."""
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    q, qp = _d(q)
    f, fp_ = _d(np.zeros_like(q))
    d, dp_ = _d(np.zeros_like(q))
    lib().orc_kernel_shape(k, q.size, qp, fp_, dp_)
    return f, d


def kernel_w(kernel, r, H):
    """W(r, H), dW/dr and dW/dH (H is the support radius)."""
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    r, rp = _d(r)
    H, Hp = _d(np.broadcast_to(H, r.shape))
    outs = [_d(np.zeros_like(r)) for _ in range(3)]
    lib().orc_kernel_w(k, r.size, rp, Hp, *[o[1] for o in outs])
    return tuple(o[0] for o in outs)


def neighbors(params: dict, x, y, z, H, mode: int = 0):
    """CSR neighbour sets (rows ascending, self excluded).

    mode 0: gather set  {j != i : r_ij^2 < H_i^2}
    mode 1: force set   {j != i : r_ij^2 < max(H_i, H_j)^2}
    """
    P = make_params(params)
    n = len(x)
    arrs = [_d(v) for v in (x, y, z, H)]
    counts, cp = _i(np.zeros(n, dtype=np.int64))
    rc = lib().orc_neighbors(ctypes.byref(P), n, *[a[1] for a in arrs], mode, cp, None, None)
    if rc != 0:
        raise RuntimeError("oracle neighbour search failed")
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    offsets, op = _i(offsets)
    idx, ip = _i(np.zeros(max(int(offsets[-1]), 1), dtype=np.int64))
    rc = lib().orc_neighbors(ctypes.byref(P), n, *[a[1] for a in arrs], mode, cp, op, ip)
    if rc != 0:
        raise RuntimeError("oracle neighbour search failed")
    return offsets, idx[: int(offsets[-1])]


def neighbor_counts(params: dict, x, y, z, H, mode: int = 0):
    """|G_i| (mode 0) or |F_i| (mode 1) per particle, without the sets."""
    P = make_params(params)
    n = len(x)
    arrs = [_d(v) for v in (x, y, z, H)]
    counts, cp = _i(np.zeros(n, dtype=np.int64))
    rc = lib().orc_neighbors(ctypes.byref(P), n, *[a[1] for a in arrs], mode, cp, None, None)
    if rc != 0:
        raise RuntimeError("oracle neighbour search failed")
    return counts


def _rows(rows, n):
    if rows is None:
        return None, None, n
    r, rp = _i(rows)
    return r, rp, r.size


def density(params: dict, x, y, z, m, H, rows=None):
    """rho, d rho / dH, Omega and |G_i| at the given support radii (optionally
    only for the particles listed in ``rows``)."""
    P = make_params(params)
    n = len(x)
    ins = [_d(v) for v in (x, y, z, m, H)]
    rr, rp, nw = _rows(rows, n)
    outs = [_d(np.zeros(nw)) for _ in range(3)]
    cnt, cp = _i(np.zeros(nw, dtype=np.int64))
    rc = lib().orc_density(ctypes.byref(P), n, *[a[1] for a in ins], rp, nw,
                           *[o[1] for o in outs], cp)
    if rc != 0:
        raise RuntimeError("oracle density failed")
    return outs[0][0], outs[1][0], outs[2][0], cnt


def solve_h(params: dict, x, y, z, m, H0, rows=None):
    """Support radii solving (4 pi/3) H^3 rho(H) = n_ngb m_i, with rho, Omega there
    (optionally only for the particles listed in ``rows``)."""
    P = make_params(params)
    n = len(x)
    ins = [_d(v) for v in (x, y, z, m, H0)]
    rr, rowp, nw = _rows(rows, n)
    H, Hp = _d(np.zeros(nw))
    rho, rp = _d(np.zeros(nw))
    om, op = _d(np.zeros(nw))
    cnt, cp = _i(np.zeros(nw, dtype=np.int64))
    its = np.zeros(nw, dtype=np.int32)
    bad = c_int64(0)
    rc = lib().orc_solve_h(ctypes.byref(P), n, *[a[1] for a in ins], rowp, nw, Hp, rp, op, cp,
                           its.ctypes.data_as(POINTER(c_int32)), ctypes.byref(bad))
    if rc != 0:
        raise RuntimeError("oracle smoothing-length solve failed")
    return {"H": H, "rho": rho, "omega": om, "count": cnt, "iters": its,
            "n_noconv": int(bad.value)}


def eos(params: dict, rho, u):
    P = make_params(params)
    rho, rp = _d(rho)
    u, up = _d(u)
    Pr, Pp = _d(np.zeros_like(rho))
    c, cp = _d(np.zeros_like(rho))
    lib().orc_eos(ctypes.byref(P), rho.size, rp, up, Pp, cp)
    return Pr, c


def forces(params: dict, x, y, z, vx, vy, vz, m, H, rho, omega, P, c, rows=None):
    """Accelerations, du/dt, per-particle time-step limit and |F_i| (optionally
    only for the particles listed in ``rows``)."""
    Pp = make_params(params)
    n = len(x)
    ins = [_d(v) for v in (x, y, z, vx, vy, vz, m, H, rho, omega, P, c)]
    rr, rowp, nw = _rows(rows, n)
    outs = [_d(np.zeros(nw)) for _ in range(6)]
    cnt, cp = _i(np.zeros(nw, dtype=np.int64))
    rc = lib().orc_forces(ctypes.byref(Pp), n, *[a[1] for a in ins], rowp, nw,
                          *[o[1] for o in outs[:5]], cp, outs[5][1])
    if rc != 0:
        raise RuntimeError("oracle forces failed")
    ax, ay, az, dudt, dti, drho = (o[0] for o in outs)
    return {"ax": ax, "ay": ay, "az": az, "dudt": dudt, "dt": dti, "count": cnt, "drho": drho}


def imbalance(params: dict, x, y, z, m, H, mat=None, alpha=None, rows=None):
    """Kernel imbalance I_i (eq:Kernel_imbalance) at the given H (mat None:
    one material; alpha defaults to params['ic_alpha'], else 10: the paper
    gives no value; 10 puts I near 1.5 at the free surface of a uniform
    body)."""
    P = make_params(params)
    n = len(x)
    if alpha is None:
        alpha = float(params.get("ic_alpha", 10.0))
    ins = [_d(v) for v in (x, y, z, m, H)]
    matp = None
    if mat is not None:
        mat_a = _d(mat)   # (kept alive until the call returns)
        matp = mat_a[1]
    rr, rp, nw = _rows(rows, n)
    out, op = _d(np.zeros(nw))
    rc = lib().orc_imbalance(ctypes.byref(P), n, *[a[1] for a in ins], matp, float(alpha), rp,
                             nw, op)
    if rc != 0:
        raise RuntimeError("oracle imbalance failed")
    return out


def ic_average(params: dict, x, y, z, H, I, T, Pr, rows=None):
    """Interface-correction averages (Tbar, Pbar) with weights exp(-I_j^2) W_ij(h_i)."""
    P = make_params(params)
    n = len(x)
    ins = [_d(v) for v in (x, y, z, H, I, T, Pr)]
    rr, rp, nw = _rows(rows, n)
    tb, tbp = _d(np.zeros(nw))
    pb, pbp = _d(np.zeros(nw))
    rc = lib().orc_ic_average(ctypes.byref(P), n, *[a[1] for a in ins], rp, nw, tbp, pbp)
    if rc != 0:
        raise RuntimeError("oracle interface averages failed")
    return tb, pb


def rho_from_eos(params: dict, T, Pr):
    """rho_EOS(T, P) with the temperature T = u (c_v = 1): ideal gas
    P / ((gamma - 1) T), stiffened gas (P + gamma P0) / ((gamma - 1) T)."""
    g = float(params.get("gamma", 5.0 / 3.0))
    if params.get("eos", "ideal") in ("stiffened", 1):
        return (Pr + g * float(params.get("P0", 0.0))) / ((g - 1.0) * T)
    return Pr / ((g - 1.0) * T)


def interface_correct(params: dict, x, y, z, m, H, mat, rho, u, Pr):
    """Interface correction (Sec. 2.3.4) of the fluid values at the given H:
    I from eq:Kernel_imbalance, (Tbar, Pbar), P~ = e P + (1 - e) Pbar and
    T~ likewise with e = exp(-I^2), rho~ = rho_EOS(T~, P~) (the uncorrected
    rho where that is not a positive number), c~ from the EOS at (rho~, T~).
    T = u."""
    I = imbalance(params, x, y, z, m, H, mat)
    Tbar, Pbar = ic_average(params, x, y, z, H, I, u, Pr)
    e = np.exp(-I * I)
    Pc = e * Pr + (1.0 - e) * Pbar
    Tc = e * u + (1.0 - e) * Tbar
    with np.errstate(divide="ignore", invalid="ignore"):
        rc = rho_from_eos(params, Tc, Pc)
    ok = np.isfinite(rc) & (rc > 0.0)
    rc = np.where(ok, rc, rho)
    _, cc = eos(params, rc, Tc)
    return {"I": I, "Tbar": Tbar, "Pbar": Pbar, "P": Pc, "T": Tc, "rho": rc, "c": cc}


def isentrope(params: dict, rho_old, u_old, rho_new):
    """u(rho_new, s(rho_old, u_old)): the entropy-conserving update (Sec. 2.3.5)."""
    P = make_params(params)
    ro, rop = _d(rho_old)
    uo, uop = _d(u_old)
    rn, rnp = _d(rho_new)
    un, unp = _d(np.zeros_like(ro))
    lib().orc_isentrope(ctypes.byref(P), ro.size, rop, uop, rnp, unp)
    return un


# ---------------------------------------------------------------------------
# Time integration (Sec. 2.3.6), global time step.  State arrays are FP64.
# Start-up (not spelt out in the paper): density and forces at t0.  One step:
#   1. opening kick   v_half = v + (dt/2) a,   u_half = u + (dt/2) du
#   2. drift          x = x + dt v_half, wrapped into the periodic box
#   3. density pass at the new positions (H from the previous step as guess)
#   4. predictor      v_p = v_half + (dt/2) a_old,  u_p likewise
#   5. EOS at (rho, u_p), forces with (v_p, u_p)
#   6. closing kick   v = v_half + (dt/2) a_new,   u likewise
# which is the paper's density / predict / force+closing kick / opening kick
# / drift loop regrouped so that a step ends with synchronised v and u.
# ---------------------------------------------------------------------------

STATE_KEYS = ("x", "y", "z", "vx", "vy", "vz", "m", "u", "H")


def init(params: dict, state: dict) -> dict:
    """Density and forces at the initial time; fills rho, omega, P, c, a, dudt, dt
    (and, for the entropy-conserving update, rho_old; for evolved density, drho)."""
    s = {k: np.array(state[k], dtype=np.float64, copy=True) for k in STATE_KEYS}
    d = solve_h(params, s["x"], s["y"], s["z"], s["m"], s["H"])
    s["H"], s["rho"], s["omega"] = d["H"], d["rho"], d["omega"]
    s["n_noconv"] = d["n_noconv"]
    s["P"], s["c"] = eos(params, s["rho"], s["u"])
    rho_f = s["rho"]
    if params.get("interface"):
        ic = interface_correct(params, s["x"], s["y"], s["z"], s["m"], s["H"], state.get("mat"),
                               s["rho"], s["u"], s["P"])
        rho_f, s["P"], s["c"], s["imb"], s["rho_c"] = ic["rho"], ic["P"], ic["c"], ic["I"], ic["rho"]
    f = forces(params, s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"], s["H"],
               rho_f, s["omega"], s["P"], s["c"])
    for k in ("ax", "ay", "az", "dudt", "dt", "drho"):
        s[k] = f[k]
    if state.get("mat") is not None:
        s["mat"] = np.array(state["mat"], dtype=np.float64, copy=True)
    if params.get("entropy"):
        s["rho_old"] = s["rho"].copy()
    s["n_d"] = int(d["count"].sum())
    s["n_f"] = int(f["count"].sum())
    return s


def global_dt(params: dict, s: dict) -> float:
    return float(min(np.min(s["dt"]) if len(s["dt"]) else np.inf, params.get("dt_max", 1.0)))


def _wrap(params: dict, v, a):
    if not params.get("periodic", True):
        return v
    lo = float(params.get("box_lo", (0.0, 0.0, 0.0))[a])
    hi = float(params.get("box_hi", (1.0, 1.0, 1.0))[a])
    L = hi - lo
    return v - L * np.floor((v - lo) / L)


def step(params: dict, s: dict, dt: float | None = None) -> dict:
    """One kick-drift-kick step in place; returns the FP64 report.

    Interface correction (Sec. 2.3.4): after the EOS at the predicted u, the
    force pass takes the corrected density, pressure and sound speed.

    Entropy-conserving update (Sec. 2.3.5): du/dt holds only the viscous
    heating; after the density pass the half-step u is carried along the
    adiabat from the old to the new density (isentrope), then rho_old moves
    on.  Evolved density (Sec. 2.3.3): rho is a state variable kicked and
    predicted like u with d rho/dt from the force pass; the density pass only
    supplies H and Omega."""
    if dt is None or dt <= 0:
        dt = global_dt(params, s)
    hdt = 0.5 * dt
    evolved = bool(params.get("evolved"))
    vxh = s["vx"] + hdt * s["ax"]
    vyh = s["vy"] + hdt * s["ay"]
    vzh = s["vz"] + hdt * s["az"]
    uh = s["u"] + hdt * s["dudt"]
    if evolved:
        rhoh = s["rho"] + hdt * s["drho"]
    s["x"] = _wrap(params, s["x"] + dt * vxh, 0)
    s["y"] = _wrap(params, s["y"] + dt * vyh, 1)
    s["z"] = _wrap(params, s["z"] + dt * vzh, 2)
    d = solve_h(params, s["x"], s["y"], s["z"], s["m"], s["H"])
    s["H"], s["omega"] = d["H"], d["omega"]
    if evolved:
        rho_f = rhoh + hdt * s["drho"]
    else:
        s["rho"] = d["rho"]
        rho_f = s["rho"]
    if params.get("entropy"):
        uh = isentrope(params, s["rho_old"], uh, s["rho"])
        s["rho_old"] = s["rho"].copy()
    vxp = vxh + hdt * s["ax"]
    vyp = vyh + hdt * s["ay"]
    vzp = vzh + hdt * s["az"]
    up = uh + hdt * s["dudt"]
    s["P"], s["c"] = eos(params, rho_f, up)
    if params.get("interface"):
        ic = interface_correct(params, s["x"], s["y"], s["z"], s["m"], s["H"], s.get("mat"),
                               rho_f, up, s["P"])
        rho_f, s["P"], s["c"], s["imb"], s["rho_c"] = ic["rho"], ic["P"], ic["c"], ic["I"], ic["rho"]
    f = forces(params, s["x"], s["y"], s["z"], vxp, vyp, vzp, s["m"], s["H"],
               rho_f, s["omega"], s["P"], s["c"])
    for k in ("ax", "ay", "az", "dudt", "dt", "drho"):
        s[k] = f[k]
    s["vx"] = vxh + hdt * s["ax"]
    s["vy"] = vyh + hdt * s["ay"]
    s["vz"] = vzh + hdt * s["az"]
    s["u"] = uh + hdt * s["dudt"]
    if evolved:
        s["rho"] = rhoh + hdt * s["drho"]
    s["n_noconv"] = d["n_noconv"]
    s["n_d"] = int(d["count"].sum())
    s["n_f"] = int(f["count"].sum())
    rep = reductions(s)
    rep["dt"] = dt
    return rep


def reductions(s: dict) -> dict:
    """Total momentum, kinetic and internal energy (FP64 sums)."""
    m = s["m"]
    px = float(np.sum(m * s["vx"]))
    py = float(np.sum(m * s["vy"]))
    pz = float(np.sum(m * s["vz"]))
    ek = float(np.sum(0.5 * m * (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2)))
    ei = float(np.sum(m * s["u"]))
    return {"momentum": (px, py, pz), "e_kin": ek, "e_int": ei, "e_tot": ek + ei}


# ---- individual time steps (Sec. 2.3.6) ---------------------------------------
#
# Every particle steps with a power-of-two fraction 2^-r of the base step dt0
# (dt_max); r is its rung, 0 <= r <= rung_max.  Time is counted in units of
# the finest step dt0 2^-rung_max, so a particle on rung r has a step of
# L = 2^(rung_max - r) units and its steps start at multiples of L.  A
# substep runs from the current time T to the next step boundary of any
# particle.  State between substeps: particles at a step boundary (T a
# multiple of their L) hold v, u at T; the others hold their half-step
# values.

def step_units(params: dict, rung):
    R = int(params.get("rung_max", 8))
    return np.left_shift(np.int64(1), (R - np.asarray(rung, dtype=np.int64)))


def desired_rung(params: dict, dt):
    """The smallest r >= 0 whose step dt0 2^-r fits under the particle's limit
    dt (min(dt_a, dt_CFL) >= 2^-r dt0); rung_max when none does."""
    R = int(params.get("rung_max", 8))
    dt0 = float(params.get("dt_max", 1.0))
    dt = np.asarray(dt, dtype=np.float64)
    out = np.full(dt.shape, R, dtype=np.int64)
    for k in range(R, -1, -1):
        out = np.where(dt >= math.ldexp(dt0, -k), k, out)
    return out


def neighbour_max_rung(params: dict, x, y, z, H, rung, rows):
    """max_{j in F_i} r_j for the listed particles (-1 for an empty set)."""
    off, idx = neighbors(params, x, y, z, H, mode=1)
    out = np.full(len(rows), -1, dtype=np.int64)
    for k, i in enumerate(rows):
        nb = idx[off[i]:off[i + 1]]
        if nb.size:
            out[k] = int(np.max(rung[nb]))
    return out


def limit_rungs(r_des, nb_max):
    """Saitoh-Makino: a particle's step is at most four times that of any
    particle it interacts with, r_i >= r_j - 2."""
    return np.maximum(r_des, nb_max - 2)


def align_down(params: dict, r_old, r_new, T):
    """A particle moves to a longer step only at a boundary of that step: the
    lowest rung in [r_new, r_old] whose step divides T (moving up is free)."""
    out = np.array(r_new, dtype=np.int64, copy=True)
    for k in range(out.size):
        if out[k] < r_old[k]:
            r = int(out[k])
            while int(T) % int(step_units(params, r)) != 0:
                r += 1
            out[k] = r
    return out


def predict_coeff(T, L, delta):
    """Predictor weight at time T of a particle whose current step of L units
    ends at or after T: (T - T_mid) delta, T_mid the middle of the step (at a
    step end this is half the step, the predictor of the global scheme)."""
    Tb = np.where(T % L == 0, T - L, T - T % L)
    return ((T - Tb).astype(np.float64) - 0.5 * L.astype(np.float64)) * delta


def _assign_rungs(params: dict, s: dict, rows, old):
    R = int(params.get("rung_max", 8))
    rd = desired_rung(params, s["dt"][rows])
    nb = neighbour_max_rung(params, s["x"], s["y"], s["z"], s["H"], old, rows)
    return np.minimum(limit_rungs(rd, nb), R)


def rung_init(params: dict, state: dict) -> dict:
    """init at T = 0, then every particle's rung: its desired rung, raised by
    the limiter against the desired rungs of its force set (the same single
    pass a rung update takes in a substep, where the neighbours' rungs are
    those before the update)."""
    s = init(params, state)
    n = len(s["x"])
    s["T"] = 0
    rows = np.arange(n)
    s["rung"] = _assign_rungs(params, s, rows, desired_rung(params, s["dt"]))
    return s


def substep(params: dict, s: dict) -> dict:
    """One substep in place (Sec. 2.3.6): opening kick of the particles at a
    step boundary, drift of all particles to the next boundary T', density of
    all particles, prediction of v and u at T', EOS, forces of the particles
    whose step ends at T' (the active ones), their closing kick and new rung.
    Returns the report (dt = the substep's length, the active count)."""
    R = int(params.get("rung_max", 8))
    dt0 = float(params.get("dt_max", 1.0))
    delta = math.ldexp(dt0, -R)
    T = int(s["T"])
    L = step_units(params, s["rung"])
    at_boundary = (T % L) == 0
    h = 0.5 * L.astype(np.float64) * delta
    for v, a in (("vx", "ax"), ("vy", "ay"), ("vz", "az"), ("u", "dudt")):
        s[v] = np.where(at_boundary, s[v] + h * s[a], s[v])
    Tn = int(np.min(T - T % L + L))
    dT = Tn - T
    for k, ax in (("x", 0), ("y", 1), ("z", 2)):
        s[k] = _wrap(params, s[k] + (dT * delta) * s["v" + k], ax)
    d = solve_h(params, s["x"], s["y"], s["z"], s["m"], s["H"])
    s["H"], s["rho"], s["omega"] = d["H"], d["rho"], d["omega"]
    cf = predict_coeff(np.int64(Tn), L, delta)
    vxp = s["vx"] + cf * s["ax"]
    vyp = s["vy"] + cf * s["ay"]
    vzp = s["vz"] + cf * s["az"]
    up = s["u"] + cf * s["dudt"]
    s["P"], s["c"] = eos(params, s["rho"], up)
    active = (Tn % L) == 0
    rows = np.nonzero(active)[0]
    f = forces(params, s["x"], s["y"], s["z"], vxp, vyp, vzp, s["m"], s["H"],
               s["rho"], s["omega"], s["P"], s["c"], rows=rows)
    for k in ("ax", "ay", "az", "dudt", "dt"):
        s[k][rows] = f[k]
    ha = h[rows]
    for v, a in (("vx", "ax"), ("vy", "ay"), ("vz", "az"), ("u", "dudt")):
        s[v][rows] = s[v][rows] + ha * s[a][rows]
    old = s["rung"].copy()
    rn = _assign_rungs(params, s, rows, old)
    s["rung"][rows] = align_down(params, old[rows], rn, Tn)
    s["T"] = Tn
    s["n_d"] = int(d["count"].sum())
    s["n_f"] = int(f["count"].sum())
    return {"dt": dT * delta, "n_active": int(rows.size), "T": Tn}
