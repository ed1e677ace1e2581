"""Python binding of the MI355X SPH neighbour-interaction sweep (libsph_mi355x.so).

Argument marshalling only: every step of the sweep runs in the HIP kernels of
the C library (include/sph.h).  PyTorch provides device memory and streams.
The module raises ImportError when the library has not been built; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph_mi355x.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2511_11425_amd.build` "
        "(or __graft_entry__.build()); the SPH sweep has no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

(SPH_OK, SPH_ERR_INVALID, SPH_ERR_OOM, SPH_ERR_HIP, SPH_ERR_CAPACITY, SPH_ERR_NOCONV, SPH_ERR_STATE,
 SPH_ERR_NONFINITE) = range(8)
KERNELS = {"m4": 0, "wc2": 1, "wc4": 2, "wc6": 3}
PRECISIONS = {"fp64": 0, "mixed": 1}
EOS = {"ideal": 0, "stiffened": 1}
MODE_GATHER, MODE_FORCE = 0, 1

# Exported symbols declared in include/sph.h.
SYMBOLS = ("sph_default_params", "sph_version", "sph_last_error", "sph_create",
           "sph_create_batch", "sph_destroy", "sph_build_tree", "sph_neighbors", "sph_density",
           "sph_forces", "sph_init", "sph_step", "sph_graph_capture_step", "sph_graph_launch",
           "sph_autotune", "sph_get_stats", "sph_set_timing", "sph_init_noalloc")


class Params(ctypes.Structure):
    _fields_ = [
        ("kernel", c_int32), ("precision", c_int32), ("eos", c_int32), ("periodic", c_int32),
        ("n_ngb", c_double), ("box_lo", c_double * 3), ("box_hi", c_double * 3),
        ("gamma", c_double), ("P0", c_double),
        ("alpha", c_double), ("beta", c_double), ("eps_av", c_double),
        ("eta_c", c_double), ("eta_a", c_double), ("dt_max", c_double),
        ("h_max", c_double), ("oversel", c_double), ("nr_tol", c_double),
        ("nr_maxit", c_int32), ("bucket", c_int32), ("stack_limit", c_int32),
        ("flags", c_int32), ("ic_alpha", c_double),
        ("rung_max", c_int32), ("launch", c_int32), ("fastgas", c_double),
    ]


FLAG_ENTROPY, FLAG_EVOLVED, FLAG_INTERFACE, FLAG_DYNAMIC, FLAG_RUNGS = 1, 2, 4, 8, 16
LAUNCH_GROUPS, LAUNCH_PERSISTENT, LAUNCH_WALK = 0, 1, 2
LAUNCH_NAMES = {"groups": LAUNCH_GROUPS, "persistent": LAUNCH_PERSISTENT, "walk": LAUNCH_WALK}


FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m", "u", "H",
          "rho", "omega", "P", "c", "ax", "ay", "az", "dudt", "dt", "drhodt", "mat", "imb",
          "rhoc", "rung")


class Particles(ctypes.Structure):
    _fields_ = [(f, c_void_p) for f in FIELDS]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n", c_int64), ("pairs_density", c_int64), ("pairs_force", c_int64),
        ("cand_density", c_int64), ("cand_force", c_int64), ("nr_iter_max", c_int64),
        ("nr_scans", c_int64), ("n_noconv", c_int64), ("n_rewalk", c_int64),
        ("n_overflow", c_int64), ("momentum", c_double * 3), ("e_kin", c_double),
        ("e_int", c_double), ("dt_next", c_double), ("dt_used", c_double),
        ("pairs_density_total", c_int64), ("pairs_force_total", c_int64),
        ("t_tree_ms", c_double), ("t_density_ms", c_double), ("t_forces_ms", c_double),
        ("t_total_ms", c_double), ("n_iter_limit", c_int64), ("n_nonfinite", c_int64),
        ("n_retest", c_int64), ("status", c_int32), ("reserved_", c_int32),
        ("slots_density", c_int64), ("slots_force", c_int64), ("groups_by_level", c_int64 * 4),
        ("t_units", c_int64), ("n_active", c_int64), ("n_dens", c_int64),
        ("n_fastgas_miss", c_int64), ("launch", c_int64), ("workgroups_force", c_int64),
        ("t_force_walk_ms", c_double), ("t_density_walk_ms", c_double),
        ("groups_walked", c_int64),
    ]


_ctx_p = c_void_p
_lib.sph_default_params.argtypes = [POINTER(Params)]
_lib.sph_version.restype = c_char_p
_lib.sph_last_error.restype = c_char_p
_lib.sph_last_error.argtypes = [_ctx_p]
_lib.sph_create.argtypes = [POINTER(Params), POINTER(_ctx_p)]
_lib.sph_create_batch.argtypes = [POINTER(Params), c_int32, POINTER(c_int64), POINTER(c_double),
                                  POINTER(_ctx_p)]
_lib.sph_destroy.argtypes = [_ctx_p]
_lib.sph_destroy.restype = None
_lib.sph_build_tree.argtypes = [_ctx_p, POINTER(Particles), c_int64, c_void_p]
_lib.sph_neighbors.argtypes = [_ctx_p, POINTER(Particles), c_int32, c_void_p, c_void_p, c_int64,
                               POINTER(c_int64), c_void_p]
_lib.sph_density.argtypes = [_ctx_p, POINTER(Particles), c_void_p]
_lib.sph_forces.argtypes = [_ctx_p, POINTER(Particles), c_void_p]
_lib.sph_init.argtypes = [_ctx_p, POINTER(Particles), c_int64, c_void_p]
_lib.sph_step.argtypes = [_ctx_p, POINTER(Particles), c_double, c_void_p]
_lib.sph_graph_capture_step.argtypes = [_ctx_p, POINTER(Particles), c_double, c_void_p]
_lib.sph_graph_launch.argtypes = [_ctx_p, c_void_p]
_lib.sph_autotune.argtypes = [_ctx_p, POINTER(Particles), POINTER(c_int32), c_void_p]
_lib.sph_get_stats.argtypes = [_ctx_p, POINTER(Stats)]
_lib.sph_set_timing.argtypes = [_ctx_p, c_int32]
_lib.sph_init_noalloc.argtypes = [POINTER(Params), POINTER(Particles), c_int64, c_void_p]
for _f in ("sph_create", "sph_create_batch", "sph_build_tree", "sph_neighbors", "sph_density",
           "sph_forces", "sph_init", "sph_step", "sph_graph_capture_step", "sph_graph_launch",
           "sph_autotune", "sph_get_stats", "sph_set_timing", "sph_init_noalloc"):
    getattr(_lib, _f).restype = ctypes.c_int


class SphError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def version() -> str:
    return _lib.sph_version().decode()


def init_noalloc(params: dict, P: "ParticleArrays", stream=None) -> None:
    """sph_init_noalloc: the start-up pass without a context or any allocation
    (n <= 65536; work arrays in the library's static device array)."""
    q = make_params(params)
    st = _lib.sph_init_noalloc(ctypes.byref(q), ctypes.byref(P.c), P.n, _stream_ptr(stream))
    if st != SPH_OK:
        raise SphError(st, "sph_init_noalloc failed")


def make_params(p: dict) -> Params:
    """C parameter block from the dict used by the input generators."""
    q = Params()
    _lib.sph_default_params(ctypes.byref(q))
    k = p.get("kernel", "m4")
    q.kernel = KERNELS[k] if isinstance(k, str) else int(k)
    pr = p.get("precision", "fp64")
    q.precision = PRECISIONS[pr] if isinstance(pr, str) else int(pr)
    e = p.get("eos", "ideal")
    q.eos = EOS[e] if isinstance(e, str) else int(e)
    q.periodic = int(bool(p.get("periodic", True)))
    q.n_ngb = float(p["n_ngb"])
    lo = p.get("box_lo", (0.0, 0.0, 0.0))
    hi = p.get("box_hi", (1.0, 1.0, 1.0))
    for a in range(3):
        q.box_lo[a] = float(lo[a])
        q.box_hi[a] = float(hi[a])
    for name in ("gamma", "P0", "alpha", "beta", "eps_av", "eta_c", "eta_a", "dt_max", "h_max",
                 "oversel", "nr_tol", "ic_alpha", "fastgas"):
        if name in p:
            setattr(q, name, float(p[name]))
    for name in ("nr_maxit", "bucket", "stack_limit", "rung_max"):
        if name in p:
            setattr(q, name, int(p[name]))
    if "launch" in p:
        v = p["launch"]
        q.launch = LAUNCH_NAMES[v] if isinstance(v, str) else int(v)
    q.flags = ((FLAG_ENTROPY if p.get("entropy") else 0) | (FLAG_EVOLVED if p.get("evolved") else 0)
               | (FLAG_INTERFACE if p.get("interface") else 0)
               | (FLAG_DYNAMIC if p.get("dynamic") else 0)
               | (FLAG_RUNGS if p.get("rungs") else 0))
    return q


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


class ParticleArrays:
    """The caller-owned FP64 device columns of include/sph.h (torch tensors)."""

    def __init__(self, tensors: dict):
        self.t = tensors
        self.n = int(tensors["x"].numel())
        for f in FIELDS:
            v = tensors[f]
            if v.dtype != __import__("torch").float64 or not v.is_cuda or not v.is_contiguous():
                raise ValueError(f"column {f} must be a contiguous float64 CUDA tensor")
            if v.numel() != self.n:
                raise ValueError(f"column {f} has {v.numel()} elements, expected {self.n}")
        self.c = Particles(*[c_void_p(tensors[f].data_ptr()) for f in FIELDS])

    @classmethod
    def from_state(cls, state: dict, device="cuda"):
        import numpy as np
        import torch
        n = len(state["x"])
        t = {}
        for f in FIELDS:
            if f in state:
                t[f] = torch.as_tensor(np.ascontiguousarray(state[f], dtype=np.float64)).to(device)
            else:
                t[f] = torch.zeros(n, dtype=torch.float64, device=device)
        return cls(t)

    def numpy(self) -> dict:
        return {f: self.t[f].detach().cpu().numpy() for f in FIELDS}

    def __getitem__(self, k):
        return self.t[k]


class Context:
    """One sph_ctx: a single particle set, or a batch of independent sets."""

    def __init__(self, params: dict, set_offsets=None, set_box=None):
        self.params = dict(params)
        self._p = make_params(params)
        self._h = _ctx_p()
        if set_offsets is None:
            st = _lib.sph_create(ctypes.byref(self._p), ctypes.byref(self._h))
            self.nsets = 1
        else:
            offs = (c_int64 * len(set_offsets))(*[int(v) for v in set_offsets])
            box = None
            if set_box is not None:
                flat = [float(v) for v in set_box]
                box = (c_double * len(flat))(*flat)
            self.nsets = len(set_offsets) - 1
            st = _lib.sph_create_batch(ctypes.byref(self._p), self.nsets, offs, box,
                                       ctypes.byref(self._h))
        if st != SPH_OK:
            raise SphError(st, "sph_create failed (invalid parameters)")

    def close(self):
        if self._h:
            _lib.sph_destroy(self._h)
            self._h = _ctx_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != SPH_OK:
            raise SphError(st, _lib.sph_last_error(self._h).decode())

    def build_tree(self, P: ParticleArrays, stream=None):
        self._check(_lib.sph_build_tree(self._h, ctypes.byref(P.c), P.n, _stream_ptr(stream)))

    def density(self, P: ParticleArrays, stream=None):
        self._check(_lib.sph_density(self._h, ctypes.byref(P.c), _stream_ptr(stream)))

    def forces(self, P: ParticleArrays, stream=None):
        self._check(_lib.sph_forces(self._h, ctypes.byref(P.c), _stream_ptr(stream)))

    def init(self, P: ParticleArrays, stream=None):
        self._check(_lib.sph_init(self._h, ctypes.byref(P.c), P.n, _stream_ptr(stream)))

    def step(self, P: ParticleArrays, dt: float = 0.0, stream=None):
        self._check(_lib.sph_step(self._h, ctypes.byref(P.c), float(dt), _stream_ptr(stream)))

    def graph_capture_step(self, P: ParticleArrays, dt: float = 0.0, stream=None):
        self._check(_lib.sph_graph_capture_step(self._h, ctypes.byref(P.c), float(dt),
                                                _stream_ptr(stream)))

    def graph_launch(self, stream=None):
        self._check(_lib.sph_graph_launch(self._h, _stream_ptr(stream)))

    def autotune(self, P: ParticleArrays, stream=None) -> int:
        b = c_int32(0)
        self._check(_lib.sph_autotune(self._h, ctypes.byref(P.c), ctypes.byref(b),
                                      _stream_ptr(stream)))
        return int(b.value)

    def neighbors(self, P: ParticleArrays, mode: int = MODE_GATHER, stream=None):
        """CSR (offsets int64 [n+1], idx int32) of the gather or force sets."""
        import torch
        dev = P.t["x"].device
        offsets = torch.zeros(P.n + 1, dtype=torch.int64, device=dev)
        need = c_int64(0)
        st = _lib.sph_neighbors(self._h, ctypes.byref(P.c), mode, c_void_p(offsets.data_ptr()),
                                None, 0, ctypes.byref(need), _stream_ptr(stream))
        if st not in (SPH_OK, SPH_ERR_CAPACITY):
            self._check(st)
        idx = torch.empty(max(int(need.value), 1), dtype=torch.int32, device=dev)
        st = _lib.sph_neighbors(self._h, ctypes.byref(P.c), mode, c_void_p(offsets.data_ptr()),
                                c_void_p(idx.data_ptr()), idx.numel(), ctypes.byref(need),
                                _stream_ptr(stream))
        self._check(st)
        return offsets, idx[: int(need.value)]

    def set_timing(self, on: bool = True):
        self._check(_lib.sph_set_timing(self._h, 1 if on else 0))

    def stats(self) -> dict:
        s = Stats()
        self._check(_lib.sph_get_stats(self._h, ctypes.byref(s)))
        d = {f: getattr(s, f) for f, _ in Stats._fields_}
        d["momentum"] = tuple(s.momentum)
        d["groups_by_level"] = tuple(s.groups_by_level)
        return d
