"""Device status word and error returns of the C interface (on the GPU).

Conditions found on the device (an iteration stopped at nr_maxit, a
non-finite result) are reported by sph_get_stats and returned once by the
next call on the context after the device has finished the call that set
them; a too-small output buffer returns SPH_ERR_CAPACITY with the size
needed.
"""
import ctypes

import numpy as np
import pytest

import sph_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_11425_amd as m
    return m


def cloud():
    return si.random_cloud(61, 3000, kernel="m4", n_ngb=50, periodic=True, clumped=True)


def test_iteration_limit_is_noconv(sph):
    c = cloud()
    s, p = c["state"], c["params"]
    # a poor first guess: one scan cannot converge
    s = dict(s, H=s["H"] * 0.6)
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(dict(p, nr_maxit=1))
    print("iteration limit -> NOCONV", flush=True)
    ctx.build_tree(P)
    ctx.density(P)
    torch.cuda.synchronize()
    # the next call reports the previous call's status and enqueues nothing
    with pytest.raises(sph.SphError) as e:
        ctx.density(P)
    assert e.value.status == sph.SPH_ERR_NOCONV
    # reported once: the call after proceeds
    ctx.density(P)
    st = ctx.stats()
    assert st["status"] == sph.SPH_ERR_NOCONV
    assert st["n_iter_limit"] > 0 and st["n_noconv"] >= st["n_iter_limit"]
    assert st["n_nonfinite"] == 0
    # a converging pass leaves the status clean
    ok = sph.Context(p)
    ok.build_tree(P)
    ok.density(P)
    st2 = ok.stats()
    assert st2["status"] == sph.SPH_OK and st2["n_iter_limit"] == 0


def test_nonfinite_input_is_reported(sph):
    c = cloud()
    s, p = c["state"], c["params"]
    s = {k: v.copy() for k, v in s.items()}
    s["x"][7] = np.nan
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(p)
    print("NaN input -> NONFINITE", flush=True)
    ctx.init(P)
    torch.cuda.synchronize()
    with pytest.raises(sph.SphError) as e:
        ctx.step(P)
    assert e.value.status == sph.SPH_ERR_NONFINITE
    ctx2 = sph.Context(p)
    P2 = sph.ParticleArrays.from_state(s)
    ctx2.init(P2)
    st = ctx2.stats()
    assert st["status"] == sph.SPH_ERR_NONFINITE and st["n_nonfinite"] >= 1
    # every other particle keeps finite results
    got = P2.numpy()
    others = np.ones(len(s["x"]), bool)
    others[7] = False
    for k in ("H", "rho", "omega", "ax", "ay", "az", "dudt", "dt"):
        assert np.all(np.isfinite(got[k][others])), k


def test_status_clean_on_normal_steps(sph):
    c = cloud()
    P = sph.ParticleArrays.from_state(c["state"])
    ctx = sph.Context(dict(c["params"], precision="mixed"))
    ctx.init(P)
    for _ in range(3):
        ctx.step(P)
        torch.cuda.synchronize()
    st = ctx.stats()
    assert st["status"] == sph.SPH_OK and st["n_nonfinite"] == 0 and st["n_iter_limit"] == 0


def test_neighbor_capacity_error(sph):
    c = cloud()
    s, p = c["state"], c["params"]
    P = sph.ParticleArrays.from_state(s)
    ctx = sph.Context(p)
    ctx.build_tree(P)
    off = torch.zeros(P.n + 1, dtype=torch.int64, device="cuda")
    idx = torch.zeros(10, dtype=torch.int32, device="cuda")
    need = ctypes.c_int64(0)
    st = sph._lib.sph_neighbors(ctx._h, ctypes.byref(P.c), sph.MODE_GATHER,
                                ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                                10, ctypes.byref(need), sph._stream_ptr(None))
    assert st == sph.SPH_ERR_CAPACITY
    assert need.value > 10
    assert int(off[-1].item()) == need.value
    # the untouched buffer is still all zeros: nothing was written to it
    assert int(idx.abs().sum().item()) == 0
