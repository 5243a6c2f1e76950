"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function include/simrank.h declares, derives the parameters the oracle
derives, and rejects malformed input before touching the device."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2304_04015_amd import simrank as S


@pytest.fixture(scope="module")
def L():
    return S.lib()


def test_exports_every_declared_function(L):
    names = S.header_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(L, name), name
    assert S.simrank_version().startswith("simrank")


@pytest.mark.parametrize("eps,c,L_,n,union", [
    (0.02, 0.6, 64, 1 << 20, False), (0.05, 0.6, 64, 1 << 20, False),
    (0.01, 0.6, 64, 1 << 20, False), (0.02, 0.6, 32, 500, True), (0.1, 0.8, 16, 100, False),
    (0.03, 0.36, 255, 10, True),
])
def test_derive_params_matches_oracle(eps, c, L_, n, union):
    q = S.make_query(0, c=c, eps=eps, delta=1e-3, walk_cap=L_, union_bound=union)
    p = S.simrank_derive_params(q, n)
    assert p.L == L_
    assert p.R == exact.hoeffding_R(eps, 1e-3, c, L_, n=n if union else None)
    assert p.T == oracle.continue_threshold(c)


def test_derive_params_defaults_and_override():
    q = S.make_query(0, walk_cap=0)
    assert S.simrank_derive_params(q, 10).L == 64
    q = S.make_query(0, R=123)
    assert S.simrank_derive_params(q, 10).R == 123


@pytest.mark.parametrize("kw", [
    dict(c=0.0), dict(c=1.0), dict(eps=0.0), dict(eps=1.0), dict(delta=0.0), dict(delta=1.0),
    dict(walk_cap=256), dict(walk_cap=-1), dict(R=-1), dict(mode=7),
    dict(eps=1e-12),                      # R beyond 2^24
    dict(mode=S.MODE_STITCHED, walk_cap=65),
])
def test_derive_params_rejects(kw):
    q = S.make_query(0, **kw)
    with pytest.raises(S.SimRankError) as e:
        S.simrank_derive_params(q, 100)
    assert e.value.code == S.SIMRANK_EINVAL


def test_eps_below_truncation_bias_rejected():
    # c^(L+1) at c = 0.9, L = 4 is 0.59: eps = 0.5 leaves nothing for sampling
    q = S.make_query(0, c=0.9, eps=0.5, walk_cap=4)
    with pytest.raises(S.SimRankError, match="c\\^\\(L\\+1\\)"):
        S.simrank_derive_params(q, 100)


@pytest.mark.parametrize("off,src,m,msg", [
    ([1, 1, 2], [0, 1], 2, "in_off\\[0\\]"),
    ([0, 2, 1], [0, 1], 2, "decreases"),
    ([0, 1, 2], [0, 1, 7], 3, "in_off\\[n\\]"),
    ([0, 1, 2], [0, 5], 2, "out of range"),
    ([0, 1, 2], [-1, 0], 2, "out of range"),
])
def test_load_graph_rejects_malformed_csr(off, src, m, msg):
    import ctypes as C
    h = C.c_void_p()
    offa = np.array(off, np.int32)
    srca = np.array(src, np.int32)
    rc = S.lib().simrank_load_graph(2, m, offa.ctypes.data, srca.ctypes.data, C.byref(h))
    assert rc == S.SIMRANK_EINVAL
    assert h.value is None
    import re
    assert re.search(msg, S.lib().simrank_last_error().decode())


def test_null_arguments_rejected():
    assert S.lib().simrank_load_graph(2, 0, None, None, None) == S.SIMRANK_EINVAL
    assert b"NULL" in S.lib().simrank_last_error()
    assert S.lib().simrank_derive_params(None, 10, None) == S.SIMRANK_EINVAL
    assert S.lib().simrank_single_source(None, 0, 0.6, 0.02, 1e-3, None) == S.SIMRANK_EINVAL
    assert S.lib().simrank_free_graph(None) == S.SIMRANK_OK
    assert S.lib().simrank_workspace_free(None) == S.SIMRANK_OK
    assert S.lib().simrank_batch(None, 0, None, 0, None, None, None) == S.SIMRANK_OK
    assert S.lib().simrank_last_error() == b""
    assert S.lib().simrank_set_tuning(None, 0, 0) == S.SIMRANK_EINVAL
    assert S.lib().simrank_tune_ex(None, None, None) == S.SIMRANK_EINVAL
    assert S.lib().simrank_tune_index(None, None, None, None, 1, None, None) == S.SIMRANK_EINVAL


def test_plan_flags_checked_before_any_device_work():
    import ctypes as C
    h, ng = C.c_void_p(), C.c_int32(-1)
    q = S.make_query(0)
    rc = S.lib().simrank_batch_plan_create_ex(None, 0, C.byref(q), 1, 2, C.byref(h), C.byref(ng))
    assert rc == S.SIMRANK_EINVAL and h.value is None and ng.value == 0
    assert b"flags" in S.lib().simrank_last_error()
    rc = S.lib().simrank_batch_plan_create_ex(None, 0, C.byref(q), 0, S.PLAN_GROUPS, C.byref(h), None)
    assert rc == S.SIMRANK_EINVAL and h.value is None


def test_union_bound_grows_R():
    q1 = S.make_query(0, eps=0.02)
    q2 = S.make_query(0, eps=0.02, union_bound=True)
    n = 1 << 20
    r1 = S.simrank_derive_params(q1, n).R
    r2 = S.simrank_derive_params(q2, n).R
    assert r2 > r1
    assert r2 == math.ceil(math.log(2 * n / 1e-3) / (2 * (0.02 - 0.6 ** 65) ** 2))


# ------------------------------------------------ length-stratified estimator

@pytest.mark.parametrize("n,c,eps,z,phi", [(500, 0.6, 0.05, 0, 0), (1 << 20, 0.6, 0.02, 0, 0),
                                           (1 << 24, 0.6, 0.02, 0, 0), (1000, 0.8, 0.03, 0, 0),
                                           (300, 0.6, 0.05, 2000, 9), (2, 0.6, 0.9, 100, 0),
                                           (4096, 0.5, 0.1, 0, 40)])
def test_derive_stratified_matches_oracle(n, c, eps, z, phi):
    q = S.make_stratified_query(0, c=c, eps=eps, z=z, phi=phi)
    p = S.simrank_derive_stratified(q, n)
    want = oracle.strat_params(n, c, eps, z=float(z), phi=phi)
    assert p.z == want.z
    assert (p.N, p.phi) == (want.N, want.phi)
    # the shuffle grid: A * 2^b >= N, 2^b about sqrt(N), fewer than 2 sqrt(N) points to spare
    assert p.shuffle_A * 2 ** p.shuffle_b >= p.N > (p.shuffle_A - 1) * 2 ** p.shuffle_b
    assert 2 ** p.shuffle_b <= 2 * math.sqrt(p.N) + 1 and p.shuffle_A <= math.sqrt(p.N) + 1
    # the generic parameter call reports N and phi as R and L
    gp = S.simrank_derive_params(q, n)
    assert (gp.R, gp.L) == (p.N, p.phi)


@pytest.mark.parametrize("kw", [dict(eps=0.006, n=500),           # eps <= 3/n
                                dict(eps=0.05, n=1),              # phi = 0
                                dict(eps=0.05, n=500, phi=256),
                                dict(eps=0.0001, n=1 << 30),      # N >= 2^24
                                dict(eps=0.05, n=500, z=-3)])
def test_derive_stratified_rejects(kw):
    n = kw.pop("n")
    q = S.make_stratified_query(0, c=0.6, **kw)
    with pytest.raises(S.SimRankError) as e:
        S.simrank_derive_stratified(q, n)
    assert e.value.code == S.SIMRANK_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library the binding raises on first use; there is no
    CPU fallback on the product path."""
    import os
    import subprocess
    import sys
    env = dict(os.environ, SIMRANK_LIB=str(tmp_path / "absent.so"))
    code = ("from paper_2304_04015_amd import simrank as S\n"
            "try:\n"
            "    S.lib()\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n"
            "else:\n"
            "    print('loaded')\n")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))), timeout=300)
    assert "raised" in r.stdout and "absent.so" in r.stdout, (r.stdout, r.stderr)


def test_device_buffers_checked_before_the_call():
    """The binding refuses device buffers the kernels would overrun or misread:
    host tensors, strided views, wrong element sizes, fewer than n elements."""
    import torch

    class Dev:                      # a stand-in for a device tensor
        def __init__(self, n, itemsize, contiguous=True):
            self.device = type("D", (), {"type": "cuda"})()
            self._n, self._s, self._c = n, itemsize, contiguous

        def is_contiguous(self):
            return self._c

        def element_size(self):
            return self._s

        def numel(self):
            return self._n

        def data_ptr(self):
            return 0x1000

    assert S._dev_ptr(Dev(10, 4), 10, 4, "x") == 0x1000
    assert S._dev_ptr(None, 10, 4, "x") is None
    assert S._dev_ptr(0x2000, 10, 4, "x") == 0x2000
    for bad in (Dev(9, 4), Dev(10, 8), Dev(10, 4, contiguous=False),
                torch.zeros(10, dtype=torch.int32)):
        with pytest.raises(S.SimRankError) as e:
            S._dev_ptr(bad, 10, 4, "x")
        assert e.value.code == S.SIMRANK_EINVAL
