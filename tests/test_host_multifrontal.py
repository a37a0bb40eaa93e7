"""Host-side checks of the multifrontal schedule of step 5 (no GPU): the
planner builds it for both pivot scopes, the update-matrix pool reuses space
(smaller than all update matrices together), the reported extend-add bytes
count every update matrix read once, and bad options are refused."""
import math

import pytest

import workloads as W

TILE_BYTES = 64 * 64 * 16


@pytest.mark.parametrize("scope", [0, 1])
def test_multifrontal_plan_sizes(scope):
    from paper_2002_05018_amd import Solver
    prob = W.make_problem(6, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=1, seed=31)
    rl = Solver.from_problem(prob, host_only=True, pivot_scope=scope).query()
    mf = Solver.from_problem(prob, host_only=True, pivot_scope=scope, multifrontal=True).query()
    assert rl["k_multifrontal"] == 0 and rl["mf_pool_bytes"] == 0
    assert mf["k_multifrontal"] == 1
    assert mf["n_units"] == rl["n_units"] and mf["n_unit_levels"] == rl["n_unit_levels"]
    assert 0 < mf["mf_pool_bytes"] <= mf["mf_update_bytes"]
    assert mf["mf_pool_bytes"] % TILE_BYTES == 0
    # every update matrix below a root is written once (initial value) and
    # read once by its parent's extend-add
    assert mf["mf_extend_add_bytes"] >= 2 * mf["mf_update_bytes"] - 1e-6
    assert mf["array_bytes"] == rl["array_bytes"] + mf["mf_pool_bytes"]
    assert mf["flops_update_gemm"] == pytest.approx(rl["flops_update_gemm"], rel=1e-12)


def test_multifrontal_pool_reuses_space_at_24_cubed():
    from paper_2002_05018_amd import Solver
    q = Solver.from_problem(W.make_config(2), host_only=True, multifrontal=True).query()
    assert q["mf_pool_bytes"] < 0.2 * q["mf_update_bytes"]


def test_multifrontal_option_validated():
    from paper_2002_05018_amd import D3MError, _lib
    import ctypes as C
    import numpy as np
    prob = W.make_config(1)
    opt = _lib._options(host_only=True)
    opt.k_multifrontal = 2
    m = _lib.d3m_mesh(prob.xyz.shape[0], prob.xyz.ctypes.data_as(C.POINTER(C.c_double)),
                      prob.tets.shape[0], prob.tets.ctypes.data_as(C.POINTER(C.c_int64)))
    part = np.ascontiguousarray(prob.part, dtype=np.int32)
    eps = np.ascontiguousarray(prob.eps_r, dtype=np.float64)
    h = C.c_void_p()
    rc = _lib._lib.d3m_setup(C.byref(m), part.ctypes.data_as(C.POINTER(C.c_int32)),
                             eps.ctypes.data_as(C.POINTER(C.c_double)), float(prob.k),
                             _lib.d3m_c128(prob.alpha.real, prob.alpha.imag), C.byref(opt), C.byref(h))
    with pytest.raises(D3MError, match="k_multifrontal"):
        _lib._check(rc)
