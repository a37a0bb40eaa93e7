"""The allocation-free FP64 solve (d3m_solve_noalloc), for callers that
cannot allocate device memory, against the ordinary d3m_solve.

Both run the same kernels on the same factors, so the fields must agree bit
for bit; two calls in a row (the second with fewer right-hand sides and
other values) check that the shared scratch keeps no state between calls.
Sizes beyond the scratch limit, host buffers and handles without FP64
factors are refused before any kernel runs.
"""
import ctypes

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver():
    from paper_2002_05018_amd import Solver
    prob = W.make_problem(5, (2, 2, 1), eps=("uniform", 1, 4), k=2 * np.pi, nrhs=6, seed=31)
    print(f"[no-alloc] n={prob.n} parts={prob.parts} nrhs={prob.nrhs}", flush=True)
    s = Solver.from_problem(prob)
    f = torch.from_numpy(s.rhs_planewave(prob.dirs, prob.pols)).cuda()
    return s, f


def test_noalloc_solve_matches_solve_on_two_calls():
    s, f = _solver()
    s.factor("fp64")
    want = s.solve(f)
    out = torch.full_like(f, complex("nan"))
    s.solve_noalloc(f, out)
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    # a second call with fewer right-hand sides and other values
    f2 = (f[1:3] * (0.5 - 0.25j)).contiguous()
    want2 = s.solve(f2)
    out2 = torch.full_like(f2, complex("nan"))
    s.solve_noalloc(f2, out2)
    torch.cuda.synchronize()
    assert torch.equal(out2, want2)
    # and the first size again (the scratch still holds the second call's data)
    out3 = torch.empty_like(f)
    s.solve_noalloc(f, out3)
    torch.cuda.synchronize()
    assert torch.equal(out3, want)


def test_noalloc_refuses_what_it_cannot_do():
    from paper_2002_05018_amd import D3MError
    from paper_2002_05018_amd._lib import _lib
    s, f = _solver()
    out = torch.empty_like(f)
    with pytest.raises(D3MError, match="ESTATE"):
        s.solve_noalloc(f, out)  # not factored
    s.factor("fp32_ir")
    with pytest.raises(D3MError, match="ESTATE"):
        s.solve_noalloc(f, out)  # FP32 factors
    s.factor("fp64")
    # more right-hand sides than the scratch holds: refused with the need
    big = torch.zeros((4096, s.n_edges), dtype=torch.complex128, device="cuda")
    with pytest.raises(D3MError, match="EINVAL.*bytes of scratch"):
        s.solve_noalloc(big, torch.empty_like(big))
    # host buffers through the C ABI directly (the binding refuses them first)
    fh = f.cpu()
    oh = torch.empty_like(fh)
    rc = _lib.d3m_solve_noalloc(s._handle, ctypes.c_void_p(fh.data_ptr()), fh.shape[0],
                                ctypes.c_void_p(oh.data_ptr()), None)
    assert rc == -1 and b"device buffers" in _lib.d3m_last_error()
