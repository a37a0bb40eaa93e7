"""The C ABI library loads, exports every symbol include/d3m.h declares, and
rejects bad input on the host (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "d3m.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(d3m_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2002_05018_amd import _lib, library_path
    lib = ctypes.CDLL(library_path)
    decl = _declared()
    assert len(decl) >= 13
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(_lib.exported_symbols)


def _setup(prob, **kw):
    from paper_2002_05018_amd import Solver
    return Solver.from_problem(prob, host_only=True, **kw)


def test_error_paths():
    from paper_2002_05018_amd import D3MError, Solver
    prob = W.make_problem(2, (2, 1, 1))
    # empty subdomain: ids must be dense
    part = prob.part.copy()
    part[part == 1] = 2
    with pytest.raises(D3MError) as ei:
        Solver(prob.xyz, prob.tets, part, prob.eps_r, prob.k, prob.alpha, host_only=True)
    assert ei.value.status == "D3M_EINVAL"
    with pytest.raises(D3MError) as ei:
        Solver(prob.xyz, prob.tets, prob.part, prob.eps_r, -1.0, prob.alpha, host_only=True)
    assert ei.value.status == "D3M_EINVAL"
    tets = prob.tets.copy()
    tets[0, 1] = tets[0, 0]
    with pytest.raises(D3MError) as ei:
        Solver(prob.xyz, tets, prob.part, prob.eps_r, prob.k, prob.alpha, host_only=True)
    assert ei.value.status == "D3M_EINVAL"
    xyz = prob.xyz.copy()
    xyz[prob.tets[0]] = xyz[prob.tets[0, 0]]  # collapse a tetrahedron
    with pytest.raises(D3MError):
        Solver(xyz, prob.tets, prob.part, prob.eps_r, prob.k, prob.alpha, host_only=True)
    s = _setup(prob)
    with pytest.raises(D3MError) as ei:
        s.factor("fp64")
    assert ei.value.status == "D3M_ESTATE"


def test_query_counts():
    s = _setup(W.make_config(1))
    q = s.query()
    assert q["n_edges"] == 1854 and q["n_lm"] == 246 and q["n_blocks"] == 4
    assert q["n_subdomains"] == 4 and q["max_block"] == 63
    assert q["flops_domain"] > 0 and q["flops_block_ldlt"] > 0


def test_debug_bk_rejects_bad_arguments_on_the_host():
    """The Bunch-Kaufman test hook validates its arguments before any HIP
    call; without a device a valid call reports D3M_ENODEV."""
    from paper_2002_05018_amd import D3MError
    from paper_2002_05018_amd._lib import debug_bk
    a = np.eye(4, dtype=np.complex128)[None]
    with pytest.raises(D3MError, match="EINVAL"):
        debug_bk(a, variant=3)
    with pytest.raises(D3MError, match="EINVAL"):
        debug_bk(a, precision=7)
    with pytest.raises(D3MError, match="EINVAL"):
        debug_bk(np.eye(300, dtype=np.complex128)[None], variant=1)  # 300 rows do not fit in LDS
    with pytest.raises(ValueError):
        debug_bk(np.zeros((2, 3, 4)))
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(D3MError, match="ENODEV"):
            debug_bk(a)


def test_binding_rejects_mismatched_buffers_on_the_host():
    """solve/adjoint check caller buffers before handing pointers to the
    library (a wrong shape, dtype, layout or device would be an out-of-bounds
    access there); eps_r must have one value per tetrahedron."""
    import torch
    prob = W.make_problem(2, (2, 1, 1))
    s = _setup(prob)
    n = s.n_edges
    f = torch.zeros((2, n), dtype=torch.complex128)
    bad_outs = [torch.zeros((2, n + 1), dtype=torch.complex128), torch.zeros((2, n), dtype=torch.complex64),
                torch.zeros((n, 2), dtype=torch.complex128).t(), torch.zeros((3, n), dtype=torch.complex128)]
    for out in bad_outs:
        with pytest.raises(ValueError):
            s.solve(f, out=out)
    with pytest.raises(ValueError):
        s.adjoint(torch.zeros((2, n), dtype=torch.complex64), f)
    with pytest.raises(ValueError):
        s.adjoint(f, torch.zeros((1, n), dtype=torch.complex128))
    with pytest.raises(ValueError):
        s.adjoint(f, f.numpy())
    with pytest.raises(ValueError):
        s.update_eps(np.ones(prob.tets.shape[0] + 1))
