"""Step 1 over nested-dissection row orders (d3m_options.s1_order = 1) on the GPU.

Reordering the edge rows of M_d (and padding each dissection group to a tile
boundary) changes the elimination order of step 1, not its result: the
domain matrices K_D^(d) are unique, so they must match the oracle's to
1e-12, and the field and multipliers to the method's 1e-10 per right-hand
side, element-wise; the FP32 factors with FP64 refinement reach the 1e-10
residual and agree with the oracle to 1e-9.  At 12^3-hex subdomains (24^3,
2x2x2) the field must agree with the default banded order's to 1e-10 and
the relative residual, evaluated on the host with the oracle's own global S
and load, must be at most 1e-10 per right-hand side.

The batch workload's largest subdomains (32^3 hexes in 2x2x2 subdomains of
16^3, four wavelengths across: workloads.make_large_subdomain_config) are
checked against the oracle's S and load on the host, both orders at 1e-10;
the two fields agree to 1e-9 (the dissection's step 1 has a multiplier
growth of about 650 there under tile-restricted pivoting, 13.5 banded).
"""
import math

import numpy as np
import pytest

import workloads as W
from parity import assert_rhs_close, host_residual, matrix_max_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "cfg1": lambda: W.make_config(1),
    "cross_lines_2x2x2": lambda: W.make_problem(4, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=3, seed=1),
    "uneven_1x3x2": lambda: W.make_problem(7, (1, 3, 2), eps=("uniform", 1, 4), k=5.0, nrhs=1, seed=4,
                                           cuts=[[0, 7], [0, 2, 3, 7], [0, 5, 7]]),
    "big_box_8x1x1": lambda: W.make_problem(8, (2, 1, 1), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=2, seed=2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_nested_dissection_against_oracle(name):
    from oracle.d3m import D3MOracle
    from paper_2002_05018_amd import Solver
    prob = CASES[name]()
    print(f"[gpu nd] case {name}: n={prob.n} parts={prob.parts} nrhs={prob.nrhs}", flush=True)
    s = Solver.from_problem(prob, s1_order=1)
    o = D3MOracle.from_problem(prob).factor()
    f = s.rhs_planewave(prob.dirs, prob.pols)
    Eo = o.solve(f)
    fd = torch.from_numpy(f).cuda()
    s.factor("fp64")
    E, info = s.solve(fd, with_info=True)
    assert_rhs_close(E.cpu().numpy(), Eo, 1e-10, "E (nested dissection)")
    assert info["residual"] <= 1e-11
    if o.dec.n_lm:
        assert_rhs_close(s.export("lambda", prob.nrhs), o.lam, 1e-10, "lambda (nested dissection)")
        for d in range(o.dec.N):
            assert matrix_max_rel(s.export("kd", d), o.dm.KD[d]) <= 1e-12, d
    s.factor("fp32_ir")
    E32, info32 = s.solve(fd, with_info=True)
    assert info32["converged"] and info32["residual"] <= 1e-10
    assert_rhs_close(E32.cpu().numpy(), Eo, 1e-9, "E FP32+IR (nested dissection)")


def test_large_subdomains_against_banded_order_and_oracle_residual():
    from oracle.fem import GlobalFEM
    from paper_2002_05018_amd import Solver
    prob = W.make_problem(24, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=4, seed=7)
    print("[gpu nd] 24^3 hexes, 2x2x2 subdomains of 12^3", flush=True)
    g = GlobalFEM(prob.xyz, prob.tets, prob.eps_r, prob.k)
    fo = g.planewave_rhs(prob.dirs, prob.pols)
    fd = torch.from_numpy(fo).cuda()
    nd = Solver.from_problem(prob, s1_order=1)
    band = Solver.from_problem(prob)
    assert nd.info["flops_domain"] < 0.6 * band.info["flops_domain"]
    nd.factor("fp64")
    band.factor("fp64")
    E = nd.solve(fd).cpu().numpy()
    Eb = band.solve(fd).cpu().numpy()
    assert_rhs_close(E, Eb, 1e-10, "E nested dissection vs banded")
    res = host_residual(g.S, E, fo)
    assert np.all(res <= 1e-10), res
    nd.factor("fp32_ir")
    E32, info = nd.solve(fd, with_info=True)
    assert info["converged"] and info["residual"] <= 1e-10
    assert np.all(host_residual(g.S, E32.cpu().numpy(), fo) <= 1e-10)


def test_large_subdomains_high_frequency_oracle_residual():
    from oracle.fem import GlobalFEM
    from paper_2002_05018_amd import Solver
    prob = W.make_large_subdomain_config()
    print("[gpu nd] 32^3 hexes, 2x2x2 subdomains of 16^3, k = 8 pi", flush=True)
    g = GlobalFEM(prob.xyz, prob.tets, prob.eps_r, prob.k)
    fo = g.planewave_rhs(prob.dirs, prob.pols)
    fd = torch.from_numpy(fo).cuda()
    band = Solver.from_problem(prob)
    band.factor("fp64")
    Eb = band.solve(fd).cpu().numpy()
    rb = host_residual(g.S, Eb, fo)
    print(f"[gpu nd] banded FP64 residual {rb.max():.2e} growth {band.growth()}", flush=True)
    assert np.all(rb <= 1e-10), rb
    del band
    torch.cuda.empty_cache()
    nd = Solver.from_problem(prob, s1_order=1)
    nd.factor("fp64")
    E = nd.solve(fd).cpu().numpy()
    r = host_residual(g.S, E, fo)
    print(f"[gpu nd] dissection FP64 residual {r.max():.2e} growth {nd.growth()}", flush=True)
    assert np.all(r <= 1e-10), r
    assert_rhs_close(E, Eb, 1e-9, "E nested dissection vs banded")
    nd.factor("fp32_ir")
    E32, info = nd.solve(fd, with_info=True)
    assert info["converged"] and info["residual"] <= 1e-10
