"""The work-queue K solve sweeps (d3m_tuning.solve_chain) on the GPU.

Each of the two sweeps over the factor of -K runs as one launch whose
work-groups take the level-by-level schedule's update tasks from a queue and
wait on write counts of the vector tiles.  Every product and sum is formed as
in the level-by-level launches, in the same order per tile, so the fields
must agree with those launches bit for bit: FP64 and FP32 factors (with FP64
refinement), 16 and 32 right-hand sides per work-group, ragged column blocks
(40 right-hand sides), the allocation-free solve, a batch of problems whose
elimination forests differ in height, and a repeat of the same solve.  The
oracle comparison (E within 1e-10 of the largest entry, per right-hand side)
covers the path once more on its own.  A zero bound on the dependency waits
makes the waits run out: the solve must fail with D3M_EHIP (every kernel
still ends), and the next solve with the normal bound must be exact again.
"""
import math

import numpy as np
import pytest

import workloads as W
from parity import assert_rhs_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "cfg1": lambda: W.make_config(1),
    "cross_lines_2x2x2": lambda: W.make_problem(4, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=3, seed=1),
    "uneven_1x3x2": lambda: W.make_problem(7, (1, 3, 2), eps=("uniform", 1, 4), k=5.0, nrhs=1, seed=4,
                                           cuts=[[0, 7], [0, 2, 3, 7], [0, 5, 7]]),
    "many_rhs_40": lambda: W.make_problem(4, (2, 2, 1), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=40, seed=5),
    "cfg2": lambda: W.make_config(2),
}

_cache = {}


def _setup(name):
    if name not in _cache:
        from paper_2002_05018_amd import Solver
        prob = CASES[name]()
        print(f"[gpu chain] case {name}: n={prob.n} parts={prob.parts} nrhs={prob.nrhs}", flush=True)
        s = Solver.from_problem(prob)
        f = torch.from_numpy(s.rhs_planewave(prob.dirs, prob.pols)).cuda()
        _cache[name] = (prob, s, f)
    return _cache[name]


def _solve_both(s, f, cols):
    s.set_tuning(solve_chain=0, solve_cols=cols)
    ref, inf0 = s.solve(f, with_info=True)
    s.set_tuning(solve_chain=1, solve_cols=cols)
    got, inf1 = s.solve(f, with_info=True)
    s.set_tuning(solve_chain=0, solve_cols=0)
    return ref, inf0, got, inf1


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("cols", [16, 32])
@pytest.mark.parametrize("name", list(CASES))
def test_chain_matches_level_launches_bitwise(name, cols, precision):
    prob, s, f = _setup(name)
    print(f"[gpu chain] {name} cols={cols} {precision}", flush=True)
    s.factor(precision)
    ref, inf0, got, inf1 = _solve_both(s, f, cols)
    assert torch.equal(got, ref)
    assert inf1["iterations"] == inf0["iterations"]
    assert inf1["residual"] == inf0["residual"] <= 1e-10


def test_chain_against_oracle():
    from oracle.d3m import D3MOracle
    prob, s, f = _setup("cross_lines_2x2x2")
    s.factor("fp64")
    s.set_tuning(solve_chain=1)
    E = s.solve(f).cpu().numpy()
    s.set_tuning(solve_chain=0)
    o = D3MOracle.from_problem(prob).factor()
    assert_rhs_close(E, o.solve(f.cpu().numpy()), 1e-10, "E (work-queue K sweeps)")


def test_chain_repeatable():
    prob, s, f = _setup("cfg2")
    s.factor("fp64")
    s.set_tuning(solve_chain=1)
    a = s.solve(f)
    b = s.solve(f)
    s.set_tuning(solve_chain=0)
    want = s.solve(f)
    assert torch.equal(a, b)
    assert torch.equal(a, want)


def test_chain_in_the_allocation_free_solve():
    # (a problem whose vectors fit the allocation-free solve's scratch)
    prob, s, f = _setup("cross_lines_2x2x2")
    s.factor("fp64")
    s.set_tuning(solve_chain=1)
    out = torch.full_like(f, complex("nan"))
    s.solve_noalloc(f, out)
    torch.cuda.synchronize()
    s.set_tuning(solve_chain=0)
    assert torch.equal(out, s.solve(f))


def test_chain_in_a_batch():
    from paper_2002_05018_amd import Solver
    probs = W.make_batch_config(seed=11, count=4, n_range=(4, 9), nrhs=3)
    print(f"[gpu chain] batch of {len(probs)}", flush=True)
    s = Solver.batch(probs, probs[0].k, probs[0].alpha)
    dirs = np.stack([p.dirs for p in probs])
    pols = np.stack([p.pols for p in probs])
    f = torch.from_numpy(s.rhs_planewave_batch(dirs, pols)).cuda()
    for precision in ("fp64", "fp32_ir"):
        s.factor(precision)
        ref, inf0, got, inf1 = _solve_both(s, f, 32)
        assert torch.equal(got, ref), precision
        assert inf1["residual"] <= 1e-10


def test_chain_wait_timeout_is_reported():
    from paper_2002_05018_amd import D3MError
    prob, s, f = _setup("cfg2")
    s.factor("fp64")
    s.set_tuning(solve_chain=0)
    want = s.solve(f)
    s.set_tuning(solve_chain=1)
    s.set_chain_wait_limit(0.0)
    print("[gpu chain] zero wait bound: the solve must fail", flush=True)
    with pytest.raises(D3MError, match="timed out"):
        s.solve(f)
    s.set_chain_wait_limit(2.0)
    got = s.solve(f)
    s.set_tuning(solve_chain=0)
    assert torch.equal(got, want)
