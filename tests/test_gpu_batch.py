"""GPU tests of the batching form, captured HIP graphs and the tuning knobs.

* A batch of independent problems with uneven subdomains is factored and
  solved as one handle; every problem's slice of the field must match the
  CPU oracle run on that problem alone (1e-10, the method's exactness bar),
  in FP64 and with FP32 factors plus FP64 refinement (residual 1e-10 per
  problem and right-hand side, 1e-9 against the oracle).
* Graph replays (opt.use_graph) must reproduce the eager launches bit for
  bit, replay after replay, with eager work and synchronisations between the
  replays and new right-hand-side values in the same buffer.
* Other launch shapes (blocked-update depths of the subdomain and K phases,
  solve column block, look-ahead threshold, panel rows per work-group)
  change only the summation order: results agree to 1e-12.
"""
import numpy as np
import pytest

import workloads as W
from parity import assert_rhs_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


_cache = {}


def _batch():
    if "b" not in _cache:
        from oracle.d3m import D3MOracle
        from paper_2002_05018_amd import Solver
        probs = W.make_batch_config(seed=11, count=3, n_range=(4, 7), nrhs=3)
        print(f"[gpu batch] n={[p.n for p in probs]} subdomains={[p.n_sub for p in probs]}", flush=True)
        s = Solver.batch(probs, probs[0].k, probs[0].alpha)
        f = s.rhs_planewave_batch(np.stack([p.dirs for p in probs]), np.stack([p.pols for p in probs]))
        _, eo, _ = s.layout()
        ref = []
        for p, prob in enumerate(probs):
            fp = f[:, eo[p]:eo[p + 1]]
            ref.append(D3MOracle.from_problem(prob).factor().solve(fp))
        _cache["b"] = (probs, s, f, eo, ref)
    return _cache["b"]


def test_batch_fp64_matches_oracle_per_problem():
    probs, s, f, eo, ref = _batch()
    s.factor("fp64")
    E, info = s.solve(torch.from_numpy(f).cuda(), with_info=True)
    E = E.cpu().numpy()
    assert info["residual"] <= 1e-11
    for p in range(len(probs)):
        assert_rhs_close(E[:, eo[p]:eo[p + 1]], ref[p], 1e-10, f"problem {p}")


def test_batch_fp32_refinement_per_problem():
    probs, s, f, eo, ref = _batch()
    s.factor("fp32_ir")
    E, info = s.solve(torch.from_numpy(f).cuda(), with_info=True)
    assert info["converged"] and info["residual"] <= 1e-10
    E = E.cpu().numpy()
    for p in range(len(probs)):
        assert_rhs_close(E[:, eo[p]:eo[p + 1]], ref[p], 1e-9, f"problem {p}")


def test_batch_scaled_problem_alone_differs_only_by_scale():
    """A problem of the batch is the unit cube at k = 2 pi n / 8 rescaled by
    s = n / 8, and its system is the unit-cube system divided by s (every
    term of the edge-element system scales alike), so with the same load the
    unit-cube field is the batch field divided by s."""
    from paper_2002_05018_amd import Solver
    probs, s, f, eo, ref = _batch()
    prob = probs[0]
    sc = prob.n / 8.0
    unit = W.Problem("unit", prob.n, prob.parts, prob.xyz / sc, prob.tets, prob.part, prob.eps_r,
                     prob.k * sc, -1j * prob.k * sc, prob.dirs, prob.pols)
    u = Solver.from_problem(unit)
    u.factor("fp64")
    fp = np.ascontiguousarray(f[:, eo[0]:eo[1]])
    Eu = u.solve(torch.from_numpy(fp).cuda()).cpu().numpy()
    assert_rhs_close(Eu, ref[0] / sc, 1e-10, "unit cube")


def test_graph_replays_match_eager_bitwise():
    from paper_2002_05018_amd import Solver
    prob = W.make_problem(4, (2, 2, 1), eps=("uniform", 1, 4), k=2 * np.pi, nrhs=5, seed=21)
    eager = Solver.from_problem(prob)
    graph = Solver.from_problem(prob, use_graph=True)
    f = torch.from_numpy(eager.rhs_planewave(prob.dirs, prob.pols)).cuda()
    eager.factor("fp64")
    want = eager.solve(f).cpu().numpy()
    fbuf = f.clone()
    out = torch.empty_like(f)
    for rep in range(3):
        graph.factor("fp64")  # capture on the first call, replay afterwards
        for scale in (1.0, 2.0):
            fbuf.copy_(f * scale)  # eager work between replays, same buffer
            torch.cuda.synchronize()
            graph.solve(fbuf, out=out)
            got = out.cpu().numpy()
            assert np.array_equal(got, want * scale), (rep, scale)
    # FP32 factors with refinement through graphs (the refinement loop itself is eager)
    graph.factor("fp32_ir")
    eager.factor("fp32_ir")
    Eg, ig = graph.solve(f, with_info=True)
    Ee, ie = eager.solve(f, with_info=True)
    assert ig["iterations"] == ie["iterations"]
    assert np.array_equal(Eg.cpu().numpy(), Ee.cpu().numpy())


@pytest.mark.parametrize("tune", [{"s1_block": 1}, {"s1_block": 4}, {"k_block": 1}, {"k_block": 8},
                                  {"lookahead_tasks": 1}, {"side_early": 1}, {"k_fuse": 1}, {"solve_cols": 16},
                                  {"panel_rows": 16}, {"panel_rows": 16, "k_fuse": 1}, {"solve_seq": 1},
                                  {"solve_seq": 1, "solve_cols": 16}, {"solve_seq": 1, "s1_block": 4},
                                  {"solve_narrow": 100000}, {"solve_narrow": 100000, "solve_seq": 1},
                                  {"k_overlap": 1}, {"k_overlap": 1, "k_block": 4, "lookahead_tasks": 1}])
def test_tuning_variants_agree(tune):
    from paper_2002_05018_amd import Solver
    prob = W.make_problem(5, (2, 2, 1), eps=("uniform", 1, 4), k=2 * np.pi, nrhs=40, seed=22)
    s = Solver.from_problem(prob)
    f = torch.from_numpy(s.rhs_planewave(prob.dirs, prob.pols)).cuda()
    s.factor("fp64")
    want = s.solve(f).cpu().numpy()
    s.set_tuning(**tune)
    s.factor("fp64")
    got, info = s.solve(f, with_info=True)
    assert info["residual"] <= 1e-11
    assert_rhs_close(got.cpu().numpy(), want, 1e-12, str(tune))


def test_autotune_picks_a_valid_tuning():
    from paper_2002_05018_amd import Solver, autotune
    prob = W.make_problem(4, (2, 2, 1), eps=("uniform", 1, 4), k=2 * np.pi, nrhs=20, seed=23)
    s = Solver.from_problem(prob)
    f = torch.from_numpy(s.rhs_planewave(prob.dirs, prob.pols)).cuda()
    s.factor("fp64")
    want = s.solve(f).cpu().numpy()
    res = autotune(s, f, "fp64", repeats=1)
    from paper_2002_05018_amd.autotune import DEFAULT_SPACE
    assert not res["cached"] and len(res["trials"]) == sum(len(v) for v in DEFAULT_SPACE.values())
    assert s.tuning() == res["tuning"]
    s.factor("fp64")
    assert_rhs_close(s.solve(f).cpu().numpy(), want, 1e-12, "autotuned")


def test_batch_residual_is_per_problem():
    """The reported residual is the largest over problems and right-hand sides
    of ||f_p - S_p E_p||_inf / ||f_p||_inf.  Problem p's load is scaled by
    1e3^p, which leaves each problem's relative residual unchanged, so the
    figure must match the host recomputation from the returned field (to the
    rounding of r, a few per cent of a residual near 1e-13), while a norm
    taken across problems would be off by orders of magnitude.  The small
    problems put problem boundaries inside the reduction's row blocks."""
    from oracle.d3m import relative_residual
    from oracle.fem import GlobalFEM
    probs, s, f, eo, ref = _batch()
    fs = f.copy()
    for p in range(len(probs)):
        fs[:, eo[p]:eo[p + 1]] *= 1e3 ** p
    s.factor("fp64")
    E, info = s.solve(torch.from_numpy(fs).cuda(), with_info=True)
    E = E.cpu().numpy()
    want = 0.0
    for p, prob in enumerate(probs):
        S = GlobalFEM(prob.xyz, prob.tets, prob.eps_r, prob.k).S
        sl = slice(eo[p], eo[p + 1])
        want = max(want, relative_residual(S, E[:, sl], fs[:, sl]))
    assert info["converged"]
    assert abs(info["residual"] - want) <= 0.05 * want, (info["residual"], want)


def test_nonfinite_load_never_counts_as_converged():
    """A NaN in the load makes the field NaN; the residual reduction must pass
    the NaN on (FP64: residual NaN, not converged; FP32 factors: refinement
    reports no convergence) instead of dropping it as a maximum would."""
    from paper_2002_05018_amd import Solver
    from paper_2002_05018_amd._lib import D3MError
    prob = W.make_problem(4, (2, 1, 1), eps=("uniform", 1, 4), k=2 * np.pi, nrhs=3, seed=24)
    s = Solver.from_problem(prob)
    f = s.rhs_planewave(prob.dirs, prob.pols)
    f[1, 7] = np.nan
    fd = torch.from_numpy(f).cuda()
    s.factor("fp64")
    _, info = s.solve(fd, with_info=True)
    assert np.isnan(info["residual"]) and not info["converged"]
    s.factor("fp32_ir")
    with pytest.raises(D3MError):
        s.solve(fd, with_info=True)


def test_overlapped_k_schedule_is_bitwise_identical():
    """k_overlap only changes which launches may run at the same time: every
    target tile still receives its updates in the same order, so the field is
    bit for bit the one of the default schedule, eager and replayed from a
    captured graph (three streams joined in the capture)."""
    from paper_2002_05018_amd import Solver
    prob = W.make_problem(8, (2, 2, 2), eps=("uniform", 1, 4), k=2 * np.pi, nrhs=3, seed=25)
    print(f"[gpu batch] k_overlap n={prob.n} parts={prob.parts}", flush=True)
    s = Solver.from_problem(prob)
    f = torch.from_numpy(s.rhs_planewave(prob.dirs, prob.pols)).cuda()
    s.set_tuning(lookahead_tasks=1, k_block=2)
    s.factor("fp64")
    want = s.solve(f).cpu().numpy()
    s.set_tuning(k_overlap=1)
    s.factor("fp64")
    assert np.array_equal(s.solve(f).cpu().numpy(), want)
    g = Solver.from_problem(prob, use_graph=True)
    g.set_tuning(lookahead_tasks=1, k_block=2, k_overlap=1)
    for _ in range(3):
        g.factor("fp64")
        got = g.solve(f).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(got, want)


def test_batch_multifrontal_and_pec_problem():
    """The batching form with step 5 in multifrontal form, and a batch whose
    middle problem holds a PEC plate: every problem equals the oracle run on
    it alone (its PEC plate included) to 1e-10, E is zero on the PEC edges."""
    from oracle.d3m import D3MOracle
    from paper_2002_05018_amd import Solver
    probs, s, f, eo, ref = _batch()
    mf = Solver.batch(probs, probs[0].k, probs[0].alpha, multifrontal=True)
    assert mf.query()["k_multifrontal"] == 1
    mf.factor("fp64")
    E = mf.solve(torch.from_numpy(f).cuda()).cpu().numpy()
    for p in range(len(probs)):
        assert_rhs_close(E[:, eo[p]:eo[p + 1]], ref[p], 1e-10, f"multifrontal problem {p}")
    import copy
    pp = [copy.copy(q) for q in probs]
    n = pp[1].n
    pp[1].pec_faces = W.plate_faces(n, pp[1].tets, 2, n // 2, [1, 1], [n - 1, n - 2])
    b = Solver.batch(pp, pp[0].k, pp[0].alpha)
    fb = b.rhs_planewave_batch(np.stack([q.dirs for q in pp]), np.stack([q.pols for q in pp]))
    _, eb, _ = b.layout()
    b.factor("fp64")
    Eb, info = b.solve(torch.from_numpy(fb).cuda(), with_info=True)
    Eb = Eb.cpu().numpy()
    assert info["residual"] <= 1e-10
    for p, prob in enumerate(pp):
        o = D3MOracle.from_problem(prob).factor()
        Eo = o.solve(fb[:, eb[p]:eb[p + 1]])
        Ep = Eb[:, eb[p]:eb[p + 1]]
        assert not np.any(Ep[:, o.fem.pec])
        assert_rhs_close(Ep, Eo, 1e-10, f"PEC batch problem {p}")
    assert o.fem.pec.sum() == 0 and D3MOracle.from_problem(pp[1]).fem.pec.sum() > 0
