"""GPU parity of the HIP path against the CPU oracle (called through the C ABI).

Tolerances (FP64): the oracle and the library solve the same exact method
with different elimination orders and pivot sequences, so agreement is to
rounding amplified by the conditioning of the reduced system.  Every
comparison is element-wise: for fields and multipliers per right-hand side
(largest entry-wise difference over the largest entry of that right-hand
side), for matrices over all entries.  The domain matrices K_D^(d) (a unique
object, step 1) must agree to 1e-12; the multipliers and the field to 1e-10
(the exactness bar of the method against the undecomposed solve); the
factorisation of -K must reconstruct the oracle's K to 1e-12.  FP32 factors
with FP64 refinement must reach the 1e-10 relative residual and then agree
with the FP64 oracle to 1e-9.
"""
import math

import numpy as np
import pytest

import workloads as W
from parity import assert_rhs_close, matrix_max_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


CASES = {
    "cfg1": lambda: W.make_config(1),
    "cross_lines_2x2x2": lambda: W.make_problem(4, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi,
                                                nrhs=3, seed=1),
    "block_208_global_bk": lambda: W.make_problem(8, (2, 1, 1), eps=("uniform", 1, 4), k=2 * math.pi,
                                                  nrhs=2, seed=2),
    "single_subdomain": lambda: W.make_problem(3, (1, 1, 1), eps=("uniform", 1, 4), k=2 * math.pi,
                                               nrhs=2, seed=3),
    "uneven_1x3x2": lambda: W.make_problem(7, (1, 3, 2), eps=("uniform", 1, 4), k=5.0, nrhs=1, seed=4,
                                           cuts=[[0, 7], [0, 2, 3, 7], [0, 5, 7]]),
    "many_rhs_40": lambda: W.make_problem(4, (2, 2, 1), eps=("uniform", 1, 4), k=2 * math.pi,
                                          nrhs=40, seed=5),
}

_cache = {}


def _pair(name):
    if name not in _cache:
        from oracle.d3m import D3MOracle
        from paper_2002_05018_amd import Solver
        prob = CASES[name]()
        print(f"[gpu parity] case {name}: n={prob.n} parts={prob.parts} nrhs={prob.nrhs}", flush=True)
        s = Solver.from_problem(prob)
        o = D3MOracle.from_problem(prob).factor()
        f = s.rhs_planewave(prob.dirs, prob.pols)
        Eo = o.solve(f)
        _cache[name] = (prob, s, o, f, Eo, o.lam.copy())
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_field_multipliers_domain_matrices(name):
    prob, s, o, f, Eo, lamo = _pair(name)
    s.factor("fp64")
    E, info = s.solve(torch.from_numpy(f).cuda(), with_info=True)
    E = E.cpu().numpy()
    assert_rhs_close(E, Eo, 1e-10, "E")
    assert info["residual"] <= 1e-11
    # subdomain copies of shared edges agree to the rounding of lambda, on
    # both sides (step 7; continuity of eq. (1))
    scale = np.abs(Eo).max()
    assert o.copy_discrepancy <= 1e-10 * scale
    if o.dec.N > 1:
        assert 0.0 < info["copy_discrepancy"] <= 1e-10 * scale, info
    else:
        assert info["copy_discrepancy"] == 0.0
    if o.dec.n_lm:
        lam = s.export("lambda", prob.nrhs)
        assert_rhs_close(lam, lamo, 1e-10, "lambda")
        for d in range(o.dec.N):
            assert matrix_max_rel(s.export("kd", d), o.dm.KD[d]) <= 1e-12, d


@pytest.mark.parametrize("name,scope", [("cfg1", 0), ("cross_lines_2x2x2", 0), ("block_208_global_bk", 0),
                                        ("cfg1", 1), ("block_208_global_bk", 1)])
def test_factor_reconstructs_minus_K(name, scope):
    """P L D L^T P^T over the pivot units must equal -K (oracle) in the
    library's block order; scope 1 restricts pivots to whole blocks (the
    paper's Algorithm 1), scope 0 to pieces of at most 64 rows."""
    from paper_2002_05018_amd import Solver
    prob, _, o, f, Eo, lamo = _pair(name)
    s = Solver.from_problem(prob, pivot_scope=scope)
    s.factor("fp64")
    sizes, perm, d0, d1, L = s.export("kfactor")
    order = s.export("order")
    dec = o.dec
    if scope == 1:
        assert list(sizes) == [int(dec.block_start[b + 1] - dec.block_start[b]) for b in order]
    else:
        assert max(sizes) <= 64
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    n = off[-1]
    P = np.zeros((n, n))
    for j in range(len(sizes)):
        sj = slice(off[j], off[j + 1])
        P[off[j] + perm[sj], off[j] + np.arange(sizes[j])] = 1.0
    Lg = L.copy()
    for i in range(len(sizes)):
        si = slice(off[i], off[i + 1])
        for j in range(i):
            sj = slice(off[j], off[j + 1])
            Lg[si, sj] = P[si, si].T @ L[si, sj]  # L_ij = P_i^T Lhat_ij
    D = np.diag(d0) + np.diag(d1[:-1], -1) + np.diag(d1[:-1], 1)
    rec = P @ Lg @ D @ Lg.T @ P.T
    idx = np.concatenate([np.arange(dec.block_start[b], dec.block_start[b + 1]) for b in order])
    K = o.dm.assemble_dense()[np.ix_(idx, idx)]
    assert matrix_max_rel(rec, -K) <= 1e-12
    if scope == 1:
        # the same block order on the oracle's side: every block's pivot
        # decisions (permutation, 1x1/2x2 sequence) equal the oracle's
        from oracle.d3m import D3MOracle
        oo = D3MOracle.from_problem(prob, order=order).factor()
        two = swaps = 0
        for j in range(len(sizes)):
            sj = slice(off[j], off[j + 1])
            fj = oo.ldlt.diag[j]
            assert list(perm[sj]) == list(fj.perm), j
            first = [k for k, size, _ in fj.pivots if size == 2]
            assert sorted(np.nonzero(d1[sj][:-1])[0].tolist()) == first, j
            two += len(first)
            swaps += int(any(p != k for k, _, p in fj.pivots))
        print(f"[gpu parity] {name}: {two} 2x2 pivots, {swaps} blocks with interchanges", flush=True)
        assert two > 0 and swaps > 0
    E = s.solve(torch.from_numpy(f).cuda()).cpu().numpy()
    assert_rhs_close(E, Eo, 1e-10, "E")


@pytest.mark.parametrize("name", ["cfg1", "cross_lines_2x2x2", "uneven_1x3x2"])
def test_fp32_with_refinement(name):
    prob, s, o, f, Eo, lamo = _pair(name)
    s.factor("fp32_ir")
    E, info = s.solve(torch.from_numpy(f).cuda(), with_info=True)
    assert info["converged"] and info["residual"] <= 1e-10
    assert_rhs_close(E.cpu().numpy(), Eo, 1e-9, "E (FP32 factors + refinement)")


def test_host_buffers_match_device_buffers():
    prob, s, o, f, Eo, lamo = _pair("cfg1")
    s.factor("fp64")
    Eh = s.solve(torch.from_numpy(f)).numpy()
    Ed = s.solve(torch.from_numpy(f).cuda()).cpu().numpy()
    assert np.array_equal(Eh, Ed)


def test_repeatable_bitwise():
    prob, s, o, f, Eo, lamo = _pair("cross_lines_2x2x2")
    fd = torch.from_numpy(f).cuda()
    s.factor("fp64")
    E1 = s.solve(fd).cpu().numpy()
    s.factor("fp64")
    E2 = s.solve(fd).cpu().numpy()
    assert np.array_equal(E1, E2)


def test_adjoint_matches_oracle():
    prob, s, o, f, Eo, lamo = _pair("cross_lines_2x2x2")
    rng = np.random.default_rng(0)
    G = rng.standard_normal(Eo.shape) + 1j * rng.standard_normal(Eo.shape)
    s.factor("fp64")
    grad, w = s.adjoint(torch.from_numpy(G).cuda(), torch.from_numpy(Eo).cuda(), want_w=True)
    go, wo = o.adjoint(G, Eo)
    assert_rhs_close(w.cpu().numpy(), wo, 1e-10, "adjoint w")
    assert_rhs_close(grad.cpu().numpy(), go, 1e-10, "gradient")


def test_autograd_gradient_vs_finite_differences():
    from paper_2002_05018_amd import D3MSolve, Solver
    prob = W.make_problem(3, (2, 1, 1), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=2, seed=13)
    s = Solver.from_problem(prob)
    f = torch.from_numpy(s.rhs_planewave(prob.dirs, prob.pols)).cuda()
    rng = np.random.default_rng(1)
    pts = 0.5 + 0.3 * (rng.random((6, 3)) - 0.5)
    edges, coef = s.probe(pts)
    ed = torch.from_numpy(edges).cuda()
    cf = torch.from_numpy(coef).cuda().to(torch.complex128)

    def objective(eps):
        E = D3MSolve.apply(eps, s, f)
        v = (E[:, ed] [..., None] * cf[None]).sum(dim=2)  # [nrhs, m, 3]
        return (v.abs() ** 2).sum()

    eps = torch.tensor(prob.eps_r, dtype=torch.float64, requires_grad=True)
    L = objective(eps)
    L.backward()
    g = eps.grad.numpy()
    h = 1e-6
    for t in rng.choice(len(prob.eps_r), 6, replace=False):
        ep = prob.eps_r.copy(); ep[t] += h
        em = prob.eps_r.copy(); em[t] -= h
        with torch.no_grad():
            fd = (objective(torch.tensor(ep)).item() - objective(torch.tensor(em)).item()) / (2 * h)
        assert abs(fd - g[t]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max()), t


def test_autograd_backward_after_a_second_forward():
    """Two forwards on one handle (eps1, then eps2) and the backward of the
    first loss: the adjoint must use the factors of eps1 (the handle is
    refactored for it), so the gradient equals that of a lone forward at
    eps1, and differs from the one at eps2."""
    from paper_2002_05018_amd import D3MSolve, Solver
    prob = W.make_problem(3, (2, 1, 1), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=2, seed=14)
    s = Solver.from_problem(prob)
    f = torch.from_numpy(s.rhs_planewave(prob.dirs, prob.pols)).cuda()
    edges, coef = s.probe(np.array([[0.4, 0.45, 0.5], [0.6, 0.3, 0.55]]))
    ed = torch.from_numpy(edges).cuda()
    cf = torch.from_numpy(coef).cuda().to(torch.complex128)

    def objective(eps):
        E = D3MSolve.apply(eps, s, f)
        return ((E[:, ed][..., None] * cf[None]).sum(dim=2).abs() ** 2).sum()

    def grad_alone(e):
        x = torch.tensor(e, dtype=torch.float64, requires_grad=True)
        objective(x).backward()
        return x.grad.numpy().copy()

    e1 = prob.eps_r.copy()
    e2 = 1.3 * prob.eps_r
    g1, g2 = grad_alone(e1), grad_alone(e2)
    x1 = torch.tensor(e1, dtype=torch.float64, requires_grad=True)
    x2 = torch.tensor(e2, dtype=torch.float64, requires_grad=True)
    L1 = objective(x1)
    L2 = objective(x2)  # the handle now holds the factors of eps2
    L1.backward()
    assert np.array_equal(x1.grad.numpy(), g1)
    L2.backward()
    assert np.array_equal(x2.grad.numpy(), g2)
    assert np.abs(g1 - g2).max() > 1e-6 * np.abs(g1).max()


def test_growth_monitor_and_whole_block_fallback():
    """d3m_factor_growth reports max |L-hat_ij| of the factor of -K; with
    whole-block pivoting (Algorithm 1's scope) and the oracle's block order
    it equals the oracle's max over its L-hat blocks.  A growth limit below
    the measured value makes a pieces-scope factorisation fall back to the
    whole-block scope, which the handle then keeps; the solution still
    matches the oracle."""
    from oracle.d3m import D3MOracle
    from paper_2002_05018_amd import Solver
    # four subdomains of 4x4x8 hexes: blocks of about 110 rows (two pieces
    # each with the default scope) and off-diagonal blocks of K
    prob = W.make_problem(8, (2, 2, 1), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=2, seed=3)
    o = D3MOracle.from_problem(prob).factor()
    s1 = Solver.from_problem(prob, pivot_scope=1)
    f = s1.rhs_planewave(prob.dirs, prob.pols)
    Eo = o.solve(f)
    s1.factor("fp64")
    g_s1, g_k = s1.growth()
    oo = D3MOracle.from_problem(prob, order=s1.export("order")).factor()
    want = max(np.abs(W).max() for W in oo.ldlt.Lhat.values())
    print(f"[gpu parity] growth: step 1 {g_s1:.3e}, K {g_k:.3e} (oracle K {want:.3e})", flush=True)
    assert abs(g_k - want) <= 1e-10 * want
    assert 0.0 < g_s1 < np.inf
    s0 = Solver.from_problem(prob)
    s0.factor("fp64")
    assert s0.query()["pivot_scope"] == 0 and s0.query()["pivot_fallbacks"] == 0
    sf = Solver.from_problem(prob, growth_limit_log10=-6)
    sf.factor("fp64")
    info = sf.query()
    assert info["pivot_scope"] == 1 and info["pivot_fallbacks"] == 1, info
    E = sf.solve(torch.from_numpy(f).cuda()).cpu().numpy()
    assert_rhs_close(E, Eo, 1e-10, "E after the fallback")
    sf.factor("fp64")  # already whole blocks: no second fallback
    assert sf.query()["pivot_fallbacks"] == 1
    assert_rhs_close(sf.solve(torch.from_numpy(f).cuda()).cpu().numpy(), Eo, 1e-10, "E")
    sz, perm, d0, d1, L = sf.export("kfactor")
    assert list(sz) == [int(o.dec.block_start[b + 1] - o.dec.block_start[b]) for b in sf.export("order")]


def test_fp32_refinement_refines_only_unconverged_rhs():
    """A zero right-hand side is solved exactly by the first FP32 pass, so
    every later correction runs over the other right-hand sides only
    (gathered, corrected, written back): the field of the loaded ones equals
    the refinement run on them alone, the zero one stays exactly zero."""
    from paper_2002_05018_amd import Solver
    prob, s, o, f, Eo, lamo = _pair("cross_lines_2x2x2")
    s.factor("fp32_ir")
    f2 = np.concatenate([f[:1], np.zeros_like(f[:1]), f[1:]])
    E2, info2 = s.solve(torch.from_numpy(f2).cuda(), with_info=True)
    E1, info1 = s.solve(torch.from_numpy(f).cuda(), with_info=True)
    E2, E1 = E2.cpu().numpy(), E1.cpu().numpy()
    assert info2["converged"] and info2["residual"] <= 1e-10 and info2["iterations"] >= 1, info2
    assert not np.any(E2[1])
    assert_rhs_close(np.concatenate([E2[:1], E2[2:]]), E1, 1e-12, "refined subset vs all")
    assert_rhs_close(np.concatenate([E2[:1], E2[2:]]), Eo, 1e-9, "refined subset vs oracle")
