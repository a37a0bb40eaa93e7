"""The library's Bunch-Kaufman kernels, called directly (d3m_debug_bk).

Restricted Bunch-Kaufman pivoting of a diagonal block (Section II, the first
line of Algorithm 1; pivot test of Bunch & Kaufman 1977 with alpha =
(1 + sqrt 17)/8, |z| = |Re z| + |Im z|, no delayed pivots).  Every kernel
variant the factorisation can take is run:
  * the register kernel (blocks of at most 64 rows: every tile of step 1 and
    every pivot unit of step 5 with the default scope),
  * the general kernel with the block in LDS (whole blocks of K of 65 to
    ~140 rows, pivot scope 1),
  * the general kernel with the block in global memory (larger blocks),
in FP64 and with FP32 storage (pivot search, D and D^{-1} in FP64).

Checks: the hand-derived cases of tests/golden/bk_hand_cases.json exactly
(pivot kinds, permutation, D, L, D^{-1}); random blocks of 8 to 208 rows with
the oracle's decisions (same permutation and 1x1/2x2 sequence: values are
continuous, so no magnitude ties) and its L and D, the reconstruction
P L D L^T P^T = A, and TT = L^{-1} P^T; a zero column reported as
D3M_ESINGULAR at the right column.
"""
import json
import os

import numpy as np
import pytest

from oracle.bk import SingularBlock, bk_ldlt
from parity import matrix_max_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_CASES = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "bk_hand_cases.json")))["cases"]


def _c(m):
    a = np.asarray(m, dtype=float)
    return a[..., 0] + 1j * a[..., 1]


def _run(blocks, precision="fp64", variant=0):
    from paper_2002_05018_amd._lib import debug_bk
    print(f"[gpu bk] n={blocks.shape[-1]} count={blocks.shape[0]} {precision} variant {variant}", flush=True)
    return debug_bk(blocks, precision=precision, variant=variant)


def _kinds(pivots, n):
    k = np.zeros(n, np.int32)
    for s, size, _ in pivots:
        if size == 2:
            k[s], k[s + 1] = 1, -1
    return k


def _dense_d(out, q):
    n = out["d"].shape[1]
    D = np.diag(out["d"][q]).astype(np.complex128)
    for i in range(n - 1):
        if out["kind"][q, i] == 1:
            D[i, i + 1] = D[i + 1, i] = out["doff"][q, i]
    return D


def _dense_dinv(out, q):
    n = out["d"].shape[1]
    Di = np.diag(out["dinv"][q]).astype(np.complex128)
    for i in range(n - 1):
        if out["kind"][q, i] == 1:
            Di[i, i + 1] = Di[i + 1, i] = out["dinvoff"][q, i]
    return Di


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("case", _CASES, ids=[c["name"] for c in _CASES])
def test_hand_derived_cases(case, variant, precision):
    A = _c(case["A"])
    rc, out = _run(A[None], precision, variant)
    if "singular_column" in case:
        assert rc == -2 and out["singular"][0] == case["singular_column"] + 1
        return
    assert rc == 0
    n = A.shape[0]
    tol = 1e-14 if precision == "fp64" else 2e-7
    assert list(out["perm"][0]) == case["perm"]
    want_kind = np.zeros(n, np.int32)
    for k, size, _ in case["pivots"]:
        if size == 2:
            want_kind[k], want_kind[k + 1] = 1, -1
    assert list(out["kind"][0]) == list(want_kind)
    np.testing.assert_allclose(_dense_d(out, 0), _c(case["D"]), rtol=0, atol=tol)
    np.testing.assert_allclose(out["L"][0], _c(case["L"]), rtol=0, atol=tol)
    if "dinv" in case:
        np.testing.assert_allclose(_dense_dinv(out, 0), _c(case["dinv"]), rtol=0, atol=tol)


def _random_blocks(rng, n, count, kind):
    out = np.empty((count, n, n), np.complex128)
    for q in range(count):
        X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        A = 0.5 * (X + X.T)
        if kind == "small_diagonal":  # many 2x2 pivots and interchanges
            A[np.diag_indices(n)] *= 0.02
        elif kind == "spread":  # magnitudes over four decades, symmetric scaling
            s = 10.0 ** rng.uniform(-2, 2, n)
            A = s[:, None] * A * s[None, :]
        out[q] = A
    return out


_SIZES = [(8, (0, 1, 2)), (40, (0, 1, 2)), (64, (0, 1, 2)), (65, (0, 2)), (100, (0, 2)), (136, (0, 2)),
          (208, (0,))]
_seen = {"two_by_two": 0, "interchange": 0}


@pytest.mark.parametrize("n,variants", _SIZES, ids=[str(n) for n, _ in _SIZES])
def test_random_blocks_match_oracle(n, variants):
    rng = np.random.default_rng(n)
    for kind in ("plain", "small_diagonal", "spread"):
        blocks = _random_blocks(rng, n, 5, kind)
        refs = [bk_ldlt(A) for A in blocks]
        for variant in variants:
            for precision in ("fp64", "fp32_ir"):
                if precision == "fp32_ir" and variant != variants[0]:
                    continue
                src = blocks if precision == "fp64" else blocks.astype(np.complex64).astype(np.complex128)
                rs = refs if precision == "fp64" else [bk_ldlt(A) for A in src]
                rc, out = _run(src, precision, variant)
                assert rc == 0
                tol = 1e-10 if precision == "fp64" else 1e-5
                for q, (A, f) in enumerate(zip(src, rs)):
                    label = f"n={n} {kind} block {q} variant {variant} {precision}"
                    assert list(out["perm"][q]) == list(f.perm), label
                    assert list(out["kind"][q]) == list(_kinds(f.pivots, n)), label
                    D = _dense_d(out, q)
                    assert matrix_max_rel(D, f.D) <= tol, label
                    assert matrix_max_rel(out["L"][q], f.L) <= tol, label
                    assert matrix_max_rel(_dense_dinv(out, q), f.dinv()) <= tol, label
                    P = np.eye(n)[:, out["perm"][q]]
                    rec = P @ out["L"][q] @ D @ out["L"][q].T @ P.T
                    assert matrix_max_rel(rec, A) <= (1e-12 if precision == "fp64" else 1e-5), label
                    # TT = L^{-1} P^T against the oracle's L inverted
                    tt_o = np.linalg.solve(f.L, np.eye(n)[:, f.perm].T)
                    assert matrix_max_rel(out["tt"][q], tt_o) <= (1e-10 if precision == "fp64" else 1e-5), label
                    _seen["two_by_two"] += int((out["kind"][q] == 1).sum())
                    _seen["interchange"] += int((out["perm"][q] != np.arange(n)).any())


def test_random_suite_reached_both_pivot_kinds():
    """The random suite above took 2x2 pivots and interchanges on the GPU."""
    if _seen["two_by_two"] == 0 and _seen["interchange"] == 0:
        for n, variants in _SIZES[:2]:
            test_random_blocks_match_oracle(n, variants)
    assert _seen["two_by_two"] > 50 and _seen["interchange"] > 10, _seen


@pytest.mark.parametrize("n", [64, 100, 208])
def test_zero_column_is_singular(n):
    """A diagonally dominant block takes every pivot in place, so a zero row
    and column at position 37 leave no pivot at step 37: D3M_ESINGULAR naming
    column 37 for that block, while the other block of the launch is factored
    normally."""
    rng = np.random.default_rng(7)
    good = _random_blocks(rng, n, 1, "plain")[0] + 4 * n * np.eye(n)
    bad = good.copy()
    bad[37, :] = 0
    bad[:, 37] = 0
    with pytest.raises(SingularBlock) as e:
        bk_ldlt(bad)
    assert e.value.column == 37
    for variant in ((0, 1, 2) if n == 64 else (0, 2)):
        rc, out = _run(np.stack([good, bad]), "fp64", variant)
        assert rc == -2
        assert list(out["singular"]) == [0, 38]
        assert list(out["perm"][0]) == list(range(n))
        rec = out["L"][0] @ _dense_d(out, 0) @ out["L"][0].T
        assert matrix_max_rel(rec, good) <= 1e-12


def test_singular_error_names_block_and_column():
    from paper_2002_05018_amd import D3MError
    from paper_2002_05018_amd._lib import _check, _lib
    A = np.zeros((1, 3, 3), np.complex128)
    A[0, 1, 1] = A[0, 2, 2] = 1.0
    rc, out = _run(A)
    assert rc == -2 and out["singular"][0] == 1
    with pytest.raises(D3MError, match="ESINGULAR.*block 0, column 0"):
        _check(rc)
    assert b"column 0" in _lib.d3m_last_error()
