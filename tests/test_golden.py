"""Hand-derived restricted Bunch-Kaufman decisions (tests/golden/bk_hand_cases.json).

The fixture's values were worked out by hand from the pivot test (Section
II, Algorithm 1, with the criteria of Bunch & Kaufman 1977): the 1x1 pivot
without interchange, the 1x1 interchange with the row of the largest
off-diagonal (adjacent and not), the 2x2 pivot with and without moving its
partner row, a complex-symmetric 2x2 inverse (plain transpose, no
conjugate), and a zero column.  The oracle must reproduce each one exactly
up to rounding.
"""
import json
import os

import numpy as np
import pytest

from oracle.bk import SingularBlock, bk_ldlt

_CASES = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "bk_hand_cases.json")))["cases"]


def _c(m):
    a = np.asarray(m, dtype=float)
    return a[..., 0] + 1j * a[..., 1]


@pytest.mark.parametrize("case", _CASES, ids=[c["name"] for c in _CASES])
def test_oracle_reproduces_hand_derived_pivoting(case):
    A = _c(case["A"])
    if "singular_column" in case:
        with pytest.raises(SingularBlock) as e:
            bk_ldlt(A)
        assert e.value.column == case["singular_column"]
        return
    f = bk_ldlt(A)
    assert [list(p) for p in f.pivots] == case["pivots"]
    assert list(f.perm) == case["perm"]
    np.testing.assert_allclose(f.D, _c(case["D"]), rtol=0, atol=1e-14)
    np.testing.assert_allclose(f.L, _c(case["L"]), rtol=0, atol=1e-14)
    if "dinv" in case:
        np.testing.assert_allclose(f.dinv(), _c(case["dinv"]), rtol=0, atol=1e-14)
    np.testing.assert_allclose(f.reconstruct(), A, rtol=0, atol=1e-13)
