"""Comparison helpers shared by the GPU parity tests (no method arithmetic).

Every check is per right-hand side and element-wise: for each row r (one
right-hand side) the largest entry-wise difference divided by the largest
entry of the reference row, so one bad column or one bad block cannot hide
under a norm taken over everything.
"""
import numpy as np


def rhs_max_rel(got, want, scale=None):
    """max_i |got[r, i] - want[r, i]| / max_i |want[r, i]| for every row r.

    ``scale`` (optional, [nrhs]) replaces the denominator, e.g. the maximum
    of the full reference vector when only sampled entries are compared."""
    got = np.atleast_2d(np.asarray(got))
    want = np.atleast_2d(np.asarray(want))
    assert got.shape == want.shape, (got.shape, want.shape)
    den = np.abs(want).max(axis=1) if scale is None else np.asarray(scale, dtype=np.float64)
    num = np.abs(got - want).max(axis=1)
    return num / np.maximum(den, np.finfo(np.float64).tiny)


def assert_rhs_close(got, want, tol, what="", scale=None):
    err = rhs_max_rel(got, want, scale)
    bad = np.nonzero(~(err <= tol))[0]
    assert bad.size == 0, f"{what}: right-hand sides {bad.tolist()} exceed {tol:g}: {err[bad].tolist()}"
    return err


def matrix_max_rel(got, want):
    """max |got - want| / max |want| over all entries of one matrix."""
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (got.shape, want.shape)
    return float(np.abs(got - want).max() / max(np.abs(want).max(), np.finfo(np.float64).tiny))


def host_residual(S, E, f):
    """||f - S E||_inf / ||f||_inf per right-hand side (host, FP64)."""
    E = np.atleast_2d(E)
    f = np.atleast_2d(f)
    r = (S @ E.T).T - f
    return np.abs(r).max(axis=1) / np.abs(f).max(axis=1)


def factor_as_benchmarked(s, nrhs, precision):
    """Apply the entry of the committed tuning table that bench.py applies to
    this problem (none: the defaults), then factor."""
    import json
    import os

    import paper_2002_05018_amd as pkg
    from paper_2002_05018_amd.autotune import signature
    with open(os.path.join(os.path.dirname(pkg.__file__), "tuning_mi355x.json")) as fh:
        table = json.load(fh)
    entry = table.get(signature(s, nrhs, precision))
    print(f"[parity] {precision} tuning {entry}", flush=True)
    if entry:
        s.set_tuning(**entry)
    s.factor(precision)
    return entry


def load_fixture(cfg, prefix=""):
    """Oracle values at sampled unknowns written by
    tests/golden/make_fullsize_fixtures.py (no pickled objects)."""
    import os

    import pytest
    name = "fullsize_pec.npz" if cfg == "pec" else f"fullsize_config{cfg}.npz"
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    if not os.path.exists(path):
        pytest.skip(f"oracle fixture {os.path.basename(path)} not written yet "
                    "(tests/golden/make_fullsize_fixtures.py)")
    with np.load(path, allow_pickle=False) as z:
        if prefix:
            return {k[len(prefix):]: z[k] for k in z.files if k.startswith(prefix)}
        return {k: z[k] for k in z.files}
