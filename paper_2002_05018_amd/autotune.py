"""Launch-shape autotuner.

Times the factorisation and the solve of an actual handle under candidate
tunings (``d3m_set_tuning``) and keeps the fastest: parameters of the factor
schedule are scored by a whole factor + solve step (``s1_block`` also blocks
the forward sweep over the subdomain factors), those of the solve alone by
the solve.  The candidates are the launch shapes the schedules expose:

* ``s1_block``: tile columns of a subdomain matrix whose Schur updates beyond
  them are applied together (the depth of the blocked update, i.e. how many
  64x64 tile products one work-group accumulates per target tile);
* ``k_block``: the same depth for chains of pivot units of K in the
  elimination tree;
* ``lookahead_tasks``: how many off-critical update tasks an elimination step
  needs before they are moved to the second stream;
* ``side_early``: whether those start right after the step's panels or only
  after its critical updates;
* ``k_fuse``: whether the updates of the next level's columns of K get their
  own launch or are applied inside that level's pivot and panel launches;
* ``panel_rows``: rows of a panel tile per work-group (64, or 16 with four
  work-groups per tile);
* ``k_overlap``: the off-critical updates of K on one side stream behind the
  previous step, or on two side streams with per-column waits;
* ``solve_cols``: right-hand sides per work-group of the solve sweeps
  (16 or 32 columns of the MFMA tile);
* ``solve_seq``: the subdomain sweeps of the solve as one launch per
  direction (a work-group per subdomain runs its tile columns in order) or
  one launch per tile column;
* ``solve_narrow``: below how many update tasks a sweep step takes 16
  right-hand sides per work-group (more, shorter work-groups).

The search is coordinate-wise in the order of ``space``: each parameter is
timed over its values with the others held at their current best, then
fixed.  Results can be kept in a JSON file keyed by the problem's shape.
"""
from __future__ import annotations

import json
import os
import time

__all__ = ["DEFAULT_SPACE", "signature", "autotune"]

DEFAULT_SPACE = {
    "s1_block": (2, 1, 4),
    "k_block": (2, 1, 4, 8),
    "lookahead_tasks": (512, 128, 2048),
    "side_early": (0, 1),
    "k_fuse": (0, 1),
    "panel_rows": (64, 16),
    "k_overlap": (0, 1),
    "solve_seq": (0, 1),
    "solve_narrow": (0, 1024, 4096),
    "solve_cols": (32, 16),
}
_PREC = {0: "fp64", 1: "fp32_ir", "fp64": "fp64", "fp32_ir": "fp32_ir"}
# parameters that change the factorisation schedule (the rest only the solve)
_FACTOR_KEYS = ("s1_block", "k_block", "lookahead_tasks", "side_early", "k_fuse", "panel_rows", "k_overlap")


def signature(solver, nrhs, precision) -> str:
    """Key of a tuning result: problem shape, right-hand sides, precision and device."""
    import torch
    i = solver.info
    if torch.cuda.is_available():  # architecture and compute units (the marketing name varies by runtime)
        prop = torch.cuda.get_device_properties(0)
        dev = f"{prop.gcnArchName.split(':')[0]}/{prop.multi_processor_count}"
    else:
        dev = "none"
    key = {"n_edges": i["n_edges"], "n_subdomains": i["n_subdomains"], "n_blocks": i["n_blocks"],
           "n_lm": i["n_lm"], "n_problems": i["n_problems"], "nrhs": int(nrhs),
           "precision": _PREC.get(precision, str(precision)), "device": dev}
    if i.get("s1_order", 0):  # another row order of step 1: another schedule
        key["s1_order"] = int(i["s1_order"])
    return json.dumps(key, sort_keys=True)


def _time(fn, repeats):
    import torch
    fn()  # warm-up (and graph capture when the handle uses graphs)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def autotune(solver, rhs, precision="fp64", space=None, repeats=2, cache=None, log=None):
    """Tune ``solver`` for right-hand sides ``rhs`` (device tensor [nrhs, n_edges]).

    Returns ``{"tuning": {...}, "trials": [...], "cached": bool}`` and leaves
    the best tuning applied (the factors are invalidated; factor again).
    ``cache``: optional JSON file path; a stored result for the same
    signature is applied without timing, a new one is written back.
    """
    import torch
    space = dict(DEFAULT_SPACE if space is None else space)
    nrhs = int(rhs.shape[0])
    if nrhs <= 16:  # one column block covers every right-hand side
        space.pop("solve_cols", None)
        space.pop("solve_narrow", None)
    key = signature(solver, nrhs, precision)
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            store = json.load(fh)
        if key in store:
            solver.set_tuning(**store[key])
            return {"tuning": dict(store[key]), "trials": [], "cached": True}
    out = torch.empty_like(rhs)

    def run_factor():
        solver.factor(precision)

    def run_step():
        solver.factor(precision)
        solver.solve(rhs, out=out)

    def run_solve():
        solver.solve(rhs, out=out)

    def fkey(c):
        return tuple(c.get(k) for k in _FACTOR_KEYS)

    best = solver.tuning()
    trials = []
    factored_with = None  # factor-side tuning of the factors in place
    for name, values in space.items():
        scores = {}
        for v in values:
            cand = dict(best, **{name: v})
            solver.set_tuning(**cand)
            if name in _FACTOR_KEYS:
                t = _time(run_step, repeats)
                factored_with = fkey(cand)
            else:
                if factored_with != fkey(cand):
                    run_factor()
                    factored_with = fkey(cand)
                t = _time(run_solve, repeats)
            scores[v] = t
            trials.append({"param": name, "value": v, "seconds": t})
            if log:
                log(f"autotune {name}={v}: {t * 1e3:.2f} ms")
        best[name] = min(scores, key=scores.get)
    solver.set_tuning(**best)
    if cache:
        store[key] = best
        try:
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as fh:
                json.dump(store, fh, indent=1, sort_keys=True)
        except OSError:
            pass  # a read-only cache location still serves stored entries
    return {"tuning": best, "trials": trials, "cached": False}
