"""Writes the oracle's solutions of the full-size workloads at sampled
unknowns: tests/golden/fullsize_config{2,4,5}.npz, fullsize_config3.npz and
fullsize_pec.npz (the PEC-plate workload: plane waves and point dipoles).

Imports only ``oracle`` and ``workloads``: every stored value is the CPU
oracle's (the seven steps of Section II in complex128, sparse LU per
subdomain, Algorithm 1 on K).  Run from the repository root:

    python tests/golden/make_fullsize_fixtures.py 2 4 5 3 pec

Each file holds, for one workload (one problem of the batch for config 3,
keys prefixed ``p<index>_``):
  edges      int64 [ns]          sampled global edges (half of them edges
                                 shared by two or more subdomains)
  E          complex128 [nrhs, ns] oracle E at those edges
  E_inf      float64 [nrhs]      max over all edges of |E| per right-hand side
  lms        int64 [nl]          sampled multipliers (global LM order)
  lam        complex128 [nrhs, nl] oracle lambda there
  lam_inf    float64 [nrhs]      max over all multipliers of |lambda|
  residual   float64 [nrhs]      ||S E - f||_inf / ||f||_inf of the oracle
                                 solution (oracle S and f; on the unknowns,
                                 i.e. without PEC edges)
  f          complex128 [nrhs, ns] oracle plane-wave load at the sampled edges
and the oracle's phase timings on the machine that wrote it (seconds).  For
the dielectric-sphere workload (receivers and learnable tetrahedra) also
  grad_tets  int64 [ng]          the finite-difference tetrahedra and a sample
                                 of the other learnable ones
  grad       float64 [ng]        dL/d eps_r there, L = sum_rhs sum_m
                                 |E(r_m)|^2 at the receivers, by the oracle's
                                 adjoint solve
  grad_max   float64             max |dL/d eps_r| over the learnable tetrahedra

The right-hand sides are the oracle's plane-wave loads for the workload's
directions and polarisations (Section II, second line of the BVP), followed
for the PEC workload by its point-dipole loads (the impressed current of the
first line).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.d3m import D3MOracle  # noqa: E402
from oracle.fem import probe_matrix  # noqa: E402

SAMPLES = {2: (4096, 2048), 4: (2048, 1024), 5: (4096, 2048), 3: (256, 128), "pec": (4096, 2048)}


def _sample(rng, o, n_edge, n_lm):
    dec = o.dec
    mult = np.array([len(s) for s in dec.sub_of_edge])  # 0 on PEC edges
    shared = np.nonzero(mult >= 2)[0]
    single = np.nonzero(mult == 1)[0]
    h = min(n_edge // 2, shared.size)
    e = np.concatenate([rng.choice(shared, h, replace=False),
                        rng.choice(single, min(n_edge - h, single.size), replace=False)])
    lm = rng.choice(dec.n_lm, min(n_lm, dec.n_lm), replace=False) if dec.n_lm else np.zeros(0, np.int64)
    return np.sort(e).astype(np.int64), np.sort(lm).astype(np.int64)


def solve_problem(prob, seed, n_edge, n_lm, log):
    t0 = time.perf_counter()
    o = D3MOracle.from_problem(prob)
    t1 = time.perf_counter()
    log(f"  setup {t1 - t0:.1f} s ({o.fem.topo.n_edges} edges, {o.dec.N} subdomains, {o.dec.n_lm} LMs)")
    o.factor()
    t2 = time.perf_counter()
    log(f"  factor {t2 - t1:.1f} s {o.timings}")
    f = o.fem.planewave_rhs(prob.dirs, prob.pols)
    if prob.dip_pos.shape[0]:
        f = np.concatenate([f, o.fem.dipole_rhs(prob.dip_pos, prob.dip_moment)])
    E = o.solve(f)
    t3 = time.perf_counter()
    log(f"  solve {t3 - t2:.1f} s")
    free = o.fem.free
    r = np.abs((o.fem.system() @ E[:, free].T).T - f[:, free]).max(axis=1) / np.abs(f[:, free]).max(axis=1)
    assert float(r.max()) == o.fem.relative_residual(E, f)
    log(f"  residual {r.max():.2e}")
    rng = np.random.default_rng(seed)
    e, lm = _sample(rng, o, n_edge, n_lm)
    tim = {k: float(v) for k, v in o.timings.items()}
    lam = o.lam.copy()  # the adjoint solve below replaces the oracle's lambda
    extra = {}
    if prob.receivers.shape[0] and prob.learnable.size:
        # gradient of L = sum_rhs sum_m |E(r_m)|^2 (receivers r_m) with respect
        # to eps_r by the oracle's adjoint: G = dL/dRe E + j dL/dIm E =
        # 2 sum_m P_m^T (P_m E) for the real probe rows P_m
        P = probe_matrix(o.fem.topo, prob.receivers).reshape(-1, o.fem.topo.n_edges)
        G = 2.0 * (P.T @ (P @ E.T)).T
        g, _ = o.adjoint(G, E)
        t = np.union1d(prob.fd_tets, rng.choice(prob.learnable, min(256, prob.learnable.size), replace=False))
        extra = {"grad_tets": t.astype(np.int64), "grad": g[t], "grad_max": np.array(np.abs(g[prob.learnable]).max())}
        log(f"  adjoint gradient: max |g| over learnable tets {extra['grad_max']:.3e}")
    out = {"edges": e, "E": E[:, e], "E_inf": np.abs(E).max(axis=1), "lms": lm,
           "lam": lam[:, lm], "lam_inf": np.abs(lam).max(axis=1) if lam.size else np.zeros(E.shape[0]),
           "residual": r, "f": f[:, e],
           "timing_names": np.array(sorted(tim)), "timing_s": np.array([tim[k] for k in sorted(tim)])}
    out.update(extra)
    return out


def main(cfgs):
    def log(m):
        print(m, flush=True)

    for cfg in cfgs:
        n_edge, n_lm = SAMPLES[cfg]
        path = os.path.join(HERE, "fullsize_pec.npz" if cfg == "pec" else f"fullsize_config{cfg}.npz")
        log(f"config {cfg} -> {path}")
        if cfg == "pec":
            data = solve_problem(W.make_pec_config(), 1006, n_edge, n_lm, log)
        elif cfg == 3:
            probs = W.make_batch_config()
            data = {}
            for p, prob in enumerate(probs):
                log(f" problem {p}: {prob.n}^3 hexes, boxes {prob.parts}")
                out = solve_problem(prob, 3000 + p, n_edge, n_lm, log)
                for k, v in out.items():
                    data[f"p{p}_{k}"] = v
            data["count"] = np.array(len(probs))
        else:
            data = solve_problem(W.make_config(cfg), 1000 + cfg, n_edge, n_lm, log)
        np.savez_compressed(path, **data)


if __name__ == "__main__":
    main([a if a == "pec" else int(a) for a in sys.argv[1:]] or [2, 4, 5, 3, "pec"])
