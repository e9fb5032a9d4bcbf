"""Autotuner for the launch shapes and the inner-solve policy of an ensemble.

It times candidate settings on the live ensemble, a step or two each, by
coordinate descent:
1. the CG initial guess: the previous increment, or its linear or quadratic
   extrapolation from the increments of the last steps;
2. the inner iteration policy of the mixed path (tolerance-driven CG, a fixed
   CG count that keeps every member's lanes busy, or a fixed-degree Chebyshev
   iteration after the step's first CG solve);
3. threads per block of the element-by-element launches;
4. CG iterations per host convergence check (the hipGraph chunk length);
5. co-resident blocks per CU of the cluster launches (64 and more member slots).

Every trial step is a complete, converged step of the simulation.  Only the
iteration path inside the outer FP64 tolerance depends on the choice.  The
winner is cached per problem shape in memory, and optionally in a JSON file.
"""
from __future__ import annotations

import json
import os
import time

# (inner_tol, inner_maxit, inner_method): method 0 CG, 1 Chebyshev of degree inner_maxit
INNER_POLICIES = [(0.1, 50, 0), (0.01, 60, 0), (1e-12, 12, 0), (1e-12, 16, 0), (1e-12, 20, 0),
                  (1e-12, 24, 0), (1e-12, 16, 1), (1e-12, 20, 1)]
PREDICTORS = [0, 1, 2]  # degree of the extrapolation of the previous increments
EBE_BLOCKS = [256, 128]
CHECK_EVERY = [8, 16, 4]
CHECK_EVERY_FP64 = [8, 4, 2]  # a plain FP64 PCG iteration is long: checking often costs little
CLUSTER_BLOCKS = [3, 2, 4]

_cache: dict = {}


def shape_key(mesh, prob, members_padded: int) -> str:
    return (f"ne{mesh.n_tets}-nn{mesh.n_nodes}-mb{members_padded}-ns{prob.n_springs}-"
            f"p{prob.precision}-d{getattr(prob, 'inner_dtype', 0)}")


def members_padded(n: int) -> int:
    """Member slots of an ensemble of n members (the library pads to a power
    of two up to 256, then to a multiple of 256)."""
    if n <= 1:
        return 1
    if n <= 256:
        p = 1
        while p < n:
            p *= 2
        return p
    return (n + 255) // 256 * 256


def trial_steps(prob, steps_per_trial: int = 1) -> int:
    """Steps an uncached tuning run takes: every candidate of a stage runs
    twice (palindromic order), the incumbent included; the mixed path adds
    one untimed step that makes the Chebyshev spectrum estimate."""
    n_pol = len(INNER_POLICIES) if prob.precision == 1 else 1
    n_cl = len(CLUSTER_BLOCKS) if 64 <= members_padded(prob.n_members) <= 256 else 1
    n_ce = len(CHECK_EVERY if prob.precision == 1 else CHECK_EVERY_FP64)
    stages = [len(PREDICTORS), n_pol, len(EBE_BLOCKS), n_ce, n_cl]
    return 2 * steps_per_trial * sum(n for n in stages if n > 1) + (1 if prob.precision == 1 else 0)


def _apply(ens, c):
    ens.set_tuning(c["ebe_block"], c["check_every"], 1, c["inner_maxit"], c["inner_tol"],
                   cluster_blocks=c["cluster_blocks"], inner_method=c.get("inner_method", 0),
                   predictor=c.get("predictor", 0))


def tune(ens, mesh, prob, steps_per_trial: int = 1, cache_file: str | None = None, log=None) -> dict:
    """Tune ``ens`` in place; returns the chosen settings and the trial times.

    The cost of a step drifts as the wave evolves, so each stage times its
    candidates in the order A B C ... C B A and scores each by its faster
    visit: a slow drift moves both visits of neighbours alike, and a single
    step made slow by one member's hard convergence does not decide."""
    st = ens.stats()
    key = shape_key(mesh, prob, st["members_padded"])
    if cache_file and os.path.exists(cache_file):
        try:
            with open(cache_file) as fh:
                _cache.update(json.load(fh))
        except (OSError, ValueError):
            pass
    if key in _cache:
        best = _cache[key]
        _apply(ens, best)
        return dict(best, cached=True)
    trials = []

    def stage(cands):
        if len(cands) < 2:
            return cands[0], None
        ms = [float("inf")] * len(cands)
        for i in list(range(len(cands))) + list(reversed(range(len(cands)))):
            _apply(ens, cands[i])
            t0 = time.perf_counter()
            ens.step(steps_per_trial)
            dt = (time.perf_counter() - t0) / steps_per_trial * 1e3
            ms[i] = min(ms[i], dt)
            trials.append(dict(cands[i], ms=dt))
            if log:
                log(f"autotune {cands[i]} -> {dt:.1f} ms/step")
        i = min(range(len(cands)), key=ms.__getitem__)
        return cands[i], ms[i]

    cur = dict(ebe_block=EBE_BLOCKS[0], check_every=CHECK_EVERY[0], cluster_blocks=CLUSTER_BLOCKS[0],
               inner_tol=prob.inner_tol, inner_maxit=prob.inner_maxit, inner_method=0, predictor=PREDICTORS[0])
    cur, best_ms = stage([dict(cur, predictor=k) for k in PREDICTORS])
    if prob.precision == 1:
        # the first Chebyshev step also estimates the top of the spectrum (a
        # cost shared by the next 32 steps): make it here, untimed
        cheb = [p for p in INNER_POLICIES if p[2] == 1]
        if cheb:
            _apply(ens, dict(cur, inner_tol=cheb[0][0], inner_maxit=cheb[0][1], inner_method=1))
            ens.step(1)
        cur, best_ms = stage([dict(cur, inner_tol=t, inner_maxit=m, inner_method=k) for t, m, k in INNER_POLICIES])
    cur, ms = stage([dict(cur, ebe_block=b) for b in EBE_BLOCKS])
    best_ms = ms if ms is not None else best_ms
    cur, ms = stage([dict(cur, check_every=c) for c in (CHECK_EVERY if prob.precision == 1 else CHECK_EVERY_FP64)])
    best_ms = ms if ms is not None else best_ms
    if 64 <= st["members_padded"] <= 256:  # the cluster path
        cur, ms = stage([dict(cur, cluster_blocks=b) for b in CLUSTER_BLOCKS])
        best_ms = ms if ms is not None else best_ms
    _apply(ens, cur)
    best = dict(cur, ms=best_ms)
    _cache[key] = best
    if cache_file:
        try:
            with open(cache_file, "w") as fh:
                json.dump(_cache, fh, indent=1)
        except OSError:
            pass
    return dict(best, cached=False, trials=trials)
