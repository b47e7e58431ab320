"""Autotuner for the batched Jacobi SVT kernel.

The kernel's main free parameter is the number of lanes G that hold one column
pair (the rows per lane follow from it); one value serves a whole batch: the
register-resident items' launch and, where their kernel takes it (4, 8 or 16
lanes), the warm-started items' launches.  For a set of slice shapes, each
feasible G is timed on synthetic problems of exactly those shape classes (random
data, the completion's default options, so the same kernels run as in the
batch; a fixed number of Jacobi sweeps so every candidate does the same work),
with the library's HIP-event timing of all Jacobi launches of a tick; the
fastest is cached per shape signature, and the table can be saved and loaded.
"""
import json
import os

import numpy as np

_CACHE = {}


def signature(shapes):
    """Shape classes that decide the kernel: (max(I1,I2), min(I1,I2)) per problem."""
    return tuple(sorted(set((max(s[0], s[1]), min(s[0], s[1])) for s in shapes)))


def load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            for k, v in json.load(f).items():
                _CACHE[k] = v


def save(path):
    if path:
        with open(path, "w") as f:
            json.dump(_CACHE, f, indent=1, sort_keys=True)


def tune(shapes, candidates=(4, 8, 16, 32, 64), sweeps=2, slices=8, seed=0):
    """Return (best_G, {G: ms per tick of the Jacobi launch}) for a batch whose
    problems have these (I1, I2, ...) shapes."""
    import torch
    from . import lt
    key = repr(signature(shapes))
    if key in _CACHE:
        c = _CACHE[key]
        return c["G"], {int(g): t for g, t in c["ms"].items()}
    rng = np.random.default_rng(seed)
    probs = []
    for (m, n) in signature(shapes):
        shape = (m, n, slices)
        M = rng.standard_normal(shape).astype(np.float32)
        params = lt.pga_params(mu0=1.0, nu=1.0, mu_bar=1.0, max_iter=64, fixed_mu=True,
                               jacobi_tol=1e-300, max_sweeps=sweeps)
        probs.append(lt.Problem(lt.to_device(M), lt.to_device(np.ones(shape, np.uint8), torch.uint8),
                                params, ("identity",)))
    timings = {}
    for G in candidates:
        try:
            b = lt.Batch(probs, use_graph=False, jacobi_lanes=G)
        except (lt.LtError, ValueError):
            continue                      # this G cannot hold some slice
        for p in probs:
            p.reset()
        b.step(1)                         # warm the kernel
        lt.profile_begin()
        b.step(2)
        prof, _ = lt.profile_end()
        b.close()
        timings[G] = prof["jacobi"][1] / max(prof["jacobi"][0], 1)
    if not timings:
        raise ValueError("no candidate G can hold these shapes")
    best = min(timings, key=timings.get)
    _CACHE[key] = {"G": best, "ms": {str(g): t for g, t in timings.items()}}
    return best, timings
