"""AutoBatching definitions (oracle; test infrastructure only).

Section 3 of the paper: each system has a memory scaler in the units a model's memory scales
with -- ``n_atoms``, or ``n_atoms_x_density`` (atom count times number density); the largest
batch that fits is found by adding copies of a probe system until memory runs out; the
conservative maximum is the smallest (copies that fit) x (scaler) over the probes (Figure 2:
min(2 x 400, 9 x 80) = 720).  Fixed-length runs pack systems into as few bins of that capacity
as possible (1-D bin packing); variable-length runs keep a batch full from a stream of systems and
swap converged systems out for new ones.

These are the plain definitions: the optimum bin count by exhaustive search (tiny inputs only) and
a step-by-step simulation of the in-flight schedule.
"""
from __future__ import annotations

import itertools

import numpy as np


def memory_scaler(n_atoms: int, volume: float, scales_with: str) -> float:
    if scales_with == "n_atoms":
        return float(n_atoms)
    if scales_with == "n_atoms_x_density":
        return float(n_atoms) * float(n_atoms) / float(volume)
    raise ValueError(scales_with)


def max_memory_scaler(probes):
    """probes: list of (copies that fit, scaler of the probe system); conservative maximum."""
    return min(n * s for n, s in probes)


def copies_that_fit(fits, scaler: float, limit: int = 1 << 20) -> int:
    """Largest k with fits(k * scaler) true, found by adding one copy at a time until the first
    failure ("out of memory")."""
    k = 0
    while k < limit and fits((k + 1) * scaler):
        k += 1
    return k


def optimal_bin_count(sizes, capacity: float) -> int:
    """Minimum number of bins of the given capacity holding every item (exhaustive; tiny inputs)."""
    sizes = list(sizes)
    n = len(sizes)
    if any(s > capacity for s in sizes):
        raise ValueError("an item exceeds the capacity")
    for nb in range(1, n + 1):
        for assign in itertools.product(range(nb), repeat=n):
            load = np.zeros(nb)
            for s, b in zip(sizes, assign):
                load[b] += s
            if np.all(load <= capacity):
                return nb
    return n


def valid_packing(bins, sizes, capacity: float) -> bool:
    seen = sorted(i for b in bins for i in b)
    return seen == list(range(len(sizes))) and all(sum(sizes[i] for i in b) <= capacity for b in bins)


def inflight_schedule(scalers, steps_to_converge, capacity: float, check_every: int):
    """Simulate the in-flight batcher: fill from the stream in order while the next system fits,
    advance, and every ``check_every`` steps remove converged systems and refill.  Returns the
    list of (step, batch as a tuple of system indices) at every refill."""
    stream = list(range(len(scalers)))
    active, done, step, log = [], {}, 0, []
    progress = {}

    def refill():
        while stream and sum(scalers[i] for i in active) + scalers[stream[0]] <= capacity:
            i = stream.pop(0)
            active.append(i)
            progress[i] = 0

    refill()
    log.append((step, tuple(active)))
    while active:
        for _ in range(check_every):
            for i in active:
                progress[i] += 1
            step += 1
        finished = [i for i in active if progress[i] >= steps_to_converge[i]]
        for i in finished:
            active.remove(i)
            done[i] = step
        refill()
        log.append((step, tuple(active)))
    return log, done
