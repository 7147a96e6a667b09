"""AutoBatching on the host (paper Section 3): memory scalers, maximum-batch estimation by
probing, bin packing for fixed-length runs and an in-flight batcher for variable-length runs.

The device work runs through the C ABI (one batch at a time); this module only decides which
systems form each batch.  For the classical potentials the memory of a batch is known exactly, so
``DeviceMemoryModel`` gives the probe a byte count instead of provoking an out-of-memory error;
the probing procedure itself is the paper's (add copies of a probe system until it no longer
fits; take the smallest resulting capacity over the probes).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Iterable, List, Sequence

import numpy as np


def memory_scaler(n_atoms: int, volume: float, scales_with: str = "n_atoms") -> float:
    """Units of memory of one system: its atom count, or atom count x number density."""
    if scales_with == "n_atoms":
        return float(n_atoms)
    if scales_with == "n_atoms_x_density":
        return float(n_atoms) * (float(n_atoms) / float(volume))
    raise ValueError(f"unknown memory scaling {scales_with!r}")


def estimate_max_scaler(fits: Callable[[int, int], bool], probe_systems: Sequence[int],
                        scalers: Sequence[float], limit: int = 1 << 20) -> float:
    """Conservative maximum memory scaler.  ``fits(system, copies)`` reports whether a batch of
    ``copies`` copies of ``system`` fits.  For each probe system copies are added one at a time
    until the first failure; the capacity is the smallest copies x scaler over the probes."""
    best = np.inf
    for s in probe_systems:
        k = 0
        while k < limit and fits(s, k + 1):
            k += 1
        if k == 0:
            raise RuntimeError(f"system {s} does not fit on its own")
        best = min(best, k * float(scalers[s]))
    return float(best)


def default_probes(scalers: Sequence[float]) -> List[int]:
    """The largest and the smallest system (the two probes of the paper's Figure 2)."""
    order = np.argsort(np.asarray(scalers), kind="stable")
    return sorted({int(order[-1]), int(order[0])}, key=lambda i: -scalers[i])


def bin_pack(scalers: Sequence[float], capacity: float) -> List[List[int]]:
    """First-fit decreasing 1-D bin packing: systems sorted by decreasing scaler go into the first
    bin with room.  Returns bins as lists of system indices (each bin sorted)."""
    order = sorted(range(len(scalers)), key=lambda i: (-scalers[i], i))
    bins: List[List[int]] = []
    load: List[float] = []
    for i in order:
        if scalers[i] > capacity:
            raise ValueError(f"system {i} (scaler {scalers[i]}) exceeds the capacity {capacity}")
        for b in range(len(bins)):
            if load[b] + scalers[i] <= capacity:
                bins[b].append(i)
                load[b] += scalers[i]
                break
        else:
            bins.append([i])
            load.append(scalers[i])
    return [sorted(b) for b in bins]


@dataclasses.dataclass
class InFlightBatcher:
    """Keeps a batch full from a stream of systems (in stream order) and swaps converged systems
    out: ``batch()`` is the current set; ``update(converged)`` removes the converged ones and
    refills while the next system fits."""

    scalers: Sequence[float]
    capacity: float
    stream: Iterable[int] = None

    def __post_init__(self):
        self._stream = list(range(len(self.scalers)) if self.stream is None else self.stream)
        self._active: List[int] = []
        self.completed: List[int] = []
        self._fill()

    def _fill(self):
        load = sum(self.scalers[i] for i in self._active)
        while self._stream and load + self.scalers[self._stream[0]] <= self.capacity:
            i = self._stream.pop(0)
            self._active.append(i)
            load += self.scalers[i]
        if not self._active and self._stream:
            raise ValueError(f"system {self._stream[0]} exceeds the capacity")

    def batch(self) -> List[int]:
        return list(self._active)

    def update(self, converged: Sequence[bool]) -> List[int]:
        """``converged[k]`` refers to ``batch()[k]``.  Returns the new batch."""
        keep = [i for i, c in zip(self._active, converged) if not c]
        self.completed += [i for i, c in zip(self._active, converged) if c]
        self._active = keep
        self._fill()
        return self.batch()

    @property
    def done(self) -> bool:
        return not self._active and not self._stream


@dataclasses.dataclass
class DeviceMemoryModel:
    """Bytes a batch needs on the device for the NVE / FIRE entry points (positions, velocities,
    forces, masses, species, system index, list rows and reference positions, workspace)."""

    max_nbr: int
    budget_bytes: int
    force_bytes: int = 4

    def bytes(self, n_atoms: int, n_systems: int) -> int:
        per_atom = 24 + 24 + 3 * self.force_bytes + 8 + 4 + 4 + 4 * self.max_nbr + 4 + 24 + 24 + 40
        per_system = 8 + 72 + 72 + 200
        return n_atoms * per_atom + n_systems * per_system

    def fits(self, n_atoms: int, n_systems: int) -> bool:
        return self.bytes(n_atoms, n_systems) <= self.budget_bytes
