"""Synthetic batched-state generators (inputs only; no simulation arithmetic).

Layout produced here is the host-side, row-vector convention used throughout the project:

* ``pos``, ``vel``: ``(N, 3)`` float64, Cartesian, atoms of system ``s`` contiguous in
  ``[sys_offsets[s], sys_offsets[s+1])`` (atom-wise attributes concatenated, as the paper's
  batched state does, Section 3).
* ``cell``: ``(S, 3, 3)`` float64, row ``a`` is lattice vector ``a``; Cartesian = fractional @ cell
  (the ASE/pymatgen convention the paper interoperates with, Section 2).
* ``mass``: ``(N,)`` float64 (amu, or 1 in reduced units); ``species``: ``(N,)`` int32.

Units: Angstrom, eV, amu, fs, K for the argon/copper workloads; reduced units
(epsilon = sigma_small = m = k_B = 1) for the soft-sphere jamming workload.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Optional

import numpy as np

# Input-generation constants (used only to draw velocities of a given temperature).
# k_B in eV/K (CODATA 2018 exact value of k_B divided by the exact elementary charge).
_K_B_EV = 8.617333262145179e-5
# 1 eV/(Angstrom*amu) expressed in Angstrom/fs^2 (CODATA 2018 e and u).
_EV_PER_A_AMU_IN_A_FS2 = 0.009648533215665327

ARGON_MASS = 39.948
COPPER_MASS = 63.546


@dataclasses.dataclass
class PotentialSpec:
    """Pair potential parameters for a batch.

    ``kind`` is ``"lj"``, ``"morse"`` or ``"soft_sphere"``.  ``params[si, sj]`` holds
    LJ ``(epsilon, sigma, 0)``, Morse ``(D, alpha, r0)`` or soft-sphere ``(epsilon, sigma_ij, 0)``.
    ``cutoff`` is the pair cutoff r_c (soft sphere: the largest sigma_ij).  ``shift_energy``
    subtracts phi(r_c) from every pair energy inside the cutoff.
    """

    kind: str
    params: np.ndarray  # (n_species, n_species, 3) float64
    cutoff: float
    shift_energy: bool = False

    @property
    def n_species(self) -> int:
        return int(self.params.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    pos: np.ndarray
    vel: np.ndarray
    mass: np.ndarray
    species: np.ndarray
    sys_offsets: np.ndarray
    cell: np.ndarray
    potential: PotentialSpec
    skin: float = 0.0
    dt: float = 1.0
    n_steps: int = 0
    pair_prec: str = "f64"  # "f32" or "f64"
    accel: float = _EV_PER_A_AMU_IN_A_FS2  # (force/mass) -> length/time^2 conversion
    kinetic_factor: float = 1.0 / _EV_PER_A_AMU_IN_A_FS2  # m v^2 -> energy
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_systems(self) -> int:
        return int(self.cell.shape[0])

    @property
    def system_idx(self) -> np.ndarray:
        counts = np.diff(self.sys_offsets)
        return np.repeat(np.arange(self.n_systems, dtype=np.int32), counts)

    def system(self, s: int) -> slice:
        return slice(int(self.sys_offsets[s]), int(self.sys_offsets[s + 1]))

    def subset(self, systems) -> "Workload":
        """The same workload restricted to the listed systems (copies)."""
        systems = list(systems)
        parts = [self.system(s) for s in systems]
        cat = lambda a: np.concatenate([a[p] for p in parts], axis=0)  # noqa: E731
        counts = [p.stop - p.start for p in parts]
        offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        return dataclasses.replace(
            self,
            name=f"{self.name}[{len(systems)} systems]",
            pos=cat(self.pos).copy(),
            vel=cat(self.vel).copy(),
            mass=cat(self.mass).copy(),
            species=cat(self.species).copy(),
            sys_offsets=offs,
            cell=self.cell[systems].copy(),
            extra=dict(self.extra),
        )


# ----------------------------------------------------------------------------- lattices


def fcc_cell(a: float):
    """Conventional FCC cell: 4-site basis (fractional) and cubic cell."""
    basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]], dtype=np.float64)
    return basis, np.eye(3) * a


def bcc_cell(a: float):
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0.5]], dtype=np.float64)
    return basis, np.eye(3) * a


def supercell(basis: np.ndarray, cell: np.ndarray, reps):
    """Replicate a basis ``reps = (n1, n2, n3)`` times.  Returns (pos (M,3), cell (3,3))."""
    n1, n2, n3 = (int(x) for x in reps)
    grid = np.array(list(itertools.product(range(n1), range(n2), range(n3))), dtype=np.float64)
    frac = (grid[:, None, :] + basis[None, :, :]).reshape(-1, 3) / np.array([n1, n2, n3])
    sc = cell * np.array([n1, n2, n3], dtype=np.float64)[:, None]
    return frac @ sc, sc


def most_cubic_supercell(n_basis: int, target_sites: int, max_rep: int = 24):
    """Repetitions (n1 <= n2 <= n3) whose site count is nearest ``target_sites``;
    ties go to the most cubic shape (smallest n3 - n1), then the smaller count."""
    best = None
    for n1 in range(1, max_rep + 1):
        for n2 in range(n1, max_rep + 1):
            for n3 in range(n2, max_rep + 1):
                m = n_basis * n1 * n2 * n3
                key = (abs(m - target_sites), n3 - n1, m)
                if best is None or key < best[0]:
                    best = (key, (n1, n2, n3))
    return best[1]


def maxwell_boltzmann(rng: np.random.Generator, mass: np.ndarray, temperature: float,
                      k_b: float = _K_B_EV, accel: float = _EV_PER_A_AMU_IN_A_FS2):
    """Per-component Gaussian velocities of variance k_B T accel / m, then the
    mass-weighted mean velocity is removed (zero net momentum).  No rescale to the exact T."""
    std = np.sqrt(k_b * temperature * accel / mass)
    v = rng.standard_normal((mass.shape[0], 3)) * std[:, None]
    p = (mass[:, None] * v).sum(0) / mass.sum()
    return v - p[None, :]


def concat_systems(name, systems, potential: PotentialSpec, **kw) -> Workload:
    """systems: list of dicts with pos, vel, mass, species, cell."""
    counts = [s["pos"].shape[0] for s in systems]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return Workload(
        name=name,
        pos=np.concatenate([s["pos"] for s in systems]).astype(np.float64),
        vel=np.concatenate([s["vel"] for s in systems]).astype(np.float64),
        mass=np.concatenate([s["mass"] for s in systems]).astype(np.float64),
        species=np.concatenate([s["species"] for s in systems]).astype(np.int32),
        sys_offsets=offs,
        cell=np.stack([s["cell"] for s in systems]).astype(np.float64),
        potential=potential,
        **kw,
    )


# ----------------------------------------------------------------------------- parameters

LJ_AR_SIGMA = 3.405
LJ_AR_EPS = 0.0104


def lj_argon_params(eps: float = LJ_AR_EPS, sigma: float = LJ_AR_SIGMA, cutoff: float = 2.5 * LJ_AR_SIGMA,
                    shift: bool = True) -> PotentialSpec:
    p = np.zeros((1, 1, 3))
    p[0, 0] = (eps, sigma, 0.0)
    return PotentialSpec("lj", p, float(cutoff), shift)


def morse_copper_params(D=0.3429, alpha=1.3588, r0=2.866, cutoff=7.0, shift=False) -> PotentialSpec:
    p = np.zeros((1, 1, 3))
    p[0, 0] = (D, alpha, r0)
    return PotentialSpec("morse", p, float(cutoff), shift)


def soft_sphere_params(diameters=(1.0, 1.4), eps=1.0) -> PotentialSpec:
    """Additive diameters: sigma_ij = (sigma_i + sigma_j) / 2."""
    d = np.asarray(diameters, dtype=np.float64)
    ns = d.shape[0]
    p = np.zeros((ns, ns, 3))
    for a in range(ns):
        for b in range(ns):
            p[a, b] = (eps, 0.5 * (d[a] + d[b]), 0.0)
    return PotentialSpec("soft_sphere", p, float(p[:, :, 1].max()), False)


# ----------------------------------------------------------------------------- workloads


def _argon_system(rng, reps, a, temperature, jitter=0.05):
    basis, cell0 = fcc_cell(a)
    pos, cell = supercell(basis, cell0, reps)
    pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    mass = np.full(pos.shape[0], ARGON_MASS)
    vel = maxwell_boltzmann(rng, mass, temperature)
    return dict(pos=pos, vel=vel, mass=mass, species=np.zeros(pos.shape[0], np.int32), cell=cell)


def argon_single(seed: int = 0) -> Workload:
    """One LJ argon system: FCC 4x4x4 (256 atoms), a = 5.26 A, jitter N(0, 0.05 A),
    Maxwell-Boltzmann 300 K, zero net momentum; FP64 pair math; dt = 1 fs, 100 steps,
    shifted energy at r_c = 2.5 sigma, list rebuilt every step (skin 0)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    sys0 = _argon_system(rng, (4, 4, 4), 5.26, 300.0)
    return concat_systems("argon_256_fp64", [sys0], lj_argon_params(), skin=0.0, dt=1.0, n_steps=100,
                          pair_prec="f64")


def argon_batch(n_systems: int = 64, reps=(6, 6, 6), seed: int = 1, n_steps: int = 1000,
                name: str = "argon_64x864") -> Workload:
    """Uniform batch of LJ argon systems (864 atoms each by default): lattice scale
    U[0.97, 1.03] x 5.26 A, temperature U[50, 300] K, jitter N(0, 0.05 A); FP32 pair math,
    FP64 integration, dt = 2 fs, skin 0.3 A."""
    children = np.random.SeedSequence(seed).spawn(n_systems)
    systems = []
    for ss in children:
        rng = np.random.default_rng(ss)
        scale = rng.uniform(0.97, 1.03)
        temp = rng.uniform(50.0, 300.0)
        systems.append(_argon_system(rng, reps, 5.26 * scale, temp))
    return concat_systems(name, systems, lj_argon_params(), skin=0.3, dt=2.0, n_steps=n_steps,
                          pair_prec="f32")


def argon_adjoint_batch(n_systems: int = 16, seed: int = 3, n_steps: int = 500) -> Workload:
    """Differentiable-trajectory batch: 16 argon systems as the 864-atom batch (seed 3),
    500 NVE steps at dt = 2 fs, checkpoint every 50 steps; RDF loss with 200 bins to 10 A,
    Gaussian smearing s = 0.05 A (standard deviation)."""
    w = argon_batch(n_systems, seed=seed, n_steps=n_steps, name="argon_adjoint_16x864")
    w.extra.update(dict(checkpoint_every=50, rdf_bins=200, rdf_rmax=10.0, rdf_sigma=0.05, target_scale=1.05))
    return w


def copper_uneven_batch(n_systems: int = 512, seed: int = 2, min_sites: int = 32, max_sites: int = 2048) -> Workload:
    """Uneven Morse copper batch: FCC (a = 3.61) or BCC (a = 2.87) with p = 1/2; site count
    M ~ U{min..max} realised as the most-cubic supercell with the nearest site count; vacancy
    fraction U[0, 0.05]; random symmetric strain U[-0.05, 0.05] on the six independent components,
    cell = cell0 (I + e); positions strained with the cell, plus N(0, 0.1 A) noise; zero velocities."""
    children = np.random.SeedSequence(seed).spawn(n_systems)
    systems = []
    for ss in children:
        rng = np.random.default_rng(ss)
        if rng.random() < 0.5:
            basis, cell0 = fcc_cell(3.61)
        else:
            basis, cell0 = bcc_cell(2.87)
        m = int(rng.integers(min_sites, max_sites + 1))
        reps = most_cubic_supercell(basis.shape[0], m)
        pos, cell = supercell(basis, cell0, reps)
        vac = rng.uniform(0.0, 0.05)
        n_remove = int(np.floor(vac * pos.shape[0]))
        if n_remove > 0:
            keep = np.sort(rng.permutation(pos.shape[0])[n_remove:])
            pos = pos[keep]
        e6 = rng.uniform(-0.05, 0.05, size=6)
        e = np.array([[e6[0], e6[3], e6[4]], [e6[3], e6[1], e6[5]], [e6[4], e6[5], e6[2]]])
        deform = np.eye(3) + e
        pos = pos @ deform + rng.normal(0.0, 0.1, size=pos.shape)
        cell = cell @ deform
        n = pos.shape[0]
        systems.append(dict(pos=pos, vel=np.zeros((n, 3)), mass=np.full(n, COPPER_MASS),
                            species=np.zeros(n, np.int32), cell=cell))
    w = concat_systems(f"copper_uneven_{n_systems}", systems, morse_copper_params(), skin=0.3, dt=0.1,
                       pair_prec="f32", accel=1.0, kinetic_factor=1.0)
    w.extra.update(dict(fire=dict(dt_start=0.1, dt_max=1.0, alpha_start=0.1, f_inc=1.1, f_dec=0.5, f_alpha=0.99,
                                  n_min=5, fmax=0.01, relax_cell=True, max_iter=100000)))
    return w


def soft_sphere_jamming_batch(n_systems: int = 8, n_atoms: int = 32000, seed: int = 4,
                              packing_fraction: float = 0.64) -> Workload:
    """Binary soft-sphere jamming batch (reduced units): 50:50 mixture, diameters 1.0 and 1.4,
    species randomly permuted, cubic cell at the given packing fraction, uniform random positions."""
    diam = np.array([1.0, 1.4])
    half = n_atoms // 2
    v_spheres = (np.pi / 6.0) * (half * diam[0] ** 3 + (n_atoms - half) * diam[1] ** 3)
    L = (v_spheres / packing_fraction) ** (1.0 / 3.0)
    children = np.random.SeedSequence(seed).spawn(n_systems)
    systems = []
    for ss in children:
        rng = np.random.default_rng(ss)
        species = np.concatenate([np.zeros(half, np.int32), np.ones(n_atoms - half, np.int32)])
        species = species[rng.permutation(n_atoms)]
        pos = rng.uniform(0.0, L, size=(n_atoms, 3))
        systems.append(dict(pos=pos, vel=np.zeros((n_atoms, 3)), mass=np.ones(n_atoms), species=species,
                            cell=np.eye(3) * L))
    w = concat_systems(f"soft_sphere_{n_systems}x{n_atoms}", systems, soft_sphere_params(diam), skin=0.2,
                       dt=0.01, n_steps=2000, pair_prec="f32", accel=1.0, kinetic_factor=1.0)
    w.extra.update(dict(fire=dict(dt_start=0.01, dt_max=0.1, alpha_start=0.1, f_inc=1.1, f_dec=0.5, f_alpha=0.99,
                                  n_min=5, fmax=1e-6, relax_cell=False, max_iter=100000),
                        nve_temperature=1e-4))
    return w


def random_small_batch(seed: int, n_systems: int = 3, n_range=(2, 40), kind: str = "lj",
                       triclinic: bool = True, density: Optional[float] = None, n_species: int = 1,
                       pair_prec: str = "f64", skin: float = 0.0, unwrap_spread: float = 0.0,
                       jitter: float = 0.2) -> Workload:
    """Small random periodic systems for parity tests: random triclinic cells (possibly narrower
    than the cutoff, so several images of one pair are in range), positions on randomly occupied
    sites of a jittered grid (``jitter`` in grid spacings), optional
    displacement of whole atoms by lattice vectors (``unwrap_spread``: positions not wrapped)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    if kind == "lj":
        sig = 1.0 + 0.2 * np.arange(n_species)
        p = np.zeros((n_species, n_species, 3))
        for a in range(n_species):
            for b in range(n_species):
                p[a, b] = (1.0 + 0.1 * (a + b), 0.5 * (sig[a] + sig[b]), 0.0)
        pot = PotentialSpec("lj", p, 2.5, True)
        dens = density or 0.8
    elif kind == "morse":
        p = np.zeros((n_species, n_species, 3))
        for a in range(n_species):
            for b in range(n_species):
                p[a, b] = (0.3 + 0.05 * (a + b), 1.4, 1.1 + 0.05 * (a + b))
        pot = PotentialSpec("morse", p, 2.6, False)
        dens = density or 0.8
    elif kind == "soft_sphere":
        pot = soft_sphere_params(1.0 + 0.4 * np.arange(n_species) / max(n_species - 1, 1))
        if n_species == 1:
            pot = soft_sphere_params([1.0])
        dens = density or 1.2
    else:
        raise ValueError(kind)
    systems = []
    for _ in range(n_systems):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        vol = n / dens
        base = np.eye(3) * vol ** (1.0 / 3.0)
        if triclinic:
            tilt = rng.uniform(-0.3, 0.3, size=(3, 3))
            tilt[np.diag_indices(3)] = rng.uniform(-0.2, 0.2, size=3)
            cell = base @ (np.eye(3) + tilt)
        else:
            cell = base
        # occupied sites of a jittered m^3 grid: random, but no two atoms closer than
        # (1 - 2 jitter) grid spacings (in fractional terms)
        m = int(np.ceil(n ** (1.0 / 3.0) - 1e-9))
        sites = rng.permutation(m ** 3)[:n]
        grid = np.stack([sites // (m * m), (sites // m) % m, sites % m], axis=1).astype(np.float64)
        frac = (grid + 0.5 + rng.uniform(-jitter, jitter, size=(n, 3))) / m
        pos = frac @ cell
        if unwrap_spread > 0:
            k = rng.integers(-int(unwrap_spread), int(unwrap_spread) + 1, size=(n, 3))
            pos = pos + k @ cell
        mass = rng.uniform(0.5, 2.0, size=n)
        vel = rng.normal(0.0, 0.05, size=(n, 3))
        species = rng.integers(0, n_species, size=n).astype(np.int32)
        systems.append(dict(pos=pos, vel=vel, mass=mass, species=species, cell=cell))
    return concat_systems(f"random_{kind}_{seed}", systems, pot, skin=skin, dt=0.002, n_steps=10,
                          pair_prec=pair_prec, accel=1.0, kinetic_factor=1.0)


def narrow_triclinic_batch(seed: int, n_systems: int = 3, n_range=(2100, 2600), narrow: float = 4.2,
                           density: float = 0.85, tilt: float = 0.25, unwrap_spread: int = 2,
                           empty_first: bool = False) -> Workload:
    """Large random LJ systems (reduced units, cutoff 2.5) in sheared cells that are narrow along the
    first lattice direction (perpendicular width near ``narrow``, below twice a list radius of 2.8,
    so several images of one pair are in range) and wide along the other two; uniform random
    fractional positions, a third of the atoms displaced by whole lattice vectors up to
    ``unwrap_spread`` (positions not wrapped).  ``empty_first`` prepends a system with no atoms."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    p = np.zeros((1, 1, 3))
    p[0, 0] = (1.0, 1.0, 0.0)
    pot = PotentialSpec("lj", p, 2.5, True)
    systems = []
    if empty_first:
        systems.append(dict(pos=np.zeros((0, 3)), vel=np.zeros((0, 3)), mass=np.zeros(0),
                            species=np.zeros(0, np.int32), cell=np.diag([narrow, 20.0, 20.0])))
    for _ in range(n_systems):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        side = np.sqrt(n / (density * narrow))
        shear = np.eye(3)
        shear[np.triu_indices(3, 1)] = rng.uniform(-tilt, tilt, size=3)
        shear[np.tril_indices(3, -1)] = rng.uniform(-0.5 * tilt, 0.5 * tilt, size=3)
        cell = np.diag([narrow, side, side]) @ shear
        frac = rng.uniform(0.0, 1.0, size=(n, 3))
        pos = frac @ cell
        moved = rng.random(n) < 1.0 / 3.0
        k = rng.integers(-unwrap_spread, unwrap_spread + 1, size=(n, 3))
        pos[moved] += k[moved] @ cell
        systems.append(dict(pos=pos, vel=np.zeros((n, 3)), mass=np.ones(n), species=np.zeros(n, np.int32),
                            cell=cell))
    return concat_systems(f"narrow_triclinic_{seed}", systems, pot, skin=0.3, dt=0.002, n_steps=10,
                          pair_prec="f64", accel=1.0, kinetic_factor=1.0)


def insert_empty_systems(w: Workload, at) -> Workload:
    """The workload with a system of no atoms inserted before each listed system index (``at``
    refers to the original numbering; ``len(systems)`` appends at the end).  The empty systems get
    the cell of the system they precede (or of the last one)."""
    at = sorted(int(a) for a in at)
    counts = list(np.diff(w.sys_offsets))
    cells = list(w.cell)
    new_counts, new_cells = [], []
    for s in range(w.n_systems + 1):
        for a in at:
            if a == s:
                new_counts.append(0)
                new_cells.append(cells[min(s, w.n_systems - 1)])
        if s < w.n_systems:
            new_counts.append(counts[s])
            new_cells.append(cells[s])
    offs = np.concatenate([[0], np.cumsum(new_counts)]).astype(np.int64)
    return dataclasses.replace(w, name=f"{w.name}+{len(at)} empty", sys_offsets=offs,
                               cell=np.stack(new_cells).astype(np.float64), extra=dict(w.extra))
