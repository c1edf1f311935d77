"""Seeded synthetic inputs for the truncated Lennard-Jones MD workloads.

This module produces *inputs only*: lattice and random positions, species
labels, Maxwell-Boltzmann velocities and the pair-parameter tables of the
workloads. It holds none of the method's arithmetic (no forces, no lists,
no integration), so that the GPU path and the CPU oracle can both consume
exactly the same arrays without sharing any computation.

The paper describes a periodic box of N particles under a truncated pair
potential (Sec. 1; Sec. 3, "Code structure") and benchmarks a truncated-force
system of 1e5 particles at several temperatures (Sec. 5, "Truncated Force
Performance Study"); no dataset is involved, so every workload here is
synthetic and seeded.

Conventions (reduced LJ units, sigma_AA = eps_AA = m = k_B = 1):
  * positions are float64 arrays of shape (N, 3), velocities likewise;
  * species are int32 in {0, 1};
  * pair tables are length-4 float64 arrays indexed [a * 2 + b].
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

MASTER_SEED = 20240606


def config_rng(index: int) -> np.random.Generator:
    """Generator for workload ``index`` (0-based) from one master seed."""
    ss = np.random.SeedSequence(MASTER_SEED).spawn(5)[index]
    return np.random.default_rng(ss)


@dataclass
class LJParams:
    """Pair-potential and integration parameters of one system.

    ``rcut`` is an absolute length per species pair; ``skin`` is the Verlet
    list skin, so the list radius of pair (a, b) is rcut[ab] + skin.
    """
    nspecies: int = 1
    eps: np.ndarray = field(default_factory=lambda: np.array([1.0, 1.0, 1.0, 1.0]))
    sigma: np.ndarray = field(default_factory=lambda: np.array([1.0, 1.0, 1.0, 1.0]))
    rcut: np.ndarray = field(default_factory=lambda: np.array([2.5, 2.5, 2.5, 2.5]))
    mass: np.ndarray = field(default_factory=lambda: np.array([1.0, 1.0]))
    shift_energy: int = 1
    skin: float = 0.3
    dt: float = 0.005
    dim: int = 3

    def copy(self) -> "LJParams":
        return LJParams(self.nspecies, self.eps.copy(), self.sigma.copy(),
                        self.rcut.copy(), self.mass.copy(), self.shift_energy,
                        self.skin, self.dt, self.dim)


def single_species_params(rc: float = 2.5, skin: float = 0.3, dt: float = 0.005) -> LJParams:
    return LJParams(1, np.ones(4), np.ones(4), np.full(4, rc), np.ones(2), 1, skin, dt)


def binary_mixture_params(skin: float = 0.3, dt: float = 0.005) -> LJParams:
    """80:20 binary mixture with eps_AB=1.5, sigma_AB=0.8, eps_BB=0.5,
    sigma_BB=0.88 and cutoffs 2.5 sigma_ab (a Kob-Andersen-type glass former)."""
    eps = np.array([1.0, 1.5, 1.5, 0.5])
    sig = np.array([1.0, 0.8, 0.8, 0.88])
    return LJParams(2, eps, sig, 2.5 * sig, np.ones(2), 1, skin, dt)


def fcc_lattice(m: int, rho: float) -> tuple[np.ndarray, float]:
    """Face-centred cubic lattice of m^3 unit cells at number density rho.

    Particle id = 4 * (i*m*m + j*m + k) + b with basis b in
    {(0,0,0), (1/2,1/2,0), (1/2,0,1/2), (0,1/2,1/2)}; origin at 0.
    Returns (positions (4 m^3, 3), box edge L).
    """
    a = (4.0 / rho) ** (1.0 / 3.0)
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    idx = np.arange(m, dtype=np.float64)
    g = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), axis=-1).reshape(-1, 3)
    x = (g[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    return np.ascontiguousarray(x), m * a


def maxwell_boltzmann(n: int, temperature: float, mass: np.ndarray, species: np.ndarray,
                      rng: np.random.Generator) -> np.ndarray:
    """Velocities drawn per component from N(0, T/m), net momentum removed,
    then rescaled so that sum m v^2 / (3N - 3) equals T exactly."""
    m = mass[species][:, None]
    v = rng.standard_normal((n, 3)) * np.sqrt(temperature / m)
    p = (m * v).sum(axis=0) / m.sum()
    v -= p[None, :]
    t_now = (m * v * v).sum() / (3 * n - 3)
    v *= math.sqrt(temperature / t_now)
    return np.ascontiguousarray(v)


@dataclass
class Workload:
    name: str
    x: np.ndarray           # (N, 3) float64
    v: np.ndarray           # (N, 3) float64
    species: np.ndarray     # (N,) int32
    box: np.ndarray         # (3,) float64
    params: LJParams
    steps: int
    temperature: float

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def lj_fluid(m: int, rho: float = 0.8442, temperature: float = 1.0, steps: int = 100,
             rng: np.random.Generator | None = None, name: str = "lj_fluid") -> Workload:
    """Single-species fluid started from an FCC lattice of m^3 cells."""
    if rng is None:
        rng = config_rng(0)
    x, L = fcc_lattice(m, rho)
    n = x.shape[0]
    sp = np.zeros(n, dtype=np.int32)
    p = single_species_params()
    v = maxwell_boltzmann(n, temperature, p.mass, sp, rng)
    return Workload(name, x, v, sp, np.full(3, L), p, steps, temperature)


def config_small() -> Workload:
    """N=2048 (FCC 8^3), rho=0.8442, T=1.0, 100 steps: the oracle-sized case."""
    return lj_fluid(8, rng=config_rng(0), steps=100, name="lj_fcc8_n2048")


def config_headline() -> Workload:
    """N=256,000 (FCC 40^3), rho=0.8442, T=1.0, 1000 steps: the headline case."""
    return lj_fluid(40, rng=config_rng(1), steps=1000, name="lj_fcc40_n256000")


def config_mixture(n: int = 4_000_000, rho: float = 1.2, seed_index: int = 2) -> Workload:
    """Binary 80:20 mixture: uniform random positions (to be relaxed by
    steepest descent before dynamics), exactly round(0.8 n) particles of
    species 0 chosen by a seeded permutation, velocities at T=0.8."""
    rng = config_rng(seed_index)
    L = (n / rho) ** (1.0 / 3.0)
    x = rng.uniform(0.0, L, size=(n, 3))
    sp = np.ones(n, dtype=np.int32)
    sp[rng.permutation(n)[: int(round(0.8 * n))]] = 0
    p = binary_mixture_params()
    v = maxwell_boltzmann(n, 0.8, p.mass, sp, rng)
    return Workload(f"ka_mixture_n{n}", np.ascontiguousarray(x), v, sp, np.full(3, L), p, 500, 0.8)


def jittered_fcc(m: int, rho: float = 0.8442, amp: float = 0.05, temperature: float = 1.0,
                 seed_index: int = 3) -> tuple[Workload, np.ndarray, np.ndarray]:
    """FCC lattice with N(0, amp^2) jitter (a perfect lattice has zero force
    for every parameter set), MB velocities at T, and target parameters
    (eps*, sigma*) = (eps (1 + u_e), sigma (1 + u_s)), u ~ U(-0.05, 0.05).

    Returns (workload, eps_target(4), sigma_target(4))."""
    rng = config_rng(seed_index)
    x, L = fcc_lattice(m, rho)
    n = x.shape[0]
    x = x + amp * rng.standard_normal(x.shape)
    sp = np.zeros(n, dtype=np.int32)
    p = single_species_params()
    v = maxwell_boltzmann(n, temperature, p.mass, sp, rng)
    u = rng.uniform(-0.05, 0.05, size=2)
    eps_t = p.eps * (1.0 + u[0])
    sig_t = p.sigma * (1.0 + u[1])
    return (Workload(f"jittered_fcc{m}_n{n}", np.ascontiguousarray(x), v, sp, np.full(3, L), p, 50,
                     temperature), eps_t, sig_t)


def replica_draws(nrep: int = 512, seed_index: int = 4, nmin: int = 500, nmax: int = 32000):
    """Per replica: N = round(exp(U(ln nmin, ln nmax))), rho ~ U(0.7, 1.2),
    T ~ U(0.7, 1.5). Positions: FCC with M = ceil((N/4)^(1/3)) cells scaled
    to L = (N/rho)^(1/3), keeping N sites chosen by a seeded permutation."""
    rng = config_rng(seed_index)
    out = []
    for r in range(nrep):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        rho = float(rng.uniform(0.7, 1.2))
        temp = float(rng.uniform(0.7, 1.5))
        m = int(math.ceil((n / 4.0) ** (1.0 / 3.0)))
        xs, _ = fcc_lattice(m, 1.0)
        L = (n / rho) ** (1.0 / 3.0)
        xs = xs * (L / (m * (4.0 / 1.0) ** (1.0 / 3.0)))
        keep = np.sort(rng.permutation(xs.shape[0])[:n])
        x = np.ascontiguousarray(xs[keep])
        sp = np.zeros(n, dtype=np.int32)
        p = single_species_params()
        v = maxwell_boltzmann(n, temp, p.mass, sp, rng)
        out.append(Workload(f"replica{r}_n{n}", x, v, sp, np.full(3, L), p, 1000, temp))
    return out


def all_pairs_fluid(n: int = 2000, rho: float = 0.8442, temperature: float = 1.0, seed_index: int = 0,
                    steps: int = 20000) -> Workload:
    """The all-to-all workload (the paper's 2,000 particles): N sites kept,
    by a seeded permutation, from the smallest FCC lattice that holds them,
    scaled to density rho; Maxwell-Boltzmann velocities at T. The cutoffs
    are infinite: every pair of the minimum image interacts, unshifted."""
    rng = config_rng(seed_index)
    m = int(math.ceil((n / 4.0) ** (1.0 / 3.0)))
    xs, _ = fcc_lattice(m, 1.0)
    L = (n / rho) ** (1.0 / 3.0)
    xs = xs * (L / (m * 4.0 ** (1.0 / 3.0)))
    keep = np.sort(rng.permutation(xs.shape[0])[:n])
    x = np.ascontiguousarray(xs[keep])
    sp = np.zeros(n, dtype=np.int32)
    p = single_species_params()
    p.rcut = np.full(4, np.inf)
    v = maxwell_boltzmann(n, temperature, p.mass, sp, rng)
    return Workload(f"all_pairs_n{n}", x, v, sp, np.full(3, L), p, steps, temperature)


def thermostat_fluid(n: int = 100_000, rho: float = 0.8442, temperature: float = 1.0, seed_index: int = 1,
                     steps: int = 2000) -> Workload:
    """The truncated-force study shape (the paper's 100,000 particles at
    several temperatures): N sites kept, by a seeded permutation, from the
    smallest FCC lattice that holds them, scaled to density rho;
    Maxwell-Boltzmann velocities at T; cutoff 2.5 with energy shift, skin
    0.3, dt 0.005."""
    rng = config_rng(seed_index)
    m = int(math.ceil((n / 4.0) ** (1.0 / 3.0)))
    xs, _ = fcc_lattice(m, 1.0)
    L = (n / rho) ** (1.0 / 3.0)
    xs = xs * (L / (m * 4.0 ** (1.0 / 3.0)))
    keep = np.sort(rng.permutation(xs.shape[0])[:n])
    x = np.ascontiguousarray(xs[keep])
    sp = np.zeros(n, dtype=np.int32)
    p = single_species_params()
    v = maxwell_boltzmann(n, temperature, p.mass, sp, rng)
    return Workload(f"thermostat_fluid_n{n}_T{temperature:g}", x, v, sp, np.full(3, L), p, steps, temperature)


def triangular_lattice(m: int, rho: float) -> tuple[np.ndarray, np.ndarray]:
    """Two-dimensional triangular lattice of 2 m^2 sites (rectangular cell of
    two sites, m x m cells) at number density rho per unit area, in the
    plane z = 0. Returns (positions (2 m^2, 3), box edges (Lx, Ly, Lx)); the
    box is periodic in x and y (the third edge only sizes the unused z axis)."""
    a = math.sqrt(2.0 / (math.sqrt(3.0) * rho))      # nearest-neighbour distance
    bx, by = a, a * math.sqrt(3.0)                   # rectangular cell with 2 sites
    idx = np.arange(m, dtype=np.float64)
    gx, gy = np.meshgrid(idx, idx, indexing="ij")
    base = np.stack([gx.ravel() * bx, gy.ravel() * by], axis=1)
    sites = np.concatenate([base, base + np.array([0.5 * bx, 0.5 * by])], axis=0)
    x = np.zeros((sites.shape[0], 3))
    x[:, :2] = sites
    L = np.array([m * bx, m * by, m * bx])
    return x, L


def maxwell_boltzmann_2d(n: int, temperature: float, mass: np.ndarray, species: np.ndarray,
                         rng: np.random.Generator) -> np.ndarray:
    """In-plane velocities from N(0, T/m) per component, net momentum
    removed, rescaled so that sum m v^2 / (2N - 2) equals T; v_z = 0."""
    m = mass[species][:, None]
    v = np.zeros((n, 3))
    v[:, :2] = rng.standard_normal((n, 2)) * np.sqrt(temperature / m)
    p = (m * v).sum(axis=0) / m.sum()
    v -= p[None, :]
    v[:, 2] = 0.0
    t_now = (m * v * v).sum() / (2 * n - 2)
    v *= math.sqrt(temperature / t_now)
    return np.ascontiguousarray(v)


def lj_fluid_2d(m: int = 32, rho: float = 0.7, temperature: float = 1.0, seed_index: int = 3,
                jitter: float = 0.05, steps: int = 100) -> Workload:
    """Two-dimensional LJ fluid (the dimension template of the paper's
    modules, Sec. 3): a triangular lattice of 2 m^2 sites at areal density
    rho with a seeded Gaussian jitter in the plane, Maxwell-Boltzmann
    velocities in the plane; cutoff 2.5 shifted, skin 0.3, dt 0.005."""
    rng = config_rng(seed_index)
    x, L = triangular_lattice(m, rho)
    x[:, :2] += jitter * rng.standard_normal((x.shape[0], 2))
    x[:, :2] %= L[:2]
    n = x.shape[0]
    sp = np.zeros(n, dtype=np.int32)
    p = single_species_params()
    p.dim = 2
    v = maxwell_boltzmann_2d(n, temperature, p.mass, sp, rng)
    return Workload(f"lj2d_tri{m}_n{n}", np.ascontiguousarray(x), v, sp, L, p, steps, temperature)


def random_dense(n: int, rho: float, seed: int, min_dist: float = 0.85,
                 nspecies: int = 1) -> Workload:
    """Small disordered configuration for tests: random sequential insertion
    with a minimum separation, so that no pair is unphysically close."""
    rng = np.random.default_rng(seed)
    L = (n / rho) ** (1.0 / 3.0)
    pts = []
    tries = 0
    md2 = min_dist * min_dist
    while len(pts) < n:
        tries += 1
        if tries > 200 * n:
            raise RuntimeError("insertion failed; lower rho or min_dist")
        c = rng.uniform(0.0, L, size=3)
        if pts:
            d = np.asarray(pts) - c
            d -= L * np.round(d / L)
            if np.min((d * d).sum(axis=1)) < md2:
                continue
        pts.append(c)
    x = np.ascontiguousarray(np.asarray(pts))
    if nspecies == 1:
        sp = np.zeros(n, dtype=np.int32)
        p = single_species_params()
    else:
        sp = (rng.uniform(size=n) < 0.2).astype(np.int32)
        p = binary_mixture_params()
    v = maxwell_boltzmann(n, 1.0, p.mass, sp, rng)
    return Workload(f"random_n{n}", x, v, sp, np.full(3, L), p, 100, 1.0)
