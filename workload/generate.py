"""Seeded synthetic workloads for the matrix-pencil Prony method.

Every random draw of a workload is made here from one numpy PCG64 stream per
instance, spawned from a master seed, so that the CPU oracle and the GPU path
see identical inputs. Nothing here evaluates the exponential sum or any other
step of the method: the functions return nodes t_j in [0,1)^d, coefficients
c_j, additive or relative noise arrays over the sample grid, the random unit
vector mu of the combination C_mu, and random starting blocks for the block
power SVD.

Sample grid convention (shared by both sides): points p in {-n..n+1}^d stored
flat in row-major order (last coordinate fastest), (2n+2)^d entries.

Workloads (the paper's own test inputs are in `paper_efficiency_inputs`):

* ``c0``  d=2, n=15, m=5, torus separation >= 0.05, |c| ~ U[0.5,1.5],
  arg c ~ U[0,2pi), noise-free.
* ``c1``  d=2, n=63, m=20, same distributions, additive circular complex
  Gaussian noise of standard deviation 1e-6*max|c_j|.
* ``c2``  d=3, n=19, m=30, separation >= 0.08, |c| log-uniform in [1e-2,1],
  noise levels {0, 1e-8, 1e-6, 1e-4, 1e-3} (one unit-noise draw, scaled).
* ``c3``  512 instances: d ~ U{1,2,3}, N* log-uniform in [64,4096],
  n = max(1, round(N*^(1/d)) - 1) clamped so N=(n+1)^d in [64,4096],
  m ~ U{2..32}, c0 distributions, noise 1e-7. For d=1 the separation is
  min(0.05, 0.5/m) and nodes are drawn by an exact spacing construction,
  since rejection sampling cannot place 32 points 0.05 apart on a circle.
* ``c4``  64 instances of d=2, n=47, m=16, c0 distributions, noise 1e-6.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

MASTER_SEED = 201211430

# (d, n, m, separation, |c| law, noise levels)
_CONFIGS = {
    "c0": dict(d=2, n=15, m=5, sep=0.05, mag="uniform", noise=(0.0,)),
    "c1": dict(d=2, n=63, m=20, sep=0.05, mag="uniform", noise=(1e-6,)),
    "c2": dict(d=3, n=19, m=30, sep=0.08, mag="loguniform",
               noise=(0.0, 1e-8, 1e-6, 1e-4, 1e-3)),
    "c4": dict(d=2, n=47, m=16, sep=0.05, mag="uniform", noise=(1e-6,)),
}
_CONFIG_INDEX = {"c0": 0, "c1": 1, "c2": 2, "c3": 3, "c4": 4}
C3_COUNT = 512
C4_COUNT = 64


@dataclasses.dataclass
class Instance:
    """One synthetic problem: the truth (t, c) plus the random inputs of a run."""

    name: str
    d: int
    n: int
    m: int
    t: np.ndarray            # (m, d) float64, nodes in [0,1)^d
    c: np.ndarray            # (m,) complex128, nonzero coefficients
    noise_unit: np.ndarray   # ((2n+2)^d,) complex128, CN(0,1) draw
    noise_levels: tuple      # relative levels sigma; noise = sigma*max|c|*unit
    mu: np.ndarray           # (d,) complex128, unit 2-norm
    seed: tuple              # spawn key of the instance's stream

    @property
    def N(self) -> int:
        return (self.n + 1) ** self.d

    @property
    def grid_size(self) -> int:
        return (2 * self.n + 2) ** self.d

    def noise(self, level: float | None = None) -> np.ndarray:
        """Additive noise array for relative level `level` (default: first level)."""
        if level is None:
            level = self.noise_levels[0]
        return (level * float(np.max(np.abs(self.c)))) * self.noise_unit


def _torus_gap(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    diff = np.abs(a - b) % 1.0
    return np.sqrt(np.sum(np.minimum(diff, 1.0 - diff) ** 2, axis=-1))


def torus_distance(a, b):
    """Euclidean distance on the flat torus [0,1)^d (used to match nodes)."""
    return _torus_gap(np.asarray(a, float), np.asarray(b, float))


def _draw_nodes(rng: np.random.Generator, d: int, m: int, sep: float) -> np.ndarray:
    if d == 1:
        sep = min(sep, 0.5 / m)
        slack = 1.0 - m * sep
        gaps = np.sort(rng.random(m)) * slack
        t = (rng.random() + gaps + sep * np.arange(m)) % 1.0
        return rng.permutation(t).reshape(m, 1)
    pts = []
    tries = 0
    while len(pts) < m:
        tries += 1
        if tries > 200000:
            raise RuntimeError("node rejection sampling did not converge")
        cand = rng.random(d)
        if all(_torus_gap(cand, p) >= sep for p in pts):
            pts.append(cand)
    return np.array(pts)


def _draw_coeffs(rng: np.random.Generator, m: int, mag: str) -> np.ndarray:
    if mag == "uniform":
        r = rng.uniform(0.5, 1.5, m)
    else:
        r = 10.0 ** rng.uniform(-2.0, 0.0, m)
    phi = rng.uniform(0.0, 2.0 * math.pi, m)
    return r * np.exp(1j * phi)


def _draw_cn(rng: np.random.Generator, size: int) -> np.ndarray:
    """Circular complex Gaussian CN(0,1): real and imaginary parts N(0,1/2)."""
    z = rng.standard_normal((size, 2)) * math.sqrt(0.5)
    return z[:, 0] + 1j * z[:, 1]


def random_unit_vector(rng: np.random.Generator, d: int) -> np.ndarray:
    """mu uniform on the complex unit sphere: normalised complex Gaussian."""
    g = _draw_cn(rng, d)
    return g / np.linalg.norm(g)


def random_orthonormal(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Complex Gaussian rows x cols block (the caller orthonormalises it)."""
    return _draw_cn(rng, rows * cols).reshape(rows, cols)


def draw_instance(name: str, d: int, n: int, m: int, sep: float, mag: str,
                  noise_levels, seed_seq: np.random.SeedSequence) -> Instance:
    rng = np.random.Generator(np.random.PCG64(seed_seq))
    t = _draw_nodes(rng, d, m, sep)
    c = _draw_coeffs(rng, m, mag)
    noise_unit = _draw_cn(rng, (2 * n + 2) ** d)
    mu = random_unit_vector(rng, d)
    return Instance(name=name, d=d, n=n, m=m, t=t, c=c, noise_unit=noise_unit,
                    noise_levels=tuple(noise_levels), mu=mu,
                    seed=(MASTER_SEED,) + tuple(seed_seq.spawn_key))


def _config_seed(name: str) -> np.random.SeedSequence:
    return np.random.SeedSequence(MASTER_SEED).spawn(5)[_CONFIG_INDEX[name]]


def _c3_shape(rng: np.random.Generator):
    d = int(rng.integers(1, 4))
    nstar = math.exp(rng.uniform(math.log(64.0), math.log(4096.0)))
    n = max(1, int(round(nstar ** (1.0 / d))) - 1)
    while (n + 1) ** d < 64:
        n += 1
    while (n + 1) ** d > 4096:
        n -= 1
    m = int(rng.integers(2, 33))
    return d, n, m


def config_instances(name: str, count: int | None = None) -> list:
    """Instances of workload `name` ('c0'..'c4'); `count` truncates c3/c4."""
    root = _config_seed(name)
    if name in _CONFIGS:
        cfg = _CONFIGS[name]
        total = C4_COUNT if name == "c4" else 1
        if count is not None:
            total = min(total, count)
        kids = root.spawn(total) if name == "c4" else [root]
        return [draw_instance(name, cfg["d"], cfg["n"], cfg["m"], cfg["sep"],
                              cfg["mag"], cfg["noise"], kids[i])
                for i in range(total)]
    if name == "c3":
        total = C3_COUNT if count is None else min(count, C3_COUNT)
        kids = root.spawn(C3_COUNT)[:total]
        out = []
        for kid in kids:
            shape_rng = np.random.Generator(np.random.PCG64(kid.spawn(1)[0]))
            d, n, m = _c3_shape(shape_rng)
            out.append(draw_instance("c3", d, n, m, 0.05, "uniform", (1e-7,), kid))
        return out
    raise KeyError(name)


def paper_efficiency_inputs(d: int, m: int):
    """Deterministic nodes and coefficients of the paper's efficiency tests (Sec. 5):
    t_j(i) = ((i-1)m + j - 1) * 10^(-ceil(log10(d m))), c_j = j + i j (i imaginary)."""
    scale = 10.0 ** (-math.ceil(math.log10(d * m)))
    t = np.array([[((i - 1) * m + j - 1) * scale for i in range(1, d + 1)]
                  for j in range(1, m + 1)], dtype=float)
    c = np.array([j + 1j * j for j in range(1, m + 1)], dtype=complex)
    return t, c


def paper_relative_noise(seed: int, d: int, n: int, eps: float) -> np.ndarray:
    """Real relative perturbations delta_k ~ U[-eps, eps] over the sample grid
    (the accuracy experiment of Sec. 5 perturbs f(k) as f(k)(1 + delta_k))."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([MASTER_SEED, seed])))
    return rng.uniform(-eps, eps, (2 * n + 2) ** d)
