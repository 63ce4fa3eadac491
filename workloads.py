"""Seeded synthetic particle systems for the range-separated (RS) potential path.

This module only draws inputs: particle positions, charges and the run
parameters that describe a workload.  It holds none of the method's
arithmetic (no quadrature, no splitting rule, no window size derivation), so
that both the CPU oracle and the GPU path can read identical bytes without
sharing any of the computation.

The paper's own particle data (protein-type clusters of 100..782 atoms and
finite lattices with random charges, sections 3.2 and 4.2) is not available;
the systems below are synthetic stand-ins of the same kinds: uniform clouds
with a minimum separation (the sigma*-separable sets of Definition
QU_Distrib), a jittered lattice with vacancies and alternating charges, and
clustered "protein-like" clouds.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class System:
    """One particle system plus the parameters of the RS run on it."""
    name: str
    pos: np.ndarray          # (N, 3) float64, inside [-b, b]^3
    q: np.ndarray            # (N,) float64 charges
    b: float                 # half box width, Omega = [-b, b]^3
    n: int                   # grid points per axis (even)
    R: int                   # quadrature terms (R = M + 1)
    R_l: int                 # long-range terms k = 0 .. R_l - 1
    n_s: Optional[int]       # short-range window width (odd), None = derive
    kernel: str = "newton"   # "newton" | "yukawa" | "newton+yukawa"
    lam: float = 0.5         # Yukawa screening
    eps_tucker: float = 1e-6
    delta_rel: float = 1e-4  # criterion (A) threshold relative to S(0)
    seed: int = 0

    @property
    def N(self) -> int:
        return int(self.pos.shape[0])

    @property
    def h(self) -> float:
        return 2.0 * self.b / self.n


class _SepSet:
    """Points accepted so far, hashed into cells of side min_sep so that a
    candidate is compared only with points in the 27 neighbouring cells."""

    def __init__(self, capacity: int, min_sep: float):
        self.pts = np.empty((capacity, 3))
        self.count = 0
        self.min_sep = min_sep
        self.buckets: dict = {}

    def _key(self, p):
        return tuple(int(math.floor(c / self.min_sep)) for c in p)

    def try_add(self, p) -> bool:
        if self.min_sep > 0:
            key = self._key(p)
            ms2 = self.min_sep * self.min_sep
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        for idx in self.buckets.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                            d = self.pts[idx] - p
                            if d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < ms2:
                                return False
            self.buckets.setdefault(key, []).append(self.count)
        self.pts[self.count] = p
        self.count += 1
        return True


def _fill(sep: _SepSet, target: int, draw, max_tries_factor: int = 1000) -> None:
    got, tries = 0, 0
    while got < target:
        tries += 1
        if tries > max_tries_factor * max(target, 1):
            raise RuntimeError(f"could not place {target} points with min separation {sep.min_sep}")
        p = draw()
        if p is not None and sep.try_add(p):
            got += 1


def _min_sep_uniform(rng: np.random.Generator, N: int, lo: float, hi: float,
                     min_sep: float) -> np.ndarray:
    """Sequential rejection sampling: N points uniform in [lo, hi]^3 whose
    pairwise distances are all >= min_sep."""
    sep = _SepSet(N, min_sep)
    _fill(sep, N, lambda: rng.uniform(lo, hi, size=3))
    return sep.pts


def cfg1_plain_small(seed: int = 1) -> System:
    """Newton 1/r on [-10,10]^3, n=128, R=20, R_l=8, n_s=9; N=64 uniform in
    [-6,6]^3 with min separation 0.8, charges uniform in [-1,1]."""
    rng = np.random.default_rng(seed)
    pos = _min_sep_uniform(rng, 64, -6.0, 6.0, 0.8)
    q = rng.uniform(-1.0, 1.0, size=64)
    return System("cfg1_uniform64_n128", pos, q, b=10.0, n=128, R=20, R_l=8,
                  n_s=9, eps_tucker=1e-6, seed=seed)


def lattice_with_vacancies(rng, side: int, spacing: float, n_vac: int,
                           jitter_sd: float) -> Tuple[np.ndarray, np.ndarray]:
    ii, jj, kk = np.meshgrid(np.arange(side), np.arange(side), np.arange(side), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    centre = (side - 1) / 2.0
    pos = np.stack([ii - centre, jj - centre, kk - centre], axis=1) * spacing
    q = np.where((ii + jj + kk) % 2 == 0, 1.0, -1.0)
    vac = rng.choice(pos.shape[0], size=n_vac, replace=False)
    keep = np.ones(pos.shape[0], dtype=bool)
    keep[vac] = False
    pos = pos[keep] + rng.normal(0.0, jitter_sd, size=(int(keep.sum()), 3))
    return pos, q[keep]


def cfg2_lattice(seed: int = 2, n_s: Optional[int] = 17) -> System:
    """Cubic lattice 10x10x10, spacing 1.0, 10% random vacancies (exactly 100),
    positions jittered by N(0, 0.05^2), alternating +-1 charges; n=512, box
    [-12,12]^3, R=24, R_l=10, n_s=17."""
    rng = np.random.default_rng(seed)
    pos, q = lattice_with_vacancies(rng, 10, 1.0, 100, 0.05)
    return System("cfg2_lattice900_n512", pos, q, b=12.0, n=512, R=24, R_l=10,
                  n_s=n_s, eps_tucker=1e-6, seed=seed)


def cfg3_protein_like(seed: int = 3, N: int = 10000, n: int = 1024) -> System:
    """N=10000 charges in 40 Gaussian blobs (sigma=2.0, centres uniform in
    [-19,19]^3) inside [-25,25]^3, charges drawn from {-1,-0.5,0.5,1}; n=1024,
    R=32, R_l=12; window derived by criterion (A).  A minimum separation of
    0.8 is imposed (the separability assumption of Definition QU_Distrib)."""
    rng = np.random.default_rng(seed)
    n_blobs = 40
    centres = rng.uniform(-19.0, 19.0, size=(n_blobs, 3))
    per = N // n_blobs
    sep = _SepSet(N, 0.8)
    for blob in range(n_blobs):
        target = per if blob < n_blobs - 1 else N - per * (n_blobs - 1)
        c = centres[blob]

        def draw(c=c):
            p = rng.normal(c, 2.0)
            return None if np.any(np.abs(p) > 25.0 - 1e-9) else p

        _fill(sep, target, draw)
    q = rng.choice(np.array([-1.0, -0.5, 0.5, 1.0]), size=N)
    return System(f"cfg3_protein{N}_n{n}", sep.pts, q, b=25.0, n=n, R=32, R_l=12,
                  n_s=None, eps_tucker=1e-6, seed=seed)


def cfg4_forces(seed: int = 4, N: int = 4096, kernel: str = "newton+yukawa") -> System:
    """N=4096 uniform in [-15,15]^3 with min separation 0.7, charges +-1
    summing to zero; n=512, R=28; kernel 1/r + e^{-0.5 r}/r.  The box half
    width b=18 and R_l=11 are chosen here (the workload's statement leaves
    them open)."""
    rng = np.random.default_rng(seed)
    pos = _min_sep_uniform(rng, N, -15.0, 15.0, 0.7)
    q = np.concatenate([np.ones(N // 2), -np.ones(N - N // 2)])
    rng.shuffle(q)
    return System(f"cfg4_forces{N}_n512", pos, q, b=18.0, n=512, R=28, R_l=11,
                  n_s=None, kernel=kernel, lam=0.5, eps_tucker=1e-6, seed=seed)


@dataclasses.dataclass
class Request:
    idx: int
    arrival_s: float
    N: int
    n: int
    R: int
    R_l: int
    seed: int
    b: float = 25.0

    def system(self) -> System:
        rng = np.random.default_rng(self.seed)
        pos = rng.uniform(-20.0, 20.0, size=(self.N, 3))
        q = rng.uniform(-1.0, 1.0, size=self.N)
        return System(f"req{self.idx}", pos, q, b=self.b, n=self.n, R=self.R,
                      R_l=self.R_l, n_s=None, eps_tucker=1e-6, seed=self.seed)


def cfg5_trace(seed: int = 5, n_requests: int = 2000, rate_hz: float = 200.0,
               n_choices=(256, 512, 1024), N_lo: int = 32, N_hi: int = 20000) -> List[Request]:
    """Poisson arrivals (rate 200/s); each request a random system with N
    log-uniform in [32, 20000], uniform positions in [-20,20]^3 inside the box
    [-25,25]^3, charges uniform in [-1,1], n in {256,512,1024}, R in 24..32,
    R_l = round(0.4 R)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    Ns = np.rint(np.exp(rng.uniform(math.log(N_lo), math.log(N_hi), size=n_requests))).astype(int)
    ns = rng.choice(np.array(n_choices), size=n_requests)
    Rs = rng.integers(24, 33, size=n_requests)
    seeds = rng.integers(0, 2**31 - 1, size=n_requests)
    out = []
    for i in range(n_requests):
        R = int(Rs[i])
        out.append(Request(i, float(arrivals[i]), int(Ns[i]), int(ns[i]), R,
                           int(round(0.4 * R)), int(seeds[i])))
    return out


def tiny_system(seed: int, N: int, b: float, n: int, R: int, R_l: int,
                n_s: Optional[int], min_sep: float = 0.0, box_frac: float = 0.6,
                kernel: str = "newton", neutral: bool = False,
                eps_tucker: float = 1e-6) -> System:
    """Small seeded systems for brute-force and parity cases."""
    rng = np.random.default_rng(seed)
    lo, hi = -box_frac * b, box_frac * b
    if min_sep > 0:
        pos = _min_sep_uniform(rng, N, lo, hi, min_sep)
    else:
        pos = rng.uniform(lo, hi, size=(N, 3))
    if neutral:
        q = np.concatenate([np.ones(N // 2), -np.ones(N - N // 2)])
        rng.shuffle(q)
    else:
        q = rng.uniform(-1.0, 1.0, size=N)
    return System(f"tiny_s{seed}_N{N}_n{n}", pos, q, b=b, n=n, R=R, R_l=R_l,
                  n_s=n_s, kernel=kernel, eps_tucker=eps_tucker, seed=seed)


def grid_sample_indices(seed: int, n: int, count: int) -> np.ndarray:
    """Seeded random flat grid indices (C order, i3 fastest) for sampled checks."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, n ** 3, size=count, dtype=np.int64)
