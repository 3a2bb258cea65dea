"""Seeded synthetic inputs for the LSH indexing path.

This module only draws random numbers and lays them out: point sets shaped
like the workloads of the paper's experiments (Section 6), and the random
state that the hash families draw (count-sketch hashes h and signs s, the
per-mode hashes of the higher-order count sketch, the shifts b and the dense
Gaussian matrix R).  It contains none of the hashing arithmetic; the GPU
library and the CPU oracle both take these arrays as plain inputs.

Every generator is a pure function of its seed.  Point sets are generated in
fixed blocks of rows, each with its own PCG64 stream, so any subset of rows can
be regenerated cheaply and blocks can be drawn on several threads.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 250306737
ROW_BLOCK = 4096


def config_seed(c: int) -> int:
    """Base seed of workload ``c`` (data); +1 hash state, +2 queries, +3 stream."""
    return SEED_BASE + 1000 * c


def _rng(*words: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(words))))


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _fill_blocks(n: int, d: int, fn, dtype=np.float32, rows: np.ndarray | None = None) -> np.ndarray:
    """Build an (n, d) array block by block; ``fn(block_index, lo, hi)`` returns rows lo..hi."""
    out = np.empty((n, d), dtype=dtype)
    nblk = (n + ROW_BLOCK - 1) // ROW_BLOCK

    def work(bi):
        lo, hi = bi * ROW_BLOCK, min(n, (bi + 1) * ROW_BLOCK)
        out[lo:hi] = fn(bi, lo, hi)

    if nblk <= 1:
        for bi in range(nblk):
            work(bi)
    else:
        with _cf.ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nblk)))
    return out


# ----------------------------------------------------------------------------
# point sets
# ----------------------------------------------------------------------------

def gaussian_centres(n_centres: int, d: int, seed: int) -> np.ndarray:
    """Cluster centres mu_c ~ N(0, I_d), float64."""
    return _rng(seed, 0xCE17).standard_normal((n_centres, d))


def gaussian_clusters(n: int, d: int, n_centres: int, sigma: float, seed: int,
                      stream: int = 0) -> np.ndarray:
    """Mixture of isotropic Gaussians: x = mu_c + sigma * eps, c ~ U{0..C-1}.

    ``stream`` selects an independent draw of points around the same centres
    (0 = base set, 1 = held-out queries, 2.. = inserts).
    """
    mu = gaussian_centres(n_centres, d, seed)

    def fn(bi, lo, hi):
        g = _rng(seed, 0xDA7A, stream, bi)
        c = g.integers(0, n_centres, hi - lo)
        eps = g.standard_normal((hi - lo, d), dtype=np.float32)
        return (mu[c] + sigma * eps).astype(np.float32)

    return _fill_blocks(n, d, fn)


def sparse_uniform(n: int, d: int, density: float, seed: int, stream: int = 0) -> np.ndarray:
    """Image-like rows: x_ij = B_ij * U_ij, B ~ Bernoulli(density), U ~ U(0,1)."""

    def fn(bi, lo, hi):
        g = _rng(seed, 0x5A5E, stream, bi)
        u = g.random((hi - lo, d), dtype=np.float32)
        keep = g.random((hi - lo, d), dtype=np.float32) < density
        return np.where(keep, u, np.float32(0.0))

    return _fill_blocks(n, d, fn)


# ----------------------------------------------------------------------------
# random state drawn by the hash families
# ----------------------------------------------------------------------------

def cs_state(d: int, m: int, seed: int):
    """h:[d]->[m] uniform (unbiased bounded draw), s:[d]->{+1,-1}."""
    g = _rng(seed, 0xC5)
    h = g.integers(0, m, d, dtype=np.int64).astype(np.uint32)
    s = np.where(g.random(d) < 0.5, -1, 1).astype(np.int8)
    return h, s


def hcs_state(dk, mk, seed: int):
    """Per-mode hashes h_k:[d_k]->[m_k] and signs s_k, k = 1..N."""
    g = _rng(seed, 0x4C5)
    hk, sk = [], []
    for dd, mm in zip(dk, mk):
        hk.append(g.integers(0, mm, dd, dtype=np.int64).astype(np.uint32))
        sk.append(np.where(g.random(dd) < 0.5, -1, 1).astype(np.int8))
    return hk, sk


def cs_tables_state(d: int, K: int, L: int, seed: int):
    """Independent per-table count-sketch state: h [L][d] uniform in [0, K),
    s [L][d] in {+1, -1} (one draw per table from its own stream)."""
    h = np.empty((L, d), np.uint32)
    s = np.empty((L, d), np.int8)
    for t in range(L):
        h[t], s[t] = cs_state(d, K, seed * 1000 + t)
    return h, s


def hcs_tables_state(dk, mk, L: int, seed: int):
    """Independent per-table HCS state: for each table its per-mode hashes and
    signs, laid out as [L][sum d_k] (table t's N mode tables back to back)."""
    tot = int(sum(dk))
    h = np.empty((L, tot), np.uint32)
    s = np.empty((L, tot), np.int8)
    for t in range(L):
        hk, sk = hcs_state(dk, mk, seed * 1000 + t)
        h[t], s[t] = np.concatenate(hk), np.concatenate(sk)
    return h, s


def component_slots(m: int, seed: int) -> np.ndarray:
    """A uniformly random permutation of range(m): code position of each sketch
    component (which components form which table)."""
    return _rng(seed, 0x510).permutation(m).astype(np.uint32)


def shifts(m: int, w: float, seed: int) -> np.ndarray:
    """b_l ~ U[0, w) as float32, one per hashcode component."""
    g = _rng(seed, 0xB0)
    b = (g.random(m) * w).astype(np.float32)
    top = np.nextafter(np.float32(w), np.float32(0.0))
    return np.minimum(b, top).astype(np.float32)


def gaussian_matrix(d: int, m: int, seed: int) -> np.ndarray:
    """Dense projection R[d][m] with entries N(0,1), float32."""
    return _rng(seed, 0x6A55).standard_normal((d, m), dtype=np.float32)


# ----------------------------------------------------------------------------
# low-precision storage with per-row scales
# ----------------------------------------------------------------------------

def quantise_rows(x: np.ndarray, kind: str):
    """Store rows as BF16 or FP8-E4M3FN codes with a float32 scale per row.

    BF16: scale = max|x_i|, codes = bf16(x_i / scale) (round to nearest even).
    FP8:  scale = max|x_i| / 448, codes = e4m3fn(x_i / scale) (round to
    nearest even, saturating).  Returns (codes as uint16/uint8 bit patterns,
    scale float32).  A zero row gets scale 1.
    """
    import torch

    amax = np.abs(x).max(axis=1).astype(np.float32)
    if kind == "bf16":
        scale = np.where(amax > 0, amax, np.float32(1.0)).astype(np.float32)
        q = torch.from_numpy((x / scale[:, None]).astype(np.float32)).to(torch.bfloat16)
        return q.view(torch.int16).numpy().view(np.uint16), scale
    if kind == "fp8":
        scale = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
        v = np.clip((x / scale[:, None]).astype(np.float32), -448.0, 448.0)
        q = torch.from_numpy(v).to(torch.float8_e4m3fn)
        return q.view(torch.uint8).numpy(), scale
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    d: int
    K: int
    L: int
    w: float
    seed: int
    data: str                      # "clusters" | "sparse"
    n_centres: int = 0
    sigma: float = 0.0
    density: float = 0.0
    n_query: int = 0
    hcs: tuple = field(default_factory=tuple)   # ((dk...), (mk...)) pairs

    @property
    def m(self) -> int:
        return self.K * self.L

    def points(self, n: int | None = None, stream: int = 0) -> np.ndarray:
        n = self.n if n is None else n
        if self.data == "clusters":
            return gaussian_clusters(n, self.d, self.n_centres, self.sigma, self.seed, stream)
        return sparse_uniform(n, self.d, self.density, self.seed, stream)

    def queries(self, nq: int | None = None) -> np.ndarray:
        return self.points(self.n_query if nq is None else nq, stream=1)

    def cs(self):
        return cs_state(self.d, self.m, self.seed + 1)

    def hcs_state(self, i: int):
        dk, mk = self.hcs[i]
        return hcs_state(dk, mk, self.seed + 1)

    def slots(self) -> np.ndarray:
        return component_slots(self.m, self.seed + 1)

    def b(self) -> np.ndarray:
        return shifts(self.m, self.w, self.seed + 1)

    def R(self) -> np.ndarray:
        return gaussian_matrix(self.d, self.m, self.seed + 1)


C1 = Workload("c1-clusters-n10k-d1024-m128", n=10_000, d=1024, K=8, L=16, w=4.0,
              seed=config_seed(1), data="clusters", n_centres=50, sigma=0.1, n_query=1000)
C2 = Workload("c2-sparse-n1M-d784-m1024", n=1_000_000, d=784, K=16, L=64, w=4.0,
              seed=config_seed(2), data="sparse", density=0.2, n_query=1000)
C3 = Workload("c3-clusters-n500k-d4096-m1024", n=500_000, d=4096, K=16, L=64, w=4.0,
              seed=config_seed(3), data="clusters", n_centres=200, sigma=0.2, n_query=1000,
              hcs=(((64, 64), (32, 32)), ((16, 16, 16), (8, 8, 16))))
C4 = Workload("c4-clusters-n200k-d16384-m512", n=200_000, d=16384, K=16, L=32, w=4.0,
              seed=config_seed(4), data="clusters", n_centres=50, sigma=0.1, n_query=1000)
C5 = Workload("c5-serving-n2M-d960-m512", n=2_000_000, d=960, K=16, L=32, w=4.0,
              seed=config_seed(5), data="clusters", n_centres=200, sigma=0.05, n_query=4096)

WORKLOADS = {"c1": C1, "c2": C2, "c3": C3, "c4": C4, "c5": C5}
