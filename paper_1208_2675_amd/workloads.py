"""Seeded synthetic QAP instances shaped like the paper's workloads.

Section 4 of the paper measures on random instances built the way QAPLIB's
Tai-a family is built: symmetric flow and distance matrices with a zero
diagonal and independent uniform entries.  The instance files themselves are
not used; every instance here is drawn from numpy's PCG64 with a fixed seed,
so that both the oracle and the HIP path receive the same arrays.

This module holds only input generation.  It computes nothing the annealing
method computes (no cost, no swap costs, no temperature) so it can feed both
the oracle and the device path without coupling them.

Recipes (all entries int32, row-major):

* ``sym_uniform(n, seed)``: A and B symmetric, zero diagonal, off-diagonal
  entries uniform integers in [0, 99].  The strict upper triangle of A is drawn
  row-major and mirrored, then the same for B, from one generator.
* ``asym_sparse_grid(n, seed)``: A asymmetric; each off-diagonal entry is
  nonzero with probability 0.4 and then uniform in [1, 99].  B holds the
  Manhattan distances between the first n cells of a row-major grid with
  ceil(sqrt(n)) columns (a 10 x 15 grid when n = 150).
* ``sym_uniform_euclid(n, seed)``: A as in ``sym_uniform``; B is
  rint(100 * Euclidean distance) between n points uniform in the unit square.

The five standard workloads (single chain N=32, N=150, N=2000, the batched mix
and the served trace) are built by ``single_chain``, ``batched_mix`` and
``served_trace``.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Chain", "sym_uniform", "asym_sparse_grid", "sym_uniform_euclid",
    "random_perm", "single_chain", "batched_mix", "served_trace", "sha256",
    "SINGLE_CHAIN_CONFIGS",
]


@dataclass
class Chain:
    """One annealing chain: an instance, its start permutation and its seeds."""
    name: str
    A: np.ndarray          # (n, n) int32 flows
    B: np.ndarray          # (n, n) int32 distances
    p0: np.ndarray         # (n,) int32 start permutation, p0[i] = location of facility i
    iters: int             # schedule length I
    philox_seed: int       # 64-bit key of the counter-based generator
    chain_id: int          # third counter word of the generator
    symmetric: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.A.shape[0])


def sha256(*arrays: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def _sym_from_upper(rng: np.random.Generator, n: int, lo: int, hi: int) -> np.ndarray:
    iu = np.triu_indices(n, k=1)
    vals = rng.integers(lo, hi + 1, size=iu[0].size, dtype=np.int64)
    M = np.zeros((n, n), dtype=np.int32)
    M[iu] = vals
    M[(iu[1], iu[0])] = vals
    return M


def sym_uniform(n: int, seed) -> tuple[np.ndarray, np.ndarray]:
    rng = np.random.default_rng(seed)
    A = _sym_from_upper(rng, n, 0, 99)
    B = _sym_from_upper(rng, n, 0, 99)
    return A, B


def _grid_manhattan(n: int, cols: int) -> np.ndarray:
    k = np.arange(n)
    y, x = k // cols, k % cols
    return (np.abs(y[:, None] - y[None, :]) + np.abs(x[:, None] - x[None, :])).astype(np.int32)


def asym_sparse_grid(n: int, seed, cols: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    rng = np.random.default_rng(seed)
    nz = rng.random((n, n)) < 0.4
    vals = rng.integers(1, 100, size=(n, n), dtype=np.int64)
    A = np.where(nz, vals, 0).astype(np.int32)
    np.fill_diagonal(A, 0)
    if cols is None:
        cols = 15 if n == 150 else int(math.ceil(math.sqrt(n)))
    B = _grid_manhattan(n, cols)
    return A, B


def sym_uniform_euclid(n: int, seed) -> tuple[np.ndarray, np.ndarray]:
    rng = np.random.default_rng(seed)
    A = _sym_from_upper(rng, n, 0, 99)
    pts = rng.random((n, 2))
    d = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    B = np.rint(100.0 * d).astype(np.int32)
    np.fill_diagonal(B, 0)
    return A, B


def random_perm(n: int, seed) -> np.ndarray:
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


# name -> (n, kind, (instance seed, p0 seed, philox seed), I)
SINGLE_CHAIN_CONFIGS = {
    "n32_sym": (32, "sym_uniform", (0, 1, 2), 10**6),
    "n150_asym": (150, "asym_sparse_grid", (10, 11, 12), 10**8),
    "n2000_sym": (2000, "sym_uniform_euclid", (20, 21, 22), 10**9),
    # the general (asymmetric) form at the same size: sparse flows on a
    # 45-column Manhattan grid, for the multi-workgroup kernel's general update
    "n2000_asym": (2000, "asym_sparse_grid", (23, 24, 25), 10**9),
}

_KIND = {
    "sym_uniform": (sym_uniform, True),
    "asym_sparse_grid": (asym_sparse_grid, False),
    "sym_uniform_euclid": (sym_uniform_euclid, True),
}


def single_chain(name: str, iters: int | None = None) -> Chain:
    """The single-chain workloads: N=32 symmetric, N=150 asymmetric sparse flow
    on a 10 x 15 Manhattan grid, and N=2000 symmetric with Euclidean distances."""
    n, kind, (s_inst, s_p, s_rng), I = SINGLE_CHAIN_CONFIGS[name]
    make, sym = _KIND[kind]
    A, B = make(n, s_inst)
    return Chain(name, A, B, random_perm(n, s_p), int(iters or I), s_rng, 0, sym,
                 {"kind": kind, "seeds": (s_inst, s_p, s_rng), "sha256": sha256(A, B)})


def batched_mix(n_instances: int = 64, chains_per_instance: int = 8, iters: int = 10**7,
                n_lo: int = 20, n_hi: int = 200, seed: int = 30) -> list[Chain]:
    """Independent chains over instances of uneven size.

    Instance sizes are uniform integers in [n_lo, n_hi] drawn from ``seed``.  The
    first half of the instances are symmetric-uniform, the second half sparse
    asymmetric on a grid.  Instance i is drawn from seed (seed, i); chain c (8
    per instance by default) starts from the permutation drawn from seed
    (seed + 1, c), uses generator key ``philox_key(seed + 2, c)`` and chain id c.
    The chains of one instance share its arrays."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=n_instances)
    chains = []
    c = 0
    for i, n in enumerate(ns):
        n = int(n)
        if i < n_instances // 2:
            A, B = sym_uniform(n, (seed, i))
            kind, sym = "sym_uniform", True
        else:
            A, B = asym_sparse_grid(n, (seed, i))
            kind, sym = "asym_sparse_grid", False
        for j in range(chains_per_instance):
            p0 = random_perm(n, (seed + 1, c))
            chains.append(Chain(f"mix{i}_{j}", A, B, p0, iters, philox_key(seed + 2, c), c, sym,
                                {"kind": kind, "instance": i}))
            c += 1
    return chains


def philox_key(base: int, index: int) -> int:
    """64-bit generator key for chain ``index`` of a family with base seed ``base``:
    the base in the high word, the index in the low word."""
    return ((base & 0xFFFFFFFF) << 32) | (index & 0xFFFFFFFF)


@dataclass
class Request:
    rid: int
    arrival_s: float
    chain: Chain


def served_trace(n_requests: int = 2000, rate: float = 200.0, iters: int = 10**7,
                 n_lo: int = 32, n_hi: int = 512, seed: int = 40) -> list[Request]:
    """Open-loop Poisson arrivals at ``rate`` requests/s; instance sizes
    log-uniform in [n_lo, n_hi].  Request j uses instance seed 1000 + 3j, start
    permutation seed 1001 + 3j and generator key 1002 + 3j, with chain id j;
    instances are symmetric-uniform."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    u = rng.random(n_requests)
    ns = np.minimum(np.floor(np.exp(np.log(n_lo) + u * (np.log(n_hi + 1) - np.log(n_lo)))), n_hi)
    out = []
    for j in range(n_requests):
        n = int(ns[j])
        A, B = sym_uniform(n, 1000 + 3 * j)
        p0 = random_perm(n, 1001 + 3 * j)
        out.append(Request(j, float(arrivals[j]),
                           Chain(f"req{j}", A, B, p0, iters, 1002 + 3 * j, j, True, {"kind": "sym_uniform"})))
    return out
