"""Seeded synthetic inputs for fast count sketch workloads.

This module only draws random numbers and shapes; it holds none of the
sketch's arithmetic (no hashing, no sketching).  It is the one module that
both the oracle-side tests and the GPU-side tests and bench read inputs from,
so that both sides see identical float32 values.

Every generator is ``numpy.random.Generator(PCG64(seed))``.  Workloads follow
the synthetic set-ups of the paper (Gaussian CP factors, Gaussian dense
tensors, uniform [-5, 5] Kronecker factors, Section 4) at the sizes of the
five benchmark configurations:

* ``cp100``      order 3, I_n = 100, R = 10, J_n = 64 (J~ = 190), D = 5
* ``dense1024``  order 3, 1024^3 float32 N(0,1), J_n = 4096 (J~ = 12286), D = 8,
                 plus a 10 % Bernoulli-masked COO copy with int32 coordinates
* ``cp10k``      order 3, I_n = 10^4, R = 512, unit-norm N(0,1) columns,
                 J_n = 2^14, D = 10, 64 unit vector pairs for T(I, u, v)
* ``batch4096``  4096 uneven CP instances (N in {3,4,5}, I_n log-uniform in
                 [32, 4096], R in [1, 256], J_n = 2^{8..13}), every 16th a
                 Kronecker instance of two 256 x 256 U[-5, 5] matrices
* ``serve``      Poisson request streams over the shapes above
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 22          # entries per independently seeded chunk
_WORKERS = max(1, min(16, os.cpu_count() or 1))

DATA_SEED = {"cp100": 1001, "dense1024": 1002, "cp10k": 1003, "batch4096": 1004,
             "serve": 1005, "rtpm100": 1006,
             "als400": 1007, "rtpm50": 1008, "rtpm_asym100": 1009}
HASH_SEED = {"cp100": 2001, "dense1024": 2002, "cp10k": 2003, "batch4096": 2004,
             "serve": 2005, "rtpm100": 2006,
             "als400": 2007, "rtpm50": 2008, "rtpm_asym100": 2009}


def rng(seed: int, *stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed, *stream] if stream else seed))


# ----------------------------------------------------------------------------
# primitive draws
# ----------------------------------------------------------------------------
def cp_factors(seed: int, I, R: int, normalize: bool = False, stream: int = 0):
    """N factor matrices U_n (I_n x R), float64 N(0,1) draws cast to float32;
    with ``normalize`` every column is scaled to unit 2-norm first."""
    g = rng(seed, stream)
    out = []
    for I_n in I:
        u = g.standard_normal((int(I_n), int(R)))
        if normalize:
            u = u / np.linalg.norm(u, axis=0, keepdims=True)
        out.append(u.astype(np.float32))
    return out


def _chunked(n: int, seed: int, stream: int, fill) -> None:
    """Run fill(generator, start, end) over CHUNK-sized pieces of [0, n), each
    with its own PCG64 stream (seed, stream, chunk), on a thread pool; the
    result does not depend on the number of threads."""
    chunks = list(range((n + CHUNK - 1) // CHUNK))

    def one(k):
        s = k * CHUNK
        fill(rng(seed, stream, k), s, min(s + CHUNK, n))

    if len(chunks) <= 1:
        for k in chunks:
            one(k)
        return
    with ThreadPoolExecutor(_WORKERS) as ex:
        list(ex.map(one, chunks))


def dense_tensor(seed: int, I, stream: int = 0) -> np.ndarray:
    """vec(T) (mode 0 fastest) of a float32 N(0,1) tensor, drawn directly in
    float32, chunk by chunk."""
    n = int(np.prod([int(i) for i in I]))
    out = np.empty(n, dtype=np.float32)
    _chunked(n, seed, stream, lambda g, s, e: g.standard_normal(e - s, dtype=np.float32, out=out[s:e]))
    return out


def integer_tensor(seed: int, I, lo: int = -3, hi: int = 3, stream: int = 0):
    """Small-integer tensor (float32) whose every partial sum is exact."""
    n = int(np.prod([int(i) for i in I]))
    out = np.empty(n, dtype=np.float32)

    def fill(g, s, e):
        out[s:e] = g.integers(lo, hi + 1, size=e - s)

    _chunked(n, seed, stream, fill)
    return out


def bernoulli_coo(seed: int, T_vec: np.ndarray, I, density: float, stream: int = 1):
    """Keep each linear index with probability ``density`` (seeded, chunked);
    returns (idx int32 [N][nnz] mode-major, val float32 [nnz]) sorted by
    linear index."""
    I = [int(i) for i in I]
    total = T_vec.size
    nchunks = (total + CHUNK - 1) // CHUNK
    keep = [None] * nchunks

    def fill(g, s, e):
        keep[s // CHUNK] = np.flatnonzero(g.random(e - s, dtype=np.float32) < density).astype(np.int64) + s

    _chunked(total, seed, stream, fill)
    lin = np.concatenate(keep) if keep else np.zeros(0, np.int64)
    val = T_vec[lin].astype(np.float32)
    idx = np.empty((len(I), lin.size), dtype=np.int32)
    rem = lin
    for n, I_n in enumerate(I):
        idx[n] = (rem % I_n).astype(np.int32)
        rem = rem // I_n
    return idx, val


def unit_vectors(seed: int, count: int, size: int, stream: int = 0) -> np.ndarray:
    """``count`` x ``size`` float32 rows, N(0,1) draws scaled to unit norm."""
    v = rng(seed, stream).standard_normal((count, size))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v.astype(np.float32)


def uniform_matrix(seed: int, shape, lo=-5.0, hi=5.0, stream: int = 0):
    return rng(seed, stream).uniform(lo, hi, size=shape).astype(np.float32)


def orthonormal_columns(seed: int, size: int, count: int, stream: int = 0) -> np.ndarray:
    """``size`` x ``count`` float64 matrix with orthonormal columns: the Q
    factor of a Gaussian draw, signs fixed by R's diagonal (a random
    orthonormal basis)."""
    q, r = np.linalg.qr(rng(seed, stream).standard_normal((int(size), int(count))))
    return q * np.sign(np.diag(r))


def symmetric_cp_tensor(seed: int, size: int, weights, noise: float = 0.0, stream: int = 0):
    """The order-3 tensor sum_r w_r a_r o a_r o a_r of the RTPM experiments
    (a_r orthonormal columns of ``orthonormal_columns``) plus i.i.d.
    N(0, noise^2) entries.  Returns (vec(T) float64 with mode 0 fastest,
    A = [a_0 .. a_{R-1}] size x R)."""
    w = np.asarray(weights, dtype=np.float64)
    A = orthonormal_columns(seed, size, len(w), stream)
    T = np.einsum("r,ir,jr,kr->ijk", w, A, A, A)
    if noise:
        T = T + noise * rng(seed, stream + 1).standard_normal(T.shape)
    return T.reshape(-1, order="F"), A


def asymmetric_cp_tensor(seed: int, size: int, weights, noise: float = 0.0, stream: int = 0):
    """The order-3 tensor sum_r w_r a_r o b_r o c_r of the ALS experiment
    (each factor a set of orthonormal columns, drawn independently) plus
    i.i.d. N(0, noise^2) entries.  Returns (vec(T) float64 with mode 0
    fastest, [A, B, C])."""
    w = np.asarray(weights, dtype=np.float64)
    F = [orthonormal_columns(seed, size, len(w), stream + 3 * k) for k in range(3)]
    T = np.einsum("r,ir,jr,kr->ijk", w, *F)
    if noise:
        T = T + noise * rng(seed, stream + 1).standard_normal(T.shape)
    return T.reshape(-1, order="F"), F


def als_init(seed: int, size: int, rank: int, stream: int = 0):
    """Three float32 size x rank starting factors of ALS, N(0, 1) entries."""
    g = rng(seed, stream)
    return [g.standard_normal((int(size), int(rank))).astype(np.float32) for _ in range(3)]


def rtpm_asym_starts(seed: int, rank: int, count: int, size: int, stream: int = 0) -> np.ndarray:
    """rank x count x 3 x size float32 unit starting vectors of the
    alternating rank-1 updates (one triple per start)."""
    return unit_vectors(seed, rank * count * 3, size, stream).reshape(int(rank), int(count), 3, int(size))


def rtpm_starts(seed: int, rank: int, count: int, size: int, stream: int = 0) -> np.ndarray:
    """rank x count x size float32 unit starting vectors of the power
    iterations (one set per component)."""
    return unit_vectors(seed, rank * count, size, stream).reshape(int(rank), int(count), int(size))


# ----------------------------------------------------------------------------
# benchmark configurations
# ----------------------------------------------------------------------------
@dataclass
class CPConfig:
    name: str
    I: tuple
    J: tuple
    R: int
    D: int
    normalize: bool
    data_seed: int
    hash_seed: int
    pairs: int = 0

    def factors(self, stream: int = 0):
        return cp_factors(self.data_seed, self.I, self.R, self.normalize, stream)


CP100 = CPConfig("cp100", (100, 100, 100), (64, 64, 64), 10, 5, False,
                 DATA_SEED["cp100"], HASH_SEED["cp100"])
CP10K = CPConfig("cp10k", (10000, 10000, 10000), (16384, 16384, 16384), 512, 10,
                 True, DATA_SEED["cp10k"], HASH_SEED["cp10k"], pairs=64)


@dataclass
class DenseConfig:
    name: str
    I: tuple
    J: tuple
    D: int
    data_seed: int
    hash_seed: int
    density: float = 0.1


DENSE1024 = DenseConfig("dense1024", (1024, 1024, 1024), (4096, 4096, 4096), 8,
                        DATA_SEED["dense1024"], HASH_SEED["dense1024"])


@dataclass
class Instance:
    """One CP (or Kronecker) sketch request of the uneven batch."""
    index: int
    kind: str            # "cp" or "kron"
    I: tuple
    J: tuple
    R: int
    D: int = 1
    seed: int = 0        # data seed of this instance
    hash_seed: int = 0
    extra: dict = field(default_factory=dict)

    def factors(self):
        if self.kind == "kron":
            A = uniform_matrix(self.seed, (self.I[0], self.I[1]), stream=1)
            B = uniform_matrix(self.seed, (self.I[2], self.I[3]), stream=2)
            return [A, B]
        return cp_factors(self.seed, self.I, self.R, False, stream=0)


def batch_instances(count: int = 4096, seed: int = DATA_SEED["batch4096"],
                    hash_seed: int = HASH_SEED["batch4096"], kron_every: int = 16,
                    I_range=(32, 4096), R_range=(1, 256), logJ_range=(8, 13)):
    """The uneven batch: instance k draws its shape from stream (seed, k)."""
    out = []
    lo, hi = np.log(I_range[0]), np.log(I_range[1])
    for k in range(count):
        g = rng(seed, 7, k)
        if kron_every and k % kron_every == kron_every - 1:
            Jk = int(2 ** g.integers(logJ_range[0], logJ_range[1] + 1))
            out.append(Instance(k, "kron", (256, 256, 256, 256), (Jk,) * 4, 1,
                                seed=seed * 1000003 + k, hash_seed=hash_seed + k))
            continue
        N = int(g.integers(3, 6))
        I = tuple(int(np.exp(g.uniform(lo, hi))) for _ in range(N))
        R = int(g.integers(R_range[0], R_range[1] + 1))
        J = tuple(int(2 ** g.integers(logJ_range[0], logJ_range[1] + 1))
                  for _ in range(N))
        out.append(Instance(k, "cp", I, J, R, seed=seed * 1000003 + k,
                            hash_seed=hash_seed + k))
    return out


def instance_inputs(instances, workers: int = _WORKERS):
    """Factors of every instance, drawn in parallel (numpy releases the GIL
    while drawing); yields (instance, factors) in order."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        for ins, f in zip(instances, ex.map(lambda i: i.factors(), instances)):
            yield ins, f


def poisson_arrivals(seed: int, rate: float, count: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: cumulative exponential gaps."""
    return np.cumsum(rng(seed, 11).exponential(1.0 / rate, size=count))


SERVE_MIX = (0.90, 0.08, 0.02)      # contraction, CP build, COO sketch


def serving_requests(seed: int, rate: float, count: int, n_pairs: int, n_cp: int, n_coo: int,
                     mix=SERVE_MIX):
    """(arrival s, kind, input index) of a Poisson request stream: kinds
    drawn with probabilities `mix`, each referring to one of the pre-staged
    inputs (vector pairs, CP factor sets, COO tensors) uniformly."""
    t = poisson_arrivals(seed, rate, count)
    g = rng(seed, 12)
    kinds = g.choice(3, size=count, p=np.asarray(mix) / np.sum(mix))
    idx = np.where(kinds == 0, g.integers(0, n_pairs, size=count),
                   np.where(kinds == 1, g.integers(0, n_cp, size=count), g.integers(0, n_coo, size=count)))
    names = ("contract", "cp", "coo")
    return [(float(t[k]), names[int(kinds[k])], int(idx[k])) for k in range(count)]


def coo_nnz_sizes(seed: int, count: int, lo: float = 1e4, hi: float = 1e8) -> list:
    """nnz of the pre-staged COO tensors: log-uniform in [lo, hi]."""
    g = rng(seed, 13)
    return [int(np.exp(g.uniform(np.log(lo), np.log(hi)))) for _ in range(count)]


# ----------------------------------------------------------------------------
# inputs with a wide dynamic range (scales vary across rows and entries)
# ----------------------------------------------------------------------------
WIDE_KINDS = ("spike", "spike_each_slab", "leading_rows_large", "rows_after_16_small",
              "log_uniform_rows", "decaying_rows", "zero_head_tiny")


def wide_range_tensor(seed: int, I, kind: str, stream: int = 0) -> np.ndarray:
    """vec(T) (mode 0 fastest) of a float32 tensor whose magnitudes vary
    widely across its rows (mode-0 fibres).  A slab is the set of rows that
    share the last-mode index; ``r`` below is a row's position in its slab.

    * ``spike``: N(0, 1e-6) variance entries (sd 1e-3) and a single entry
      1e3 in row 3 of the first slab;
    * ``spike_each_slab``: the same with one 1e3 entry in row 3 of every slab;
    * ``leading_rows_large``: N(0,1), rows r < 16 of every slab times 100;
    * ``rows_after_16_small``: N(0,1), rows r >= 16 times 1e-2;
    * ``log_uniform_rows``: N(0,1), each row times 10^U(-3, 3);
    * ``decaying_rows``: N(0,1), row r times 2^(-r/8);
    * ``zero_head_tiny``: rows r < 16 zero, the others N(0, 1e-12) (sd 1e-6).
    """
    I = [int(i) for i in I]
    I0 = I[0]
    rows = int(np.prod(I[1:]))
    slab = int(np.prod(I[1:-1]))
    T = dense_tensor(seed, I, stream).reshape(rows, I0)
    r = (np.arange(rows) % slab)
    g = rng(seed, stream, 99)
    if kind in ("spike", "spike_each_slab"):
        T *= np.float32(1e-3)
        hot = [3 % slab] if kind == "spike" else list(range(3 % slab, rows, slab))
        for row in hot:
            T[row, 17 % I0] = np.float32(1e3)
    elif kind == "leading_rows_large":
        T[r < 16] *= np.float32(100.0)
    elif kind == "rows_after_16_small":
        T[r >= 16] *= np.float32(1e-2)
    elif kind == "log_uniform_rows":
        T *= (10.0 ** g.uniform(-3.0, 3.0, rows)).astype(np.float32)[:, None]
    elif kind == "decaying_rows":
        T *= (2.0 ** (-r / 8.0)).astype(np.float32)[:, None]
    elif kind == "zero_head_tiny":
        T *= np.float32(1e-6)
        T[r < 16] = 0.0
    else:
        raise ValueError(f"unknown kind {kind!r}")
    return np.ascontiguousarray(T.reshape(-1))


def wide_range_values(seed: int, nnz: int, kind: str, head: int = 16384) -> np.ndarray:
    """COO values with a wide dynamic range: ``large_head`` (N(0,1) with the
    first ``head`` values times 1e3), ``zero_head_tiny`` (first ``head`` zero,
    the rest N(0,1) times 1e-6), ``log_uniform`` (N(0,1) times 10^U(-6, 6))."""
    g = rng(seed, 5)
    v = g.standard_normal(nnz)
    if kind == "large_head":
        v[:head] *= 1e3
    elif kind == "zero_head_tiny":
        v *= 1e-6
        v[:head] = 0.0
    elif kind == "log_uniform":
        v *= 10.0 ** g.uniform(-6.0, 6.0, nnz)
    else:
        raise ValueError(f"unknown kind {kind!r}")
    return v.astype(np.float32)
