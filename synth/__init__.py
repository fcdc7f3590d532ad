"""Seeded synthetic inputs shaped like the paper's retrieval workloads.

This module only draws random numbers and lays them out. It contains none of
the search method's arithmetic (no distances, no clustering, no selection), so
both the FP64 oracle and the GPU library can take their inputs from it without
sharing any code with each other.

Recipe (the paper trains encoders on ImageNet-1K and Natural Questions, which
are not available; these mixtures stand in for their embeddings, see Section 3
"Datasets" and Appendix C for the shapes):

* ``ncomp`` component means ``g_c ~ N(0, I_d)``, uniform component weights.
* A row of component ``c`` is ``x = s * (g_c + sigma * eps)`` with
  ``eps ~ N(0, I_d)`` and the decaying spectrum ``s_i = (i + 1) ** -0.5``
  (0-based ``i``), so that a prefix ``x[:m]`` carries most of the energy,
  like a Matryoshka representation (Section 3, "Matryoshka Representations").
* Every row is then L2-normalised.
* Queries use the same component means with their own noise stream.

Determinism: every stream is a ``numpy.random.SeedSequence`` child keyed by
(root seed, stream id, chunk index); rows are produced in fixed chunks of
``CHUNK_ROWS`` and any chunk can be regenerated on its own, so the output does
not depend on how many threads produce it.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 19435
CHUNK_ROWS = 65536

# stream ids
STREAM_MEANS = 0
STREAM_DB = 1
STREAM_QUERIES = 2
STREAM_KMEANS_INIT = 3
STREAM_PQ = 4
STREAM_MISC = 5


def _rng(seed: int, stream: int, chunk: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence(entropy=seed, spawn_key=(stream, chunk))
    return np.random.Generator(np.random.PCG64(ss))


def spectrum(d: int) -> np.ndarray:
    """Per-dimension scale s_i = (i+1)^-1/2, float32."""
    return ((np.arange(d, dtype=np.float64) + 1.0) ** -0.5).astype(np.float32)


@dataclass(frozen=True)
class Mixture:
    """A seeded Gaussian mixture in R^d with a decaying spectrum."""

    d: int
    ncomp: int
    seed: int = ROOT_SEED
    sigma: float = 1.0
    _means: np.ndarray | None = field(default=None, compare=False, repr=False)

    def means(self) -> np.ndarray:
        # cached per instance via object.__setattr__ (frozen dataclass)
        if self._means is None:
            m = _rng(self.seed, STREAM_MEANS).standard_normal(
                (self.ncomp, self.d), dtype=np.float32)
            object.__setattr__(self, "_means", m)
        return self._means

    def _chunk(self, stream: int, chunk: int, rows: int, out: np.ndarray):
        rng = _rng(self.seed, stream, chunk)
        labels = rng.integers(0, self.ncomp, size=rows)
        noise = rng.standard_normal((rows, self.d), dtype=np.float32)
        if self.sigma != 1.0:
            noise *= np.float32(self.sigma)
        noise += self.means()[labels]
        noise *= spectrum(self.d)[None, :]
        nrm = np.sqrt(np.einsum("ij,ij->i", noise, noise, dtype=np.float32))
        noise /= nrm[:, None]
        out[...] = noise.astype(out.dtype, copy=False)
        return labels

    def rows(self, stream: int, n: int, dtype=np.float32, threads: int | None = None,
             return_labels: bool = False):
        """Rows [0, n) of ``stream`` as a C-contiguous [n, d] array."""
        out = np.empty((n, self.d), dtype=dtype)
        labels = np.empty(n, dtype=np.int64)
        nchunks = (n + CHUNK_ROWS - 1) // CHUNK_ROWS

        def work(c):
            a, b = c * CHUNK_ROWS, min(n, (c + 1) * CHUNK_ROWS)
            labels[a:b] = self._chunk(stream, c, b - a, out[a:b])

        if threads is None:
            threads = min(16, os.cpu_count() or 1)
        if nchunks <= 1 or threads <= 1:
            for c in range(nchunks):
                work(c)
        else:
            with ThreadPoolExecutor(threads) as ex:
                list(ex.map(work, range(nchunks)))
        return (out, labels) if return_labels else out

    def database(self, n: int, dtype=np.float32, threads=None, return_labels=False):
        return self.rows(STREAM_DB, n, dtype, threads, return_labels)

    def queries(self, nq: int, dtype=np.float32, threads=None, return_labels=False):
        return self.rows(STREAM_QUERIES, nq, dtype, threads, return_labels)


def init_rows(n: int, count: int, seed: int = ROOT_SEED, stream: int = STREAM_KMEANS_INIT,
              tag: int = 0) -> np.ndarray:
    """The first ``count`` entries of a seeded permutation of range(n).

    Lloyd's iteration starts from these rows; the draw is made here and handed
    to both implementations as an input.
    """
    if count > n:
        raise ValueError("count > n")
    rng = _rng(seed, stream, tag)
    return rng.permutation(n)[:count].astype(np.int32)


def subsample_rows(n: int, count: int, seed: int = ROOT_SEED, tag: int = 0) -> np.ndarray:
    """Sorted seeded subsample of row indices (training subsets)."""
    return np.sort(init_rows(n, count, seed, STREAM_MISC, tag)).astype(np.int64)


def random_rotation(d: int, seed: int = ROOT_SEED, tag: int = 0) -> np.ndarray:
    """A seeded random orthonormal d x d matrix (float32): the Q factor of a
    Gaussian matrix with the signs of R's diagonal folded in (Haar measure)."""
    g = _rng(seed, STREAM_PQ, 1000 + tag).standard_normal((d, d))
    q, r = np.linalg.qr(g)
    return (q * np.sign(np.diag(r))[None, :]).astype(np.float32)


# ---- named workloads (sizes of the paper's experiments; Section 3, Appendix C) ----

@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    d: int
    ncomp: int
    nq: int
    nlist: int
    d_c: int
    d_s: int
    nprobe: int
    k: int
    seed: int = ROOT_SEED
    dtype: str = "float32"

    def mixture(self) -> Mixture:
        return Mixture(self.d, self.ncomp, self.seed)


WORKLOADS = {
    # small CPU-scale case: 10k x 64, 100 components, 100 queries, nlist 32 on d_c=16
    "small": Workload("small", 10_000, 64, 100, 100, 32, 16, 64, 4, 10, seed=ROOT_SEED),
    # ImageNet-1K shape: 1,281,167 x 2048, 1000 components, 50k queries, nlist 1024
    "imagenet1k": Workload("imagenet1k", 1_281_167, 2048, 1000, 50_000, 1024, 64, 2048, 8, 10,
                           seed=ROOT_SEED + 1),
    # batching-form database: 1M x 1024
    "batching1m": Workload("batching1m", 1_000_000, 1024, 1000, 4096, 1024, 64, 1024, 16, 10,
                           seed=ROOT_SEED + 3),
    # NQ shape (fp16 storage): 21M x 768, 4096 components, nlist 16384 on d_c=64
    "nq21m": Workload("nq21m", 21_000_000, 768, 4096, 3610, 16384, 64, 768, 16, 10,
                      seed=ROOT_SEED + 4, dtype="float16"),
}
