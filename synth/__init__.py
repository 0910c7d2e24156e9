"""Seeded synthetic inputs for the RLWE-PIR first-dimension scan.

This module is the only code shared by the CPU oracle and the GPU path.
It draws random numbers and nothing else: it holds none of the scheme's
arithmetic (no NTT, no modular products, no encryption).  Every value the
scheme would draw at random -- the database bytes, the ternary secret, the
uniform mask polynomials, the Gaussian errors, the queried indices -- is
produced here from a seed and handed to whichever side consumes it.

Streams.  Each object comes from its own PCG64 generator seeded through a
SeedSequence whose entropy is ``[seed, TAG, index...]``, so any row of the
database or any query can be regenerated on its own, in any order, without
drawing the others:

* database row ``i``          -> ``[seed, TAG_DB, i]``: ``C*N`` uint8, ``[C][N]``;
* secret of query ``b``       -> ``[seed, TAG_SECRET, b]``: ``N`` values in {-1,0,1};
* mask row ``i`` of query ``b`` -> ``[seed, TAG_MASK, b, i]``: one ``N``-vector
  uniform in ``[0, q_k)`` per prime, primes in the order given;
* error row ``i`` of query ``b`` -> ``[seed, TAG_ERROR, b, i]``: ``N`` rounded
  normals of standard deviation ``sigma``, resampled while ``|e| > clip``;
* queried indices             -> ``[seed, TAG_INDEX]``: ``B`` integers in ``[0, R)``;
* uniform ciphertext stand-ins -> ``[seed, TAG_UNIFORM, b, i]``: used where a
  workload needs ciphertext-shaped data without a key (an RLWE ciphertext is
  indistinguishable from uniform, so the scan sees the same distribution);
* LWE operands of ring packing: the ``a``-part matrix in blocks of 1024 rows
  ``[seed, TAG_LWE_A, block]``, client ``beta``'s ``b``-parts
  ``[seed, TAG_LWE_B, beta]`` and LWE secret ``[seed, TAG_LWE_SECRET, beta]``;
* key material of client ``beta`` for expansion and folding: the masks and
  errors of key-switching key ``level`` ``[seed, TAG_KSK_MASK|TAG_KSK_ERROR,
  beta, level, row]`` and of RGSW ciphertext ``level`` ``[seed,
  TAG_RGSW_MASK|TAG_RGSW_ERROR, beta, level, row]``, drawn like the query's.

The error clip ``|e| <= 19`` is the fresh-noise bound ``|e| < 6*sigma`` with
``sigma = 3.2`` (cryptographic background, LWE paragraph), applied to RLWE too.
"""

from __future__ import annotations

import numpy as np

TAG_DB = 0xDB
TAG_SECRET = 0x5EC
TAG_MASK = 0xA0
TAG_ERROR = 0xE0
TAG_INDEX = 0x1D
TAG_UNIFORM = 0xBE
TAG_SIZES = 0x51
TAG_FREIVALDS = 0xF5
TAG_ARRIVALS = 0xA7
TAG_LWE_A = 0x1A
TAG_LWE_B = 0x1B
TAG_LWE_SECRET = 0x15

TAG_KSK_MASK = 0x4A
TAG_KSK_ERROR = 0x4E
TAG_RGSW_MASK = 0x6A
TAG_RGSW_ERROR = 0x6E

SIGMA = 3.2
ERROR_CLIP = 19


def _rng(*entropy: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(entropy))))


def db_row(seed: int, i: int, C: int, N: int) -> np.ndarray:
    """Row ``i`` of the plaintext database: ``[C][N]`` uint8 coefficients."""
    return _rng(seed, TAG_DB, i).integers(0, 256, size=(C, N), dtype=np.uint8)


def db_bytes(seed: int, R: int, C: int, N: int, rows: range | None = None) -> np.ndarray:
    """The database ``[R][C][N]`` uint8, or the listed rows of it."""
    rows = range(R) if rows is None else rows
    out = np.empty((len(rows), C, N), dtype=np.uint8)
    for r, i in enumerate(rows):
        out[r] = db_row(seed, i, C, N)
    return out


def db_bytes_into(seed: int, out: np.ndarray, row0: int = 0) -> None:
    """Fill ``out`` (``[rows][C][N]`` uint8) with database rows starting at ``row0``."""
    _, C, N = out.shape
    for r in range(out.shape[0]):
        out[r] = db_row(seed, row0 + r, C, N)


def db_bytes_parallel(seed: int, R: int, C: int, N: int, workers: int = 16,
                      out: np.ndarray | None = None) -> np.ndarray:
    """``db_bytes`` for large databases: rows drawn on a thread pool (same bytes)."""
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty((R, C, N), dtype=np.uint8) if out is None else out

    def fill(i0: int) -> None:
        for i in range(i0, min(R, i0 + 16)):
            out[i] = db_row(seed, i, C, N)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(fill, range(0, R, 16)))
    return out


def uniform_query_parallel(seed: int, b: int, R: int, primes: list[int], N: int,
                           workers: int = 16) -> np.ndarray:
    """``uniform_query`` drawn on a thread pool (same values)."""
    from concurrent.futures import ThreadPoolExecutor
    K = len(primes)
    out = np.empty((R, 2, K, N), dtype=np.uint32)

    def fill(i0: int) -> None:
        for i in range(i0, min(R, i0 + 64)):
            g = _rng(seed, TAG_UNIFORM, b, i)
            for c in range(2):
                for k, q in enumerate(primes):
                    out[i, c, k] = g.integers(0, q, size=N, dtype=np.uint32)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(fill, range(0, R, 64)))
    return out


def poisson_arrivals(seed: int, rate: float, count: int) -> np.ndarray:
    """Arrival times (s) of ``count`` requests of a Poisson process of ``rate``/s."""
    return np.cumsum(_rng(seed, TAG_ARRIVALS, int(rate * 1000)).exponential(1.0 / rate, size=count))


def secret(seed: int, b: int, N: int) -> np.ndarray:
    """Ternary secret of query ``b``: int64 values in {-1, 0, 1}."""
    return _rng(seed, TAG_SECRET, b).integers(-1, 2, size=N, dtype=np.int64)


def _uniform(g: np.random.Generator, primes: list[int], N: int) -> np.ndarray:
    return np.stack([g.integers(0, q, size=N, dtype=np.uint64) for q in primes])


def _gaussian(g: np.random.Generator, N: int, sigma: float, clip: int) -> np.ndarray:
    e = np.rint(g.normal(0.0, sigma, size=N)).astype(np.int64)
    bad = np.abs(e) > clip
    while bad.any():
        e[bad] = np.rint(g.normal(0.0, sigma, size=int(bad.sum()))).astype(np.int64)
        bad = np.abs(e) > clip
    return e


def mask_row(seed: int, b: int, i: int, primes: list[int], N: int) -> np.ndarray:
    """Uniform mask ``a`` of ciphertext ``i`` of query ``b``: ``[K][N]`` uint64 in ``[0, q_k)``."""
    return _uniform(_rng(seed, TAG_MASK, b, i), primes, N)


def error_row(seed: int, b: int, i: int, N: int, sigma: float = SIGMA,
              clip: int = ERROR_CLIP) -> np.ndarray:
    """Rounded-Gaussian error of ciphertext ``i`` of query ``b``: ``N`` int64, ``|e| <= clip``."""
    return _gaussian(_rng(seed, TAG_ERROR, b, i), N, sigma, clip)


def key_masks(seed: int, kind: str, beta: int, level: int, rows: int, primes: list[int],
              N: int) -> np.ndarray:
    """Masks of client ``beta``'s key-switching key (``kind = "ksk"``) or RGSW ciphertext
    (``"rgsw"``) number ``level``: ``[rows][K][N]`` uint64 uniform in ``[0, q_k)``."""
    tag = {"ksk": TAG_KSK_MASK, "rgsw": TAG_RGSW_MASK}[kind]
    return np.stack([_uniform(_rng(seed, tag, beta, level, r), primes, N) for r in range(rows)])


def key_errors(seed: int, kind: str, beta: int, level: int, rows: int, N: int,
               sigma: float = SIGMA, clip: int = ERROR_CLIP) -> np.ndarray:
    """Errors of the same rows: ``[rows][N]`` int64 rounded Gaussians, ``|e| <= clip``."""
    tag = {"ksk": TAG_KSK_ERROR, "rgsw": TAG_RGSW_ERROR}[kind]
    return np.stack([_gaussian(_rng(seed, tag, beta, level, r), N, sigma, clip)
                     for r in range(rows)])


def indices(seed: int, B: int, R: int) -> np.ndarray:
    """Queried row of each of ``B`` queries: int64 in ``[0, R)``."""
    return _rng(seed, TAG_INDEX).integers(0, R, size=B, dtype=np.int64)


def uniform_query(seed: int, b: int, R: int, primes: list[int], N: int) -> np.ndarray:
    """Ciphertext-shaped uniform data for query ``b``: ``[R][2][K][N]`` uint32, entry < q_k."""
    K = len(primes)
    out = np.empty((R, 2, K, N), dtype=np.uint32)
    for i in range(R):
        g = _rng(seed, TAG_UNIFORM, b, i)
        for c in range(2):
            for k, q in enumerate(primes):
                out[i, c, k] = g.integers(0, q, size=N, dtype=np.uint32)
    return out


def batch_sizes(seed: int, n_db: int, lo: int = 1, hi: int = 64) -> np.ndarray:
    """Per-database query counts for a multi-database batch: int64 in ``[lo, hi]``."""
    return _rng(seed, TAG_SIZES).integers(lo, hi + 1, size=n_db, dtype=np.int64)


def lwe_matrix(seed: int, D1: int, n: int, p: int) -> np.ndarray:
    """The ``a``-parts of ``D1`` LWE ciphertexts (or a hint): ``[D1][n]`` uint32 uniform in
    ``[0, p)``, ``p <= 2**32``; rows drawn in blocks of 1024 from ``[seed, TAG_LWE_A, block]``."""
    out = np.empty((D1, n), dtype=np.uint32)
    for r0 in range(0, D1, 1024):
        r1 = min(D1, r0 + 1024)
        out[r0:r1] = _rng(seed, TAG_LWE_A, r0 // 1024).integers(0, p, size=(r1 - r0, n),
                                                                 dtype=np.uint64)
    return out


def lwe_offsets(seed: int, B: int, D1: int, p: int) -> np.ndarray:
    """The ``b``-parts of client ``beta``'s ``D1`` LWE ciphertexts, ``beta < B``: ``[B][D1]``
    uint32 uniform in ``[0, p)``."""
    return np.stack([_rng(seed, TAG_LWE_B, beta).integers(0, p, size=D1, dtype=np.uint64)
                     for beta in range(B)]).astype(np.uint32)


def lwe_secret(seed: int, beta: int, n: int) -> np.ndarray:
    """Client ``beta``'s LWE secret: ``n`` int64 values in {-1, 0, 1}."""
    return _rng(seed, TAG_LWE_SECRET, beta).integers(-1, 2, size=n, dtype=np.int64)


def freivalds_vector(seed: int, draw: int, C: int, q: int) -> np.ndarray:
    """Random weights for a Freivalds check: ``C`` uint64 uniform in ``[0, q)``."""
    return _rng(seed, TAG_FREIVALDS, draw, q).integers(0, q, size=C, dtype=np.uint64)
