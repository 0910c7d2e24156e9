"""Checks of full-size answers against the oracle, spread over host threads.

At the workload sizes (GiB of raw database, thousands of rows) the oracle's
plain numpy loops are too slow to run in one thread within a test's time.
These helpers only split the work: rows of an NTT, slots of a scan, rows of
a Freivalds pass go to a thread pool, and every piece is computed by the
oracle's own functions (numpy releases the interpreter lock inside them).
Nothing here does any of the scheme's arithmetic itself.
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import synth
from oracle import ntt as on
from oracle import query as oq
from oracle import scan as osc

WORKERS = min(16, os.cpu_count() or 1)


def _pool():
    return ThreadPoolExecutor(WORKERS)


def _single_thread_blas():
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(1)
    except ImportError:                                   # pragma: no cover
        import contextlib
        return contextlib.nullcontext()


def ntt_rows(x: np.ndarray, q: int, psi: int, inverse: bool = False) -> np.ndarray:
    """oracle ntt/intt of every row of ``x`` (``[..., N]``), rows split over threads."""
    shp = x.shape
    flat = np.ascontiguousarray(x, dtype=np.uint64).reshape(-1, shp[-1])
    fn = on.intt if inverse else on.ntt
    parts = np.array_split(np.arange(flat.shape[0]), max(1, min(4 * WORKERS, flat.shape[0])))
    out = np.empty_like(flat)

    def run(idx):
        if len(idx):
            out[idx[0]:idx[-1] + 1] = fn(flat[idx[0]:idx[-1] + 1], q, psi)

    with _pool() as ex:
        list(ex.map(run, parts))
    return out.reshape(shp)


def query_ntt(query: np.ndarray, primes, psis) -> np.ndarray:
    """``oracle.scan.query_ntt`` with the rows of every prime split over threads."""
    query = np.asarray(query, dtype=np.uint64)
    out = np.empty(query.shape, dtype=np.uint64)
    for k, (q, psi) in enumerate(zip(primes, psis)):
        out[..., k, :] = ntt_rows(query[..., k, :], q, psi)
    return out


def answer_intt(ans: np.ndarray, primes, psis) -> np.ndarray:
    ans = np.asarray(ans, dtype=np.uint64)
    out = np.empty(ans.shape, dtype=np.uint64)
    for k, (q, psi) in enumerate(zip(primes, psis)):
        out[..., k, :] = ntt_rows(ans[..., k, :], q, psi, inverse=True)
    return out


def db_ntt_columns(raw: np.ndarray, cols: np.ndarray, primes, psis) -> np.ndarray:
    """``oracle.scan.db_ntt(raw[:, cols])`` -> ``[K][R][len(cols)][N]``."""
    sub = np.ascontiguousarray(raw[:, cols, :]).astype(np.uint64)
    return np.stack([ntt_rows(sub, q, psi) for q, psi in zip(primes, psis)])


def db_mul(d_hat: np.ndarray, q_hat: np.ndarray, primes) -> np.ndarray:
    """``oracle.scan.db_mul`` with its slots split over threads."""
    K, R, C, N = d_hat.shape
    B = q_hat.shape[0]
    out = np.empty((B, C, 2, K, N), dtype=np.uint64)
    chunks = np.array_split(np.arange(N), min(4 * WORKERS, N))

    def run(sl):
        out[:, :, :, :, sl[0]:sl[-1] + 1] = osc.db_mul(d_hat, q_hat, primes, slots=sl)

    with _pool() as ex:
        list(ex.map(run, chunks))
    return out


def freivalds_rows(raw: np.ndarray, rs, primes_of_r) -> np.ndarray:
    """``oracle.scan.weighted_rows_multi`` over all rows of ``raw``, rows split over threads."""
    R = raw.shape[0]
    out = np.empty((len(rs), R, raw.shape[2]), dtype=np.uint64)
    blocks = [range(i, min(R, i + 16)) for i in range(0, R, 16)]

    def run(rows):
        out[:, rows.start:rows.stop] = osc.weighted_rows_multi(raw[rows.start:rows.stop], rs,
                                                               primes_of_r)

    with _single_thread_blas(), _pool() as ex:
        list(ex.map(run, blocks))
    return out


class Expected:
    """Oracle-side expectations for one database and a pool of distinct queries.

    ``pool``: ``[P][R][2][K][N]`` coefficient-form queries.  Holds, for the
    sampled columns, the exact coefficient-form answers of every pool query,
    and, for two Freivalds draws per prime, the expected weighted sums of
    every pool query's whole answer (coefficient form).
    """

    def __init__(self, rg, raw: np.ndarray, pool: np.ndarray, seed: int, n_cols: int = 16):
        self.rg, self.seed = rg, seed
        R, C, _ = raw.shape
        rng = np.random.default_rng(seed)
        extra = rng.choice(C, size=min(C, n_cols), replace=False)
        self.cols = np.unique(np.concatenate([[0, C - 1], extra]))
        q_hat = query_ntt(pool, rg.primes, rg.psis)                      # [P][R][2][K][N]
        d_hat = db_ntt_columns(raw, self.cols, rg.primes, rg.psis)
        self.cols_coeff = answer_intt(db_mul(d_hat, q_hat, rg.primes), rg.primes, rg.psis)
        # Freivalds: two draws per prime
        self.rs, self.ks = [], []
        for k, q in enumerate(rg.primes):
            for draw in range(2):
                self.rs.append(synth.freivalds_vector(seed, draw, C, q))
                self.ks.append(k)
        w = freivalds_rows(raw, self.rs, [rg.primes[k] for k in self.ks])
        self.frei = []                                                   # [V] of [P][2][N]
        for v, k in enumerate(self.ks):
            q, psi = rg.primes[k], rg.psis[k]
            e = osc.freivalds_expected_from_rows(w[v], q_hat, k, q, psi)
            self.frei.append(on.intt(e, q, psi))

    def check(self, ans_coeff: np.ndarray, member: int) -> None:
        """Assert one answer ``[C][2][K][N]`` (coefficient form) of pool query ``member``."""
        assert np.array_equal(ans_coeff[self.cols], self.cols_coeff[member]), "sampled columns"
        for v, k in enumerate(self.ks):
            q = self.rg.primes[k]
            obs = osc.freivalds_observed(ans_coeff[None], self.rs[v], k, q)[0]
            assert np.array_equal(obs, self.frei[v][member]), f"Freivalds draw {v}"

    def decrypts(self, ans_coeff: np.ndarray, secret: np.ndarray, raw: np.ndarray,
                 i_star: int) -> None:
        rg = self.rg
        m, _ = oq.decrypt_answers(ans_coeff[self.cols], secret, rg.primes, rg.psis, rg.delta,
                                  rg.p)
        assert np.array_equal(m, raw[i_star, self.cols].astype(np.int64)), "decryption"
