"""The first-dimension scan of poly-HE folding, by its definition.

Paper basis.  Poly-HE folding starts with the database lifted from ``R_p`` to
``R_q`` and transformed by the NTT (Sec. 2.4, plaintext bloating; Sec. 3.2,
step 5), then multiplies each database polynomial with the ciphertext of
its row and sums down the rows (Sec. 3.2, step 6; Eq. he-linear):

    answer_j = sum_i DB[i][j] * ct_i        in R_q^2, for every column j.

With RNS and the NTT this is, for every prime ``q_k`` and NTT slot ``t``, an
exact modular matrix product (Sec. 4, "INT32 modular GEMM"; the
``(#RNS*N)``-parallel GEMMs of Sec. 3.5):

    Y[b][j][c][k][t] = sum_i Dhat[k][i][j][t] * Qhat[b][i][c][k][t]  (mod q_k)

for query ``b``, column ``j``, ciphertext component ``c``.  The drain is the
inverse NTT of ``Y`` back to coefficient form.

Layouts (the library's boundary uses the same ones):
  raw DB ``[R][C][N]`` uint8; query ``[B][R][2][K][N]``; answer ``[B][C][2][K][N]``.

Lift reading: a database byte ``v`` becomes ``v`` in ``Z_q`` (the unsigned
representative; the paper says only that plaintexts are lifted).
"""

from __future__ import annotations

import numpy as np

from . import ntt as _ntt


def db_ntt(raw: np.ndarray, primes: list[int], psis: list[int]) -> np.ndarray:
    """Lift + NTT every database polynomial: ``[R][C][N]`` uint8 -> ``[K][R][C][N]`` uint64."""
    raw = np.asarray(raw)
    out = np.empty((len(primes),) + raw.shape, dtype=np.uint64)
    for k, (q, psi) in enumerate(zip(primes, psis)):
        out[k] = _ntt.ntt(raw.astype(np.uint64), q, psi)
    return out


def query_ntt(query: np.ndarray, primes: list[int], psis: list[int]) -> np.ndarray:
    """Forward NTT of every query polynomial, per prime: ``[..., K, N]`` -> same shape."""
    query = np.asarray(query, dtype=np.uint64)
    out = np.empty(query.shape, dtype=np.uint64)
    for k, (q, psi) in enumerate(zip(primes, psis)):
        out[..., k, :] = _ntt.ntt(query[..., k, :], q, psi)
    return out


def answer_intt(ans: np.ndarray, primes: list[int], psis: list[int]) -> np.ndarray:
    """Inverse NTT of every answer polynomial, per prime: ``[..., K, N]`` -> same shape."""
    ans = np.asarray(ans, dtype=np.uint64)
    out = np.empty(ans.shape, dtype=np.uint64)
    for k, (q, psi) in enumerate(zip(primes, psis)):
        out[..., k, :] = _ntt.intt(ans[..., k, :], q, psi)
    return out


def db_mul(db_hat: np.ndarray, q_hat: np.ndarray, primes: list[int],
           slots: np.ndarray | None = None, cols: np.ndarray | None = None) -> np.ndarray:
    """The scan in NTT form, by definition: a running sum over rows, reduced after every term.

    ``db_hat``: ``[K][R][C][N]``; ``q_hat``: ``[B][R][2][K][N]``.  Returns
    ``[B][C'][2][K][N']`` uint64 where ``C'``/``N'`` are the selected columns/slots
    (all by default).
    """
    K, R, C, N = db_hat.shape
    B = q_hat.shape[0]
    slots = np.arange(N) if slots is None else np.asarray(slots)
    cols = np.arange(C) if cols is None else np.asarray(cols)
    out = np.zeros((B, len(cols), 2, K, len(slots)), dtype=np.uint64)
    for k, q in enumerate(primes):
        qq = np.uint64(q)
        acc = np.zeros((B, len(cols), 2, len(slots)), dtype=np.uint64)
        for i in range(R):
            d = db_hat[k, i][np.ix_(cols, slots)]              # [C'][N']
            qv = q_hat[:, i, :, k, :][:, :, slots]              # [B][2][N']
            acc = (acc + d[None, :, None, :] * qv[:, None, :, :]) % qq
        out[:, :, :, k, :] = acc
    return out


def db_mul_coeff(raw: np.ndarray, query: np.ndarray, primes: list[int]) -> np.ndarray:
    """The scan in coefficient form by the ring definition (schoolbook negacyclic products).

    ``sum_i DB[i][j] * ct[b][i][c]`` in ``R_q``, for tiny sizes only.  ``raw``:
    ``[R][C][N]``; ``query``: ``[B][R][2][K][N]`` -> ``[B][C][2][K][N]``.
    """
    R, C, N = raw.shape
    B = query.shape[0]
    K = len(primes)
    out = np.zeros((B, C, 2, K, N), dtype=np.uint64)
    for b in range(B):
        for j in range(C):
            for c in range(2):
                for k, q in enumerate(primes):
                    acc = [0] * N
                    for i in range(R):
                        prod = _ntt.negacyclic_schoolbook(raw[i, j], query[b, i, c, k], q)
                        acc = [(x + y) % q for x, y in zip(acc, prod)]
                    out[b, j, c, k] = acc
    return out


def weighted_rows(raw_rows: np.ndarray, r: np.ndarray, q: int) -> np.ndarray:
    """``sum_j r_j * DB[i][j] (mod q)`` for every row given: ``[R'][C][N]`` uint8 -> ``[R'][N]`` uint64.

    Exact: ``r`` is split in 14-bit halves so every partial sum (at most
    ``C * 2**14 * 255 < 2**53`` for ``C < 2**31``) is an integer a float64
    matrix product represents exactly.
    """
    C = raw_rows.shape[1]
    if C >= 1 << 31:
        raise ValueError("C too large for the exact float64 bound")
    r = np.asarray(r, dtype=np.uint64) % np.uint64(q)
    lo = (r & np.uint64(0x3FFF)).astype(np.float64)
    hi = (r >> np.uint64(14)).astype(np.float64)
    out = np.empty((raw_rows.shape[0], raw_rows.shape[2]), dtype=np.uint64)
    for ii in range(raw_rows.shape[0]):
        x = raw_rows[ii].astype(np.float64)                   # [C][N]
        s_lo = (lo @ x).astype(np.uint64) % np.uint64(q)
        s_hi = (hi @ x).astype(np.uint64) % np.uint64(q)
        out[ii] = (s_lo + (s_hi << np.uint64(14)) % np.uint64(q)) % np.uint64(q)
    return out


def weighted_rows_multi(raw_rows: np.ndarray, rs: list[np.ndarray], primes: list[int]) -> np.ndarray:
    """``weighted_rows`` for several (weights, prime) pairs in one pass over the rows.

    Returns ``[V][R'][N]`` uint64 with entry ``[v][i] = sum_j rs[v][j] * DB[i][j] (mod primes[v])``.
    The same exact float64 products as ``weighted_rows`` (14-bit halves of every
    weight vector stacked into one matrix), so each row is converted once.
    """
    C = raw_rows.shape[1]
    if C >= 1 << 31:
        raise ValueError("C too large for the exact float64 bound")
    V = len(rs)
    qq = [np.uint64(q) for q in primes]
    red = [np.asarray(r, dtype=np.uint64) % q for r, q in zip(rs, qq)]
    W = np.stack([(r & np.uint64(0x3FFF)).astype(np.float64) for r in red] +
                 [(r >> np.uint64(14)).astype(np.float64) for r in red])        # [2V][C]
    out = np.empty((V, raw_rows.shape[0], raw_rows.shape[2]), dtype=np.uint64)
    for ii in range(raw_rows.shape[0]):
        s = (W @ raw_rows[ii].astype(np.float64)).astype(np.uint64)           # [2V][N]
        for v in range(V):
            lo, hi = s[v] % qq[v], s[V + v] % qq[v]
            out[v, ii] = (lo + (hi << np.uint64(14)) % qq[v]) % qq[v]
    return out


def freivalds_expected_from_rows(w: np.ndarray, q_hat: np.ndarray, k: int, q: int,
                                 psi: int) -> np.ndarray:
    """``freivalds_expected`` from weighted rows ``w`` = ``weighted_rows(raw, r, q)`` (``[R][N]``)."""
    qq = np.uint64(q)
    w_hat = _ntt.ntt(w, q, psi)
    B = q_hat.shape[0]
    acc = np.zeros((B, 2, w.shape[1]), dtype=np.uint64)
    for i in range(w.shape[0]):
        acc = (acc + w_hat[i][None, None, :] * q_hat[:, i, :, k, :]) % qq
    return acc


def freivalds_expected(raw: np.ndarray, q_hat: np.ndarray, r: np.ndarray, k: int,
                       q: int, psi: int) -> np.ndarray:
    """``sum_j r_j Y[b][j][c][k][t]`` computed without ``Y``, by linearity of the NTT.

    ``sum_j r_j Y_t[j] = sum_i NTT(sum_j r_j lift(DB[i][j]))[t] * Qhat_t[i] (mod q_k)``.
    Returns ``[B][2][N]`` uint64.  ``raw``: ``[R][C][N]``; ``q_hat``: ``[B][R][2][K][N]``.
    """
    qq = np.uint64(q)
    w = weighted_rows(raw, r, q)                               # [R][N]
    w_hat = _ntt.ntt(w, q, psi)                                # [R][N]
    B = q_hat.shape[0]
    acc = np.zeros((B, 2, raw.shape[2]), dtype=np.uint64)
    for i in range(raw.shape[0]):
        acc = (acc + w_hat[i][None, None, :] * q_hat[:, i, :, k, :]) % qq
    return acc


def freivalds_observed(ans_ntt: np.ndarray, r: np.ndarray, k: int, q: int) -> np.ndarray:
    """``sum_j r_j Y[b][j][c][k][t] (mod q)`` from an NTT-form answer ``[B][C][2][K][N]``."""
    qq = np.uint64(q)
    rr = np.asarray(r, dtype=np.uint64) % qq
    B, C, _, _, N = ans_ntt.shape
    acc = np.zeros((B, 2, N), dtype=np.uint64)
    for j in range(C):
        acc = (acc + rr[j] * (np.asarray(ans_ntt[:, j, :, k, :], dtype=np.uint64) % qq)) % qq
    return acc
