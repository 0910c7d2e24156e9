"""Tiptoe-style ring packing of LWE ciphertexts into RLWE ciphertexts.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper basis (App. C.1, Eq. tiptoe-rp; Sec. 3.5, "Massive parallelism").  A
client's N LWE ciphertexts with mask rows ``A`` (``N x n`` over ``Z_p``) and
offsets ``b`` have the phase ``b + A s``.  Splitting ``A`` into its columns
``A_i`` writes that phase as ``b + sum_i A_i s_i``.  With ``iota`` mapping a
length-N vector to the polynomial whose coefficients it holds, and ``n``
RLWE ciphertexts ``ct_i`` encrypting ``s_i`` (the "special" ciphertexts),
the server evaluates

    ct_res = (0, Delta * iota(b)) + sum_i iota(A_i) * ct_i        in R_Q^2,

whose phase is ``Delta * iota(b + A s)`` plus ``sum_i iota(A_i) e_i``: it
decrypts to the N LWE phases at once.  For SimplePIR's ``D1`` answers the
``D1`` rows are cut into ``ceil(D1/N)`` chunks of N, one packed ciphertext per
chunk and client.  After the NTT this is the matrix product of Sec. 3.5,
``H * C + (0 | G)``: ``H`` the ``ceil(D1/N) x n`` matrix of transformed
``iota(A_{r,i})``, ``C`` the ``n x 2B`` matrix of the B clients' special
ciphertexts (component 0 and 1 as columns), ``G`` the transformed
``Delta * iota(b)``, added to the ``b``-component columns only.

Readings where the paper is loose:
* chunk ``r`` of column ``i`` is the polynomial with coefficient ``j`` =
  ``A[r N + j][i]`` (rows past ``D1`` are zero), and likewise for ``b``;
* ``Z_p`` values are lifted to ``Z_Q`` unsigned (``v`` stays ``v``), as the
  database bytes are, and ``Delta = floor(Q / p)`` (App. A.2);
* the plaintext modulus is a power of two ``p = 2^t``; the LWE modulus and
  the RLWE plaintext modulus are the same ``p`` (App. C).

Layouts: ``A`` ``[D1][n]``; ``b`` ``[B][D1]``; special ciphertexts
``[B][n][2][K][N]`` (coefficient form); packed result ``[B][C'][2][K][N]``,
``C' = ceil(D1/N)``.
"""

from __future__ import annotations

import numpy as np

from . import ntt as _ntt
from . import scan as _scan
from .params import scale


def n_chunks(D1: int, N: int) -> int:
    return -(-D1 // N)


def hint_polys(A: np.ndarray, N: int) -> np.ndarray:
    """``iota`` of every column chunk: ``[D1][n]`` -> ``[n][C'][N]`` uint64; polynomial
    ``(i, r)`` has coefficient ``j`` = ``A[r N + j][i]``, zero past ``D1``."""
    D1, n = A.shape
    Cp = n_chunks(D1, N)
    pad = np.zeros((Cp * N, n), dtype=np.uint64)
    pad[:D1] = A
    return np.ascontiguousarray(pad.reshape(Cp, N, n).transpose(2, 0, 1))


def offset_polys(b: np.ndarray, N: int) -> np.ndarray:
    """``iota`` of every chunk of every client's offsets: ``[B][D1]`` -> ``[B][C'][N]`` uint64."""
    B, D1 = b.shape
    Cp = n_chunks(D1, N)
    pad = np.zeros((B, Cp * N), dtype=np.uint64)
    pad[:, :D1] = b
    return pad.reshape(B, Cp, N)


def pack_coeff(A: np.ndarray, b: np.ndarray, ct: np.ndarray, primes: list[int],
               p: int) -> np.ndarray:
    """Eq. tiptoe-rp by the ring definition (schoolbook negacyclic products), tiny sizes.

    ``A`` ``[D1][n]``, ``b`` ``[B][D1]`` (values in ``[0, p)``), ``ct`` ``[B][n][2][K][N]``
    -> ``[B][C'][2][K][N]`` uint64 residues.
    """
    B, n, _, K, N = ct.shape
    H = hint_polys(A, N)
    G = offset_polys(b, N)
    delta = scale(primes, p)
    Cp = H.shape[1]
    out = np.zeros((B, Cp, 2, K, N), dtype=np.uint64)
    for beta in range(B):
        for r in range(Cp):
            for c in range(2):
                for k, q in enumerate(primes):
                    acc = [0] * N if c == 0 else [(delta % q) * int(v) % q for v in G[beta, r]]
                    for i in range(n):
                        prod = _ntt.negacyclic_schoolbook([int(v) % q for v in H[i, r]],
                                                          ct[beta, i, c, k], q)
                        acc = [(x + y) % q for x, y in zip(acc, prod)]
                    out[beta, r, c, k] = acc
    return out


def hint_ntt(A: np.ndarray, N: int, primes: list[int], psis: list[int]) -> np.ndarray:
    """``H``: the lifted, transformed hint polynomials, ``[K][n][C'][N]``."""
    H = hint_polys(A, N)
    return np.stack([_ntt.ntt(H % np.uint64(q), q, psi) for q, psi in zip(primes, psis)])


def offset_ntt(b: np.ndarray, N: int, primes: list[int], psis: list[int], p: int) -> np.ndarray:
    """``G``: ``NTT(Delta * iota(b))`` per prime, ``[B][C'][K][N]``."""
    G = offset_polys(b, N)
    delta = scale(primes, p)
    out = np.empty(G.shape[:2] + (len(primes), N), dtype=np.uint64)
    for k, (q, psi) in enumerate(zip(primes, psis)):
        qq = np.uint64(q)
        out[:, :, k] = _ntt.ntt((G % qq) * np.uint64(delta % q) % qq, q, psi)
    return out


def pack_ntt_form(A, b, ct, primes, psis, p) -> np.ndarray:
    """``H * C + (0 | G)`` per (prime, slot): ``[B][C'][2][K][N]`` in NTT form."""
    N = ct.shape[-1]
    y = _scan.db_mul(hint_ntt(A, N, primes, psis), _scan.query_ntt(ct, primes, psis), primes)
    g = offset_ntt(b, N, primes, psis, p)
    for k, q in enumerate(primes):
        y[:, :, 1, k] = (y[:, :, 1, k] + g[:, :, k]) % np.uint64(q)
    return y


def pack(A, b, ct, primes, psis, p) -> np.ndarray:
    """Eq. tiptoe-rp through the NTT (Sec. 3.5): coefficient form ``[B][C'][2][K][N]``."""
    return _scan.answer_intt(pack_ntt_form(A, b, ct, primes, psis, p), primes, psis)


def lwe_phase(A: np.ndarray, b: np.ndarray, s: np.ndarray, p: int) -> np.ndarray:
    """``b + A s (mod p)`` of every client: ``A`` ``[D1][n]``, ``b`` ``[B][D1]``, ``s`` ``[B][n]``
    ternary -> ``[B][D1]`` int64 (exact: every partial sum is below 2^62)."""
    A64 = np.asarray(A, dtype=np.int64)
    out = np.empty(b.shape, dtype=np.int64)
    for beta in range(b.shape[0]):
        out[beta] = (np.asarray(b[beta], dtype=np.int64) + A64 @ np.asarray(s[beta], np.int64)) % p
    return out
