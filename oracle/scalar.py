"""Scalar-HE database GEMM mod 2^32 (Sec. 4.1; the SimplePIR online step of Sec. 2).

The database is a D1 x D0 matrix of 8-bit plaintexts, the batch a B x D0
matrix of 32-bit LWE ciphertext words; the server computes, for every query b
and database row r,

    out[b][r] = sum_c DB[r][c] * Q[b][c]   (mod 2^32).

The paper splits each 32-bit word into four bytes and runs four INT8 GEMMs
whose results it shifts by 0, 8, 16, 24 bits and adds mod 2^32 (Sec. 4.1);
reduction mod 2^32 is free.  The oracle is the definition above, written with
numpy's int64 matrix product: every term is below 2^7 * 2^32 in magnitude and
there are at most 2^17 of them, so each sum is exact below 2^56.

Readings where the paper is loose:
* database entries are signed bytes in [-128, 127] (the INT8 operand of the
  tensor-core GEMM): any representative of a plaintext mod 2^8 decrypts to the
  same plaintext, and the signed one keeps the decryption noise smallest;
* query words are unsigned 32-bit integers (the ciphertext modulus is 2^32);
* D0 is at most 2^17, enough for the paper's D0 = 65536.

``lwe_onehot`` and ``lwe_decrypt`` are a toy SimplePIR round trip (secret
dimension n, scale 2^24 for plaintexts mod 2^8, hint = DB times the public
matrix) used to pin the GEMM's meaning end to end.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import numpy as np

MOD = 1 << 32
D0_MAX = 1 << 17


def db_gemm(db: np.ndarray, q: np.ndarray) -> np.ndarray:
    """``db``: ``[D1][D0]`` int8; ``q``: ``[B][D0]`` uint32 -> ``[B][D1]`` uint32."""
    db = np.asarray(db)
    q = np.asarray(q)
    if db.dtype != np.int8 or db.ndim != 2 or q.ndim != 2 or q.shape[1] != db.shape[1]:
        raise ValueError("db must be int8 [D1][D0] and q [B][D0]")
    if db.shape[1] > D0_MAX:
        raise ValueError("D0 above 2^17")
    prod = q.astype(np.int64) @ db.astype(np.int64).T
    return (prod % MOD).astype(np.uint32)


def lwe_onehot(A: np.ndarray, s: np.ndarray, e: np.ndarray, i_star: int, p: int = 256) -> np.ndarray:
    """LWE encryption of the one-hot vector for column ``i_star`` under secret ``s``.

    ``A``: ``[D0][n]`` uniform words, ``s``: ``[n]``, ``e``: ``[D0]`` small errors.
    Returns ``[D0]`` uint32: ``A s + e + (2^32 / p) [c == i_star]`` mod 2^32.
    """
    delta = MOD // p
    b = (A.astype(np.int64) @ s.astype(np.int64) + e.astype(np.int64)) % MOD
    b = (b + delta * (np.arange(A.shape[0]) == i_star)) % MOD
    return b.astype(np.uint32)


def lwe_decrypt(ans: np.ndarray, hint_s: np.ndarray, p: int = 256) -> np.ndarray:
    """Round ``(ans - hint s) mod 2^32`` to the nearest multiple of 2^32 / p; values mod p."""
    delta = MOD // p
    d = (ans.astype(np.int64) - hint_s.astype(np.int64)) % MOD
    return (((d + delta // 2) // delta) % p).astype(np.int64)
