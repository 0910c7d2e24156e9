"""Negacyclic products and the NTT over ``Z_q[X]/(X^N + 1)`` (Sec. 2.3).

The paper uses the NTT to turn a product in ``R_q`` into slot-wise products
mod ``q`` (Sec. 2.3, last paragraph) but fixes neither the root nor the output
order.  Reading taken here: slot ``k`` of the transform of ``a`` is the
evaluation of ``a`` at ``psi**(2*brv(k) + 1)``, where ``brv`` reverses the
``log2 N`` low bits of ``k``.  These are the N roots of ``X^N + 1``, listed in
bit-reversed order -- the order an in-place Cooley-Tukey network produces
from natural-order input.  The inverse includes the ``N^{-1}`` factor.

``negacyclic_schoolbook``, ``ntt_naive`` and ``intt_naive`` are the
definitions written out (quadratic).  ``ntt``/``intt`` are plain radix-2
networks used where the quadratic forms are too slow; the tests pin them to
the definitions.
"""

from __future__ import annotations

import numpy as np


def bitrev(k: int, bits: int) -> int:
    """Reverse the ``bits`` low bits of ``k``."""
    r = 0
    for _ in range(bits):
        r = (r << 1) | (k & 1)
        k >>= 1
    return r


def log2_exact(N: int) -> int:
    b = N.bit_length() - 1
    if N <= 0 or (1 << b) != N:
        raise ValueError("N must be a power of two")
    return b


def negacyclic_schoolbook(a, b, q: int) -> list[int]:
    """``a*b mod (X^N + 1, q)`` by definition: ``c_m = sum_{i+j=m} a_i b_j - sum_{i+j=m+N} a_i b_j``."""
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    N = len(a)
    c = [0] * N
    for i in range(N):
        for j in range(N):
            if i + j < N:
                c[i + j] += a[i] * b[j]
            else:
                c[i + j - N] -= a[i] * b[j]
    return [x % q for x in c]


def slot_exponents(N: int) -> np.ndarray:
    """Odd exponent ``2*brv(k)+1`` of the evaluation point of slot ``k``."""
    bits = log2_exact(N)
    return np.array([2 * bitrev(k, bits) + 1 for k in range(N)], dtype=np.int64)


def _power_table(psi: int, q: int, count: int) -> np.ndarray:
    t = np.empty(count, dtype=np.uint64)
    x = 1
    for e in range(count):
        t[e] = x
        x = x * psi % q
    return t


def ntt_naive(a: np.ndarray, q: int, psi: int) -> np.ndarray:
    """Definition: ``A[k] = sum_n a_n psi^((2 brv(k)+1) n) mod q``.  ``a``: ``[..., N]``."""
    a = np.asarray(a, dtype=np.uint64) % np.uint64(q)
    N = a.shape[-1]
    pw = _power_table(psi, q, 2 * N)  # psi has order 2N
    e = (slot_exponents(N)[:, None] * np.arange(N, dtype=np.int64)[None, :]) % (2 * N)
    M = pw[e]  # [k][n]
    out = np.empty(a.shape, dtype=np.uint64)
    flat_in = a.reshape(-1, N)
    flat_out = out.reshape(-1, N)
    for r in range(flat_in.shape[0]):
        flat_out[r] = ((M * flat_in[r][None, :]) % np.uint64(q)).sum(axis=1) % np.uint64(q)
    return out


def intt_naive(A: np.ndarray, q: int, psi: int) -> np.ndarray:
    """Definition: ``a_n = N^{-1} sum_k A[k] psi^(-(2 brv(k)+1) n) mod q``."""
    A = np.asarray(A, dtype=np.uint64) % np.uint64(q)
    N = A.shape[-1]
    pw = _power_table(pow(psi, -1, q), q, 2 * N)
    e = (np.arange(N, dtype=np.int64)[:, None] * slot_exponents(N)[None, :]) % (2 * N)
    M = pw[e]  # [n][k]
    ninv = np.uint64(pow(N, -1, q))
    out = np.empty(A.shape, dtype=np.uint64)
    flat_in = A.reshape(-1, N)
    flat_out = out.reshape(-1, N)
    for r in range(flat_in.shape[0]):
        s = ((M * flat_in[r][None, :]) % np.uint64(q)).sum(axis=1) % np.uint64(q)
        flat_out[r] = s * ninv % np.uint64(q)
    return out


def _rev_powers(w: int, q: int, N: int) -> np.ndarray:
    """``w^brv(i)`` for ``i < N`` (bit reversal over ``log2 N`` bits)."""
    bits = log2_exact(N)
    pw = _power_table(w, q, N)
    return pw[[bitrev(i, bits) for i in range(N)]]


def ntt(a: np.ndarray, q: int, psi: int) -> np.ndarray:
    """Radix-2 Cooley-Tukey network computing ``ntt_naive`` in O(N log N).  ``a``: ``[..., N]``.

    At the stage with ``m`` blocks of length ``2h`` (``m*2h = N``), block ``i`` pairs
    entry ``r`` of its first half with entry ``r`` of its second half and uses the
    twiddle ``psi^brv(m + i)`` (``brv`` over ``log2 N`` bits).
    """
    x = np.asarray(a, dtype=np.uint64) % np.uint64(q)
    lead = x.shape[:-1]
    N = x.shape[-1]
    x = x.reshape(-1, N).copy()
    qq = np.uint64(q)
    tw = _rev_powers(psi, q, N)
    m, h = 1, N // 2
    while m < N:
        v = x.reshape(-1, m, 2, h)
        w = tw[m:2 * m][None, :, None]
        hi = v[:, :, 1, :] * w % qq
        lo = v[:, :, 0, :].copy()
        v[:, :, 0, :] = (lo + hi) % qq
        v[:, :, 1, :] = (lo + qq - hi) % qq
        m, h = 2 * m, h // 2
    return x.reshape(*lead, N)


def intt(A: np.ndarray, q: int, psi: int) -> np.ndarray:
    """Gentleman-Sande network inverting ``ntt`` (computes ``intt_naive``)."""
    x = np.asarray(A, dtype=np.uint64) % np.uint64(q)
    lead = x.shape[:-1]
    N = x.shape[-1]
    x = x.reshape(-1, N).copy()
    qq = np.uint64(q)
    tw = _rev_powers(pow(psi, -1, q), q, N)
    m, h = N // 2, 1
    while m >= 1:
        v = x.reshape(-1, m, 2, h)
        w = tw[m:2 * m][None, :, None]
        lo = v[:, :, 0, :].copy()
        hi = v[:, :, 1, :].copy()
        v[:, :, 0, :] = (lo + hi) % qq
        v[:, :, 1, :] = (lo + qq - hi) % qq * w % qq
        m, h = m // 2, 2 * h
    x = x * np.uint64(pow(N, -1, q)) % qq
    return x.reshape(*lead, N)


def negacyclic_mul(a: np.ndarray, b: np.ndarray, q: int, psi: int) -> np.ndarray:
    """``a*b`` in ``R_q`` through the NTT (convolution theorem); broadcasts over leading axes."""
    return intt(ntt(a, q, psi) * ntt(b, q, psi) % np.uint64(q), q, psi)
