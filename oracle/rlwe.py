"""Toy RLWE encryption and decryption over RNS primes (App. A.2).

A ciphertext is ``(a, b)`` with component 0 the uniform mask ``a`` and
component 1 ``b`` (App. A.2 writes ``ct = (a(X), b(X))``).  Encryption makes
the phase ``a*s + b = Delta*m + e (mod Q)``; decryption computes the phase,
centres it in ``[-(Q-1)/2, (Q-1)/2]`` and rounds ``phase / Delta`` to the
nearest integer, which is ``m`` when every error coefficient lies in
``(-Delta/2, Delta/2)``.  Arithmetic is per RNS prime (Sec. 2.3); the
phase is recombined with the Chinese remainder theorem before rounding.

The random inputs (secret, masks, errors) are drawn by ``synth`` and passed
in; nothing here draws random numbers.

Readings where the paper is silent: the decrypted value is reported mod
``p`` in ``[0, p)`` (the plaintext is a database byte); rounding is to the
nearest integer (ties cannot occur while the error is below ``Delta/2``).
"""

from __future__ import annotations

import numpy as np

from . import ntt as _ntt
from .params import modulus


def encrypt(m: np.ndarray, s: np.ndarray, a: np.ndarray, e: np.ndarray,
            primes: list[int], psis: list[int], delta: int) -> np.ndarray:
    """Encrypt plaintext polynomials.

    ``m``: ``[..., N]`` integer plaintext coefficients; ``s``: ``[N]`` ternary;
    ``a``: ``[..., K, N]`` masks in ``[0, q_k)``; ``e``: ``[..., N]`` errors.
    Returns ``[..., 2, K, N]`` uint64 residues: component 0 = ``a``, component 1 =
    ``b = Delta*m + e - a*s (mod q_k)``.
    """
    m = np.asarray(m, dtype=np.int64)
    e = np.asarray(e, dtype=np.int64)
    s = np.asarray(s, dtype=np.int64)
    lead = m.shape[:-1]
    N = m.shape[-1]
    K = len(primes)
    out = np.empty(lead + (2, K, N), dtype=np.uint64)
    for k, (q, psi) in enumerate(zip(primes, psis)):
        qq = np.uint64(q)
        ak = np.asarray(a[..., k, :], dtype=np.uint64)
        sk = (s % q).astype(np.uint64)
        a_s = _ntt.intt(_ntt.ntt(ak, q, psi) * _ntt.ntt(sk, q, psi) % qq, q, psi)
        dm = ((delta % q) * (m % q).astype(object)) % q  # exact: Delta*m can exceed 2**63
        dm = np.asarray(dm, dtype=np.uint64)
        ek = (e % q).astype(np.uint64)
        out[..., 0, k, :] = ak
        out[..., 1, k, :] = (dm + ek + qq - a_s) % qq
    return out


def phase_residues(ct: np.ndarray, s: np.ndarray, primes: list[int], psis: list[int]) -> np.ndarray:
    """``a*s + b (mod q_k)`` per prime.  ``ct``: ``[..., 2, K, N]`` -> ``[..., K, N]`` uint64."""
    s = np.asarray(s, dtype=np.int64)
    out = np.empty(ct.shape[:-3] + ct.shape[-2:], dtype=np.uint64)
    for k, (q, psi) in enumerate(zip(primes, psis)):
        qq = np.uint64(q)
        ak = np.asarray(ct[..., 0, k, :], dtype=np.uint64) % qq
        bk = np.asarray(ct[..., 1, k, :], dtype=np.uint64) % qq
        sk = (s % q).astype(np.uint64)
        a_s = _ntt.intt(_ntt.ntt(ak, q, psi) * _ntt.ntt(sk, q, psi) % qq, q, psi)
        out[..., k, :] = (a_s + bk) % qq
    return out


def crt(res: np.ndarray, primes: list[int]) -> np.ndarray:
    """Chinese remainder theorem: residues ``[..., K, N]`` -> integers in ``[0, Q)`` (object array).

    Garner's mixed-radix form: ``x = r_0 + q_0 (y_1 + q_1 (y_2 + ...))``.
    """
    K = len(primes)
    res = np.asarray(res)
    x = res[..., 0, :].astype(object)
    radix = primes[0]
    for k in range(1, K):
        qk = primes[k]
        inv = pow(radix % qk, -1, qk)
        rk = res[..., k, :].astype(object)
        y = ((rk - x) % qk) * inv % qk
        x = x + radix * y
        radix *= qk
    return x


def decrypt(ct: np.ndarray, s: np.ndarray, primes: list[int], psis: list[int],
            delta: int, p: int) -> tuple[np.ndarray, np.ndarray]:
    """Decrypt ``[..., 2, K, N]`` ciphertexts.

    Returns ``(m, noise)``: ``m`` in ``[0, p)`` (int64) and the centred phase minus
    ``Delta*round(phase/Delta)`` (object ints), whose magnitude must stay below ``Delta/2``.
    """
    Q = modulus(primes)
    phi = crt(phase_residues(ct, s, primes, psis), primes)
    half = (Q - 1) // 2
    phi_c = np.where(phi > half, phi - Q, phi)
    # nearest integer to phi_c / delta; floor((2 phi + delta) / (2 delta)) with Python ints
    rounded = (2 * phi_c + delta) // (2 * delta)
    noise = phi_c - rounded * delta
    m = np.asarray(rounded % p, dtype=np.int64)
    return m, noise
