"""Modulus switching of answer ciphertexts from Q = q_0 q_1 ... down to 2^t.

The paper shrinks each response to one residue of about 29 bits by modulus
reduction (Sec. 2, ring packing, where #RNS drops to one; Sec. 3.6, the last
step of the hybrid protocol; Sec. 4.3 fuses it with the inverse NTT; App. D.5
bounds its rounding error).  For a ciphertext in coefficient form whose coefficient
x lies in [0, Q), held as residues mod the RNS primes, the switched
coefficient is the integer nearest to x * 2^t / Q, reduced mod 2^t.  Both
polynomials (a, b) of a ciphertext are switched; decryption then works mod
2^t with the message at scale 2^t / p.

Readings where the paper is loose:
* the target modulus is exactly 2^29 by default: the paper names a modulus
  of about 2^29, the size of one RNS residue, and its rounding errors below
  q / 2^30 are half a unit at 2^29; any 2^t with 1 <= t <= 32 is accepted;
* x is the canonical CRT value in [0, Q) (not the centred one), so a
  coefficient just below Q maps to 2^t, i.e. to 0 mod 2^t;
* rounding is to the nearest integer; Q is odd, so x * 2^(t+1) is never an
  odd multiple of Q and ties cannot occur.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import numpy as np

from . import rlwe
from . import scan as _scan
from .params import modulus

DEFAULT_BITS = 29


def switch(res: np.ndarray, primes: list[int], bits: int = DEFAULT_BITS) -> np.ndarray:
    """Residues ``[..., K, N]`` (coefficient form) -> ``[..., N]`` uint64 in ``[0, 2^bits)``.

    The nearest integer to ``x 2^bits / Q`` is ``floor((2 x 2^bits + Q) / (2 Q))``
    in exact integer arithmetic.
    """
    Q = modulus(primes)
    x = rlwe.crt(res, primes)
    y = (2 * x * (1 << bits) + Q) // (2 * Q)
    return np.asarray(y % (1 << bits), dtype=np.uint64)


def intt_switch(ans_ntt: np.ndarray, primes: list[int], psis: list[int],
                bits: int = DEFAULT_BITS) -> np.ndarray:
    """NTT-form answers ``[..., K, N]`` -> inverse NTT per prime -> switched ``[..., N]``."""
    return switch(_scan.answer_intt(ans_ntt, primes, psis), primes, bits)


def negacyclic_ternary(a: np.ndarray, s: np.ndarray) -> np.ndarray:
    """``a(X) * s(X) mod X^N + 1`` over the integers for a ternary ``s``.

    ``a``: ``[..., N]`` integers below 2^32; the full convolution has N terms
    of magnitude below 2^32 each, so int64 is exact for N <= 2^30.
    """
    a = np.asarray(a, dtype=np.int64)
    s = np.asarray(s, dtype=np.int64)
    N = a.shape[-1]
    flat = a.reshape(-1, N)
    out = np.empty_like(flat)
    for r in range(flat.shape[0]):
        full = np.convolve(flat[r], s)          # length 2N - 1
        c = full[:N].copy()
        c[:N - 1] -= full[N:]                   # X^N = -1
        out[r] = c
    return out.reshape(a.shape)


def decrypt_switched(ct: np.ndarray, s: np.ndarray, p: int,
                     bits: int = DEFAULT_BITS) -> tuple[np.ndarray, np.ndarray]:
    """Decrypt switched ciphertexts ``[..., 2, N]`` (component 0 = a, 1 = b) mod 2^bits.

    The phase ``a s + b`` mod 2^bits is centred in ``[-2^(bits-1), 2^(bits-1))``;
    the message is the nearest integer to ``phase p / 2^bits`` mod p.  Returns
    ``(m in [0, p) int64, noise)`` with noise the centred phase minus
    ``m 2^bits / p`` (a Python-int numerator over p: ``phase p - m 2^bits``).
    """
    Tm = 1 << bits
    a = np.asarray(ct[..., 0, :], dtype=np.int64)
    b = np.asarray(ct[..., 1, :], dtype=np.int64)
    phase = (negacyclic_ternary(a, s) + b) % Tm
    phase = np.where(phase >= Tm // 2, phase - Tm, phase).astype(object)
    rounded = (2 * phase * p + Tm) // (2 * Tm)
    noise_num = phase * p - rounded * Tm      # noise = noise_num / p in units of the phase
    m = np.asarray(rounded % p, dtype=np.int64)
    return m, noise_num
