"""Query expansion and RGSW folding over RNS primes -- TEST INFRASTRUCTURE ONLY.

Two server-side steps of the paper's poly-HE path, written from their
definitions:

* **Expansion** (ExpPack, Sec. 3.5 and App. C.2): the client sends one RLWE
  ciphertext of ``sum_i m_i X^i`` and the server recovers ``n`` ciphertexts,
  the ``i``-th encrypting the constant ``m_i``.  The paper uses the recursive
  expansion of SealPIR as a black box and states two facts about it: each
  output encrypts ``2^l m_i`` (``l = ceil(log2 n)``), and the server
  pre-scales the input by ``2^-l mod q`` so that the outputs encrypt ``m_i``.
  The recursion restated here: at level ``j = 0 .. l-1`` every ciphertext
  ``c`` (index ``k < 2^j``) becomes
      ``c + Subs(c, N/2^j + 1)``                          at index ``k``,
      ``c' + Subs(c', N/2^j + 1)``, ``c' = c X^(-2^j)``   at index ``k + 2^j``,
  where ``Subs(c, g)`` applies the automorphism ``X -> X^g`` and switches the
  key back from ``s(X^g)`` to ``s``.  The automorphism with ``g = N/2^j + 1``
  fixes ``X^(2^j m)`` for even ``m`` and negates it for odd ``m``, so the sum
  keeps (doubled) the coefficients whose index has bit ``j`` clear; after
  ``l`` levels index ``k`` holds coefficient ``k``.
* **RGSW folding** (Sec. 3.2 step 7; Sec. 3.6): ``log2 D`` rounds of
  RGSW-RLWE external products select one of ``D`` RLWE ciphertexts.  The
  external product of ``RGSW(m)`` with ``ct`` encrypts ``m`` times the phase of
  ``ct``; ``CMux(RGSW(b), ct0, ct1) = ct0 + RGSW(b) [x] (ct1 - ct0)`` picks
  ``ct_b``.  Round ``j`` pairs entries ``2i`` and ``2i + 1`` with bit ``j`` of
  the index.

Readings where the paper is silent (the paper gives neither the gadget nor the
key format):

* gadget: the coefficient is recombined by CRT into ``[0, Q)``, centred to
  ``(-Q/2, Q/2]`` and written in ``n_digits`` balanced digits of base
  ``2^base_log``: the low ones in ``[-2^(base_log-1), 2^(base_log-1))``, the
  top one taking the rest, which ``2^(base_log n_digits) >= Q`` keeps in
  ``[-2^(base_log-1), 2^(base_log-1)]``; the gadget vector is
  ``g_d = 2^(base_log d)``;
* key-switching key from ``s'`` to ``s``: ``n_digits`` RLWE ciphertexts
  ``(a_d, -a_d s + e_d + g_d s')``; switching ``(a, b)`` gives
  ``(sum_d D_d a_d, b + sum_d D_d (-a_d s + e_d + g_d s'))`` with ``D_d`` the
  digits of ``a``;
* RGSW(m): ``2 n_digits`` rows; row ``d`` is ``(a_d + m g_d, -a_d s + e_d)``,
  row ``n_digits + d`` is ``(a_d', -a_d' s + e_d' + m g_d)``.  The external
  product with ``(a, b)`` is ``sum_d D_d(a) row_d + D_d(b) row_{n_digits + d}``;
* ciphertext layout and component order are those of ``rlwe``: ``[2][K][N]``
  residues, component 0 the mask ``a``, phase ``a s + b``.

Random inputs (masks, errors) are drawn by ``synth`` and passed in; nothing
here draws random numbers.
"""

from __future__ import annotations

import numpy as np

from . import ntt as _ntt
from .params import modulus
from .rlwe import crt


def automorphism(a: np.ndarray, g: int, primes: list[int]) -> np.ndarray:
    """``a(X^g)`` for odd ``g``: coefficient ``j`` goes to ``j g mod 2N``, negated when
    that exponent is ``>= N`` (``X^N = -1``).  ``a``: ``[..., K, N]`` residues."""
    if g % 2 == 0:
        raise ValueError("the automorphism needs an odd exponent")
    return _move(a, np.arange(np.shape(a)[-1], dtype=np.int64) * g, primes)


def _move(a: np.ndarray, dest: np.ndarray, primes: list[int]) -> np.ndarray:
    """Coefficient ``j`` of ``a`` to exponent ``dest[j] mod 2N`` (a permutation of the
    exponents mod N), negated where that exponent is ``>= N``."""
    a = np.asarray(a, dtype=np.uint64)
    N = a.shape[-1]
    e = np.asarray(dest, dtype=np.int64) % (2 * N)
    pos = e % N
    if len(np.unique(pos)) != N:
        raise ValueError("not a permutation of the exponents")
    neg = e >= N
    out = np.empty_like(a)
    for k, q in enumerate(primes):
        qq = np.uint64(q)
        v = a[..., k, :] % qq
        v = np.where(neg, (qq - v) % qq, v)
        out[..., k, pos] = v
    return out


def monomial(a: np.ndarray, e: int, primes: list[int]) -> np.ndarray:
    """``a X^e`` in ``Z_q[X]/(X^N + 1)`` for any integer ``e``.  ``a``: ``[..., K, N]``."""
    return _move(a, np.arange(np.shape(a)[-1], dtype=np.int64) + e, primes)


def ring_mul(a: np.ndarray, b: np.ndarray, primes: list[int], psis: list[int]) -> np.ndarray:
    """Negacyclic product per prime (NTT, pointwise product, inverse NTT).  Both ``[..., K, N]``
    (broadcast over leading axes)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    shape = np.broadcast_shapes(a.shape, b.shape)
    out = np.empty(shape, dtype=np.uint64)
    for k, (q, psi) in enumerate(zip(primes, psis)):
        qq = np.uint64(q)
        fa = _ntt.ntt(np.broadcast_to(a[..., k, :], shape[:-2] + shape[-1:]) % qq, q, psi)
        fb = _ntt.ntt(np.broadcast_to(b[..., k, :], shape[:-2] + shape[-1:]) % qq, q, psi)
        out[..., k, :] = _ntt.intt(fa * fb % qq, q, psi)
    return out


def to_residues(x: np.ndarray, primes: list[int]) -> np.ndarray:
    """Signed integers ``[..., N]`` (int64 or object) -> residues ``[..., K, N]`` uint64."""
    x = np.asarray(x)
    return np.stack([np.asarray(x % q, dtype=np.uint64) for q in primes], axis=-2)


def gadget(primes: list[int], base_log: int, n_digits: int) -> list[list[int]]:
    """``g_d mod q_k = 2^(base_log d) mod q_k``: ``[n_digits][K]``."""
    return [[pow(2, base_log * d, q) for q in primes] for d in range(n_digits)]


def digits(a: np.ndarray, primes: list[int], base_log: int, n_digits: int) -> np.ndarray:
    """Balanced base-``2^base_log`` digits of the centred CRT value of every coefficient.

    ``a``: ``[..., K, N]`` residues -> ``[n_digits, ..., N]`` int64 digits ``D_d`` with
    ``sum_d D_d 2^(base_log d) = x`` exactly, ``x`` the coefficient centred in
    ``(-Q/2, Q/2]``."""
    Q = modulus(primes)
    if (1 << (base_log * n_digits)) < Q:
        raise ValueError("the gadget does not cover Q")
    x = crt(np.asarray(a, dtype=np.uint64), primes)           # object ints in [0, Q)
    x = np.where(x > Q // 2, x - Q, x)
    B, half = 1 << base_log, 1 << (base_log - 1)
    out = np.empty((n_digits,) + x.shape, dtype=np.int64)
    rest = x
    for d in range(n_digits - 1):
        r = rest % B                                           # in [0, B)
        r = np.where(r >= half, r - B, r)                      # in [-B/2, B/2)
        out[d] = np.asarray(r, dtype=np.int64)
        rest = (rest - r) // B
    # the top digit takes the rest: |x| <= Q/2 <= B^n_digits / 2 keeps it in [-B/2, B/2]
    if np.any(np.abs(rest) > half):
        raise ValueError("value outside the gadget's range")
    out[n_digits - 1] = np.asarray(rest, dtype=np.int64)
    return out


def encrypt_zero(s: np.ndarray, a: np.ndarray, e: np.ndarray, primes: list[int],
                 psis: list[int]) -> np.ndarray:
    """``(a, -a s + e)``: ``a`` ``[..., K, N]``, ``e`` ``[..., N]`` -> ``[..., 2, K, N]``."""
    a = np.asarray(a, dtype=np.uint64)
    neg_as = ring_mul(a, to_residues(-np.asarray(s, dtype=np.int64), primes), primes, psis)
    b = (neg_as + to_residues(np.asarray(e, dtype=np.int64), primes)) % np.array(
        primes, dtype=np.uint64)[:, None]
    return np.stack([a % np.array(primes, dtype=np.uint64)[:, None], b], axis=-3)


def ksk(s_from: np.ndarray, s: np.ndarray, masks: np.ndarray, errors: np.ndarray,
        primes: list[int], psis: list[int], base_log: int) -> np.ndarray:
    """Key-switching key from ``s_from`` to ``s``: ``[n_digits][2][K][N]``, row ``d`` =
    ``(a_d, -a_d s + e_d + g_d s_from)``.  ``masks`` ``[n_digits][K][N]``, ``errors``
    ``[n_digits][N]``."""
    n_digits = masks.shape[0]
    out = encrypt_zero(s, masks, errors, primes, psis)
    sf = to_residues(np.asarray(s_from, dtype=np.int64), primes)
    g = gadget(primes, base_log, n_digits)
    for d in range(n_digits):
        for k, q in enumerate(primes):
            out[d, 1, k] = (out[d, 1, k] + np.uint64(g[d][k]) * sf[k]) % np.uint64(q)
    return out


def _dot_digits(D: np.ndarray, rows: np.ndarray, primes: list[int], psis: list[int]) -> np.ndarray:
    """``sum_d D_d rows_d``: ``D`` ``[n_digits][N]`` signed, ``rows`` ``[n_digits][2][K][N]``."""
    acc = np.zeros(rows.shape[1:], dtype=np.uint64)
    Q = np.array(primes, dtype=np.uint64)[:, None]
    for d in range(D.shape[0]):
        Dd = to_residues(D[d], primes)                                  # [K][N]
        acc = (acc + ring_mul(rows[d], Dd[None], primes, psis)) % Q
    return acc


def keyswitch(ct: np.ndarray, key: np.ndarray, primes: list[int], psis: list[int],
              base_log: int) -> np.ndarray:
    """Switch ``ct`` ``[2][K][N]`` (under ``s_from``) to ``s`` with ``key = ksk(s_from, s)``."""
    D = digits(ct[0], primes, base_log, key.shape[0])
    out = _dot_digits(D, key, primes, psis)
    out[1] = (out[1] + ct[1]) % np.array(primes, dtype=np.uint64)[:, None]
    return out


def subs(ct: np.ndarray, g: int, key: np.ndarray, primes: list[int], psis: list[int],
         base_log: int) -> np.ndarray:
    """``Subs(ct, g)``: the automorphism ``X -> X^g`` then a key switch from ``s(X^g)``."""
    return keyswitch(automorphism(ct, g, primes), key, primes, psis, base_log)


def levels(n: int) -> int:
    """``l = ceil(log2 n)``: the expansion's levels (at least one)."""
    return max(1, (n - 1).bit_length())


def expansion_exponent(N: int, j: int) -> int:
    """The automorphism exponent of level ``j``: ``N/2^j + 1``."""
    return N // (1 << j) + 1


def expand(ct: np.ndarray, keys: np.ndarray, n: int, primes: list[int], psis: list[int],
           base_log: int) -> np.ndarray:
    """Expansion of ``ct`` ``[2][K][N]`` into ``n`` ciphertexts ``[n][2][K][N]``.

    ``keys[j]`` switches from ``s(X^(N/2^j + 1))`` to ``s``, ``j < levels(n)``.  The input
    is first multiplied by ``2^-l mod q_k``; output ``k`` then encrypts coefficient ``k``."""
    l = levels(n)
    N = ct.shape[-1]
    Q = np.array(primes, dtype=np.uint64)[:, None]
    inv = np.array([pow(2, -l, q) for q in primes], dtype=np.uint64)[:, None]
    cur = [np.asarray(ct, dtype=np.uint64) % Q * inv % Q]
    for j in range(l):
        g = expansion_exponent(N, j)
        nxt = [None] * (2 * len(cur))
        for k, c in enumerate(cur):
            c1 = monomial(c, -(1 << j), primes)
            nxt[k] = (c + subs(c, g, keys[j], primes, psis, base_log)) % Q
            nxt[k + (1 << j)] = (c1 + subs(c1, g, keys[j], primes, psis, base_log)) % Q
        cur = nxt
    return np.stack(cur[:n])


def rgsw(m: int, s: np.ndarray, masks: np.ndarray, errors: np.ndarray, primes: list[int],
         psis: list[int], base_log: int) -> np.ndarray:
    """``RGSW(m)``: ``[2 n_digits][2][K][N]`` from ``masks`` ``[2 n_digits][K][N]`` and
    ``errors`` ``[2 n_digits][N]``; row ``d`` gets ``m g_d`` on the mask, row
    ``n_digits + d`` on the body."""
    n_digits = masks.shape[0] // 2
    out = encrypt_zero(s, masks, errors, primes, psis)
    g = gadget(primes, base_log, n_digits)
    for d in range(n_digits):
        for k, q in enumerate(primes):
            add = np.uint64((m % q) * g[d][k] % q)
            out[d, 0, k, 0] = (out[d, 0, k, 0] + add) % np.uint64(q)
            out[n_digits + d, 1, k, 0] = (out[n_digits + d, 1, k, 0] + add) % np.uint64(q)
    return out


def external_product(C: np.ndarray, ct: np.ndarray, primes: list[int], psis: list[int],
                     base_log: int) -> np.ndarray:
    """``RGSW [x] RLWE``: ``sum_d D_d(a) C_d + D_d(b) C_{n_digits + d}``."""
    n_digits = C.shape[0] // 2
    Da = digits(ct[0], primes, base_log, n_digits)
    Db = digits(ct[1], primes, base_log, n_digits)
    Q = np.array(primes, dtype=np.uint64)[:, None]
    return (_dot_digits(Da, C[:n_digits], primes, psis) +
            _dot_digits(Db, C[n_digits:], primes, psis)) % Q


def cmux(C: np.ndarray, ct0: np.ndarray, ct1: np.ndarray, primes: list[int], psis: list[int],
         base_log: int) -> np.ndarray:
    """``ct0 + C [x] (ct1 - ct0)``: ``ct_b`` for ``C = RGSW(b)``, ``b`` in {0, 1}."""
    Q = np.array(primes, dtype=np.uint64)[:, None]
    diff = (np.asarray(ct1, dtype=np.uint64) + Q - np.asarray(ct0, dtype=np.uint64) % Q) % Q
    return (np.asarray(ct0, dtype=np.uint64) + external_product(C, diff, primes, psis,
                                                                base_log)) % Q


def fold(cts: np.ndarray, Cs: np.ndarray, primes: list[int], psis: list[int],
         base_log: int) -> np.ndarray:
    """Select one of ``D = 2^L`` ciphertexts ``cts`` ``[D][2][K][N]`` with ``L`` RGSW
    encryptions of index bits ``Cs`` ``[L][2 n_digits][2][K][N]``: round ``j`` replaces
    entries ``(2i, 2i + 1)`` by ``CMux(Cs[j], ., .)``."""
    cur = [np.asarray(c, dtype=np.uint64) for c in cts]
    for j in range(Cs.shape[0]):
        cur = [cmux(Cs[j], cur[2 * i], cur[2 * i + 1], primes, psis, base_log)
               for i in range(len(cur) // 2)]
    return cur[0]
