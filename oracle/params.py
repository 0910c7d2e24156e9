"""RNS parameters for the scan: primes, 2N-th roots of unity, the scale.

Follows the RNS prime selection rule of App. A (subsection "RNS prime
selection"): each prime satisfies ``q_k = 1 mod 2N`` so that a negacyclic NTT
of length N exists.  The paper keeps primes below 2**29 for lazy reduction;
the workloads here bound them by 2**28 and take the largest such primes.
The scale is ``Delta = floor(Q / p)`` for ``Q = prod q_k`` (App. A.2).

Root convention (the paper names the NTT but not its root): ``psi`` is the
smallest integer ``x >= 2`` with ``x**N = -1 (mod q)``; any such ``x`` has
multiplicative order exactly ``2N``.
"""

from __future__ import annotations

from functools import reduce


def is_prime(n: int) -> bool:
    """Trial division; exact for any n (used only below 2**32)."""
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    d = 3
    while d * d <= n:
        if n % d == 0:
            return False
        d += 2
    return True


def ntt_primes(N: int, count: int, bound: int = 1 << 28) -> list[int]:
    """The ``count`` largest primes ``q < bound`` with ``q = 1 (mod 2N)``, descending."""
    step = 2 * N
    q = ((bound - 2) // step) * step + 1  # largest value < bound that is 1 mod 2N
    out: list[int] = []
    while len(out) < count and q > step:
        if is_prime(q):
            out.append(q)
        q -= step
    if len(out) < count:
        raise ValueError("not enough primes below bound")
    return out


def psi_min(N: int, q: int) -> int:
    """Smallest ``x >= 2`` with ``x**N = -1 (mod q)``: a primitive 2N-th root of unity."""
    x = 2
    while pow(x, N, q) != q - 1:
        x += 1
        if x >= q:
            raise ValueError("no 2N-th root of unity: q != 1 mod 2N?")
    return x


def modulus(primes: list[int]) -> int:
    """``Q = prod q_k`` (RNS decomposition, Sec. 2.3)."""
    return reduce(lambda x, y: x * y, primes, 1)


def scale(primes: list[int], p: int) -> int:
    """``Delta = floor(Q / p)`` (App. A.2)."""
    return modulus(primes) // p
