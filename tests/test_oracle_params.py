"""Pins for oracle.params: primes, roots of unity, scale.

Pins come from outside the oracle: sympy's primality test and primitive
roots (a different algorithm from the oracle's trial division and ascending
search), the parameter values the paper prints (tests/golden/paper_params.json),
and the closed form Delta*p + 1 = Q of the RNS prime selection rule (App. A).
"""

import json
import math
import os

import pytest
import sympy

from oracle import params

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_params.json")


@pytest.mark.parametrize("N,count", [(1024, 1), (2048, 2), (4096, 2), (16, 3)])
def test_primes_are_the_largest_ntt_primes(N, count):
    qs = params.ntt_primes(N, count)
    assert qs == sorted(qs, reverse=True)
    for q in qs:
        assert q < 1 << 28 and q % (2 * N) == 1 and sympy.isprime(q)
    # maximality: sympy finds no other prime = 1 mod 2N in (q_last, 2^28)
    cands = [x for x in range(qs[-1], 1 << 28, 2 * N) if sympy.isprime(x)]
    assert sorted(cands, reverse=True) == qs


def test_two_prime_pair_serves_every_ring_degree():
    # the two largest primes for N = 2048 are also 1 mod 2*4096, so N = 4096 uses the same pair
    assert params.ntt_primes(2048, 2) == params.ntt_primes(4096, 2)
    assert params.ntt_primes(1024, 1) == params.ntt_primes(2048, 1)


def _all_primitive_2n_roots(N, q):
    g = sympy.primitive_root(q)
    base = pow(g, (q - 1) // (2 * N), q)
    return sorted(pow(base, 2 * m + 1, q) for m in range(N))


@pytest.mark.parametrize("N,bound", [(16, 1 << 16), (1024, 1 << 28), (2048, 1 << 28),
                                     (4096, 1 << 28)])
def test_psi_is_the_smallest_primitive_root(N, bound):
    for q in params.ntt_primes(N, 2, bound=bound):
        psi = params.psi_min(N, q)
        roots = _all_primitive_2n_roots(N, q)
        assert psi == roots[0]
        assert pow(psi, N, q) == q - 1 and pow(psi, 2 * N, q) == 1


def test_scale_matches_printed_parameters():
    g = json.load(open(GOLDEN))
    lwe = g["lwe"]
    assert params.scale([lwe["q"]], lwe["p"]) == lwe["delta"]
    # RLWE default: N = 2^12, p = 2^18, three primes < 2^29 with q = 1 mod 2N and q = 1 mod p
    d = g["rlwe_default"]
    p = 1 << d["p_log2"]
    step_n = max(2 * d["N"], p) // 2            # ntt_primes steps by 2*step_n
    qs = params.ntt_primes(step_n, d["n_primes"], bound=1 << d["prime_bound_log2"])
    Q = params.modulus(qs)
    delta = params.scale(qs, p)
    assert round(math.log2(Q)) == d["q_log2_approx"]
    assert round(math.log2(delta)) == d["delta_log2_approx"]
    assert delta * p + 1 == Q                    # App. A closed form


@pytest.mark.parametrize("N,K", [(1024, 1), (2048, 2)])
def test_workload_scale_closed_form_and_overflow_example(N, K):
    p = 256
    qs = params.ntt_primes(N, K)
    Q = params.modulus(qs)
    delta = params.scale(qs, p)
    assert delta * p + 1 == Q
    # App. A: Delta*(3/8)p + Delta*(3/8)p = Delta*(-p/4) - 1 (mod Q)
    lhs = (delta * (3 * p // 8) * 2) % Q
    rhs = (delta * (-(p // 4)) - 1) % Q
    assert lhs == rhs


def test_is_prime_small_values():
    assert [n for n in range(60) if params.is_prime(n)] == list(sympy.primerange(0, 60))
