"""Pins for oracle.ntt.

* schoolbook negacyclic product vs a full library convolution folded by
  X^N = -1, and vs sympy polynomial remainder;
* naive NTT vs the convolution theorem for R_q = Z_q[X]/(X^N+1) (Sec. 2.3);
* closed forms NTT(1) = (1,...,1) and NTT(X)[k] = psi^(2 brv(k)+1);
* the fast network vs the naive definition, and INTT o NTT = id.
"""

import numpy as np
import pytest
import sympy

from oracle import ntt, params

rng = np.random.default_rng(1234)


def _fold(full, N, q):
    c = [0] * N
    for m, v in enumerate(full):
        if m < N:
            c[m] += int(v)
        else:
            c[m - N] -= int(v)
    return [x % q for x in c]


@pytest.mark.parametrize("N,q", [(4, 17), (8, 97), (16, 97), (32, 193)])
def test_schoolbook_vs_library_convolution(N, q):
    for _ in range(5):
        a = rng.integers(0, q, N).tolist()
        b = rng.integers(0, q, N).tolist()
        full = np.convolve(np.array(a, dtype=object), np.array(b, dtype=object))
        assert ntt.negacyclic_schoolbook(a, b, q) == _fold(full, N, q)


def test_schoolbook_vs_sympy():
    N, q = 8, 97
    X = sympy.symbols("X")
    a = rng.integers(0, q, N).tolist()
    b = rng.integers(0, q, N).tolist()
    pa = sympy.Poly(list(reversed(a)), X, modulus=q)
    pb = sympy.Poly(list(reversed(b)), X, modulus=q)
    r = (pa * pb).rem(sympy.Poly(X**N + 1, X, modulus=q))
    coeffs = [int(c) % q for c in reversed(r.all_coeffs())]
    coeffs += [0] * (N - len(coeffs))
    assert ntt.negacyclic_schoolbook(a, b, q) == coeffs


def test_x_to_the_n_is_minus_one():
    N, q = 8, 97
    x = [0, 1] + [0] * (N - 2)
    xn1 = [0] * (N - 1) + [1]
    assert ntt.negacyclic_schoolbook(x, xn1, q) == [q - 1] + [0] * (N - 1)


def _small_cases():
    out = []
    for N in (4, 8, 16, 32, 64):
        for q in params.ntt_primes(N, 3, bound=1 << 14):
            out.append((N, q))
    return out


@pytest.mark.parametrize("N,q", _small_cases())
def test_naive_ntt_convolution_theorem(N, q):
    psi = params.psi_min(N, q)
    for _ in range(3):
        a = rng.integers(0, q, N).astype(np.uint64)
        b = rng.integers(0, q, N).astype(np.uint64)
        c = np.array(ntt.negacyclic_schoolbook(a, b, q), dtype=np.uint64)
        lhs = ntt.ntt_naive(a, q, psi) * ntt.ntt_naive(b, q, psi) % np.uint64(q)
        assert np.array_equal(lhs, ntt.ntt_naive(c, q, psi))
        assert np.array_equal(ntt.intt_naive(ntt.ntt_naive(a, q, psi), q, psi), a)


@pytest.mark.parametrize("N,bound", [(8, 1 << 14), (64, 1 << 14), (1024, 1 << 28)])
def test_naive_ntt_closed_forms(N, bound):
    q = params.ntt_primes(N, 1, bound=bound)[0]
    psi = params.psi_min(N, q)
    one = np.zeros(N, dtype=np.uint64)
    one[0] = 1
    assert np.all(ntt.ntt_naive(one, q, psi) == 1)
    x = np.zeros(N, dtype=np.uint64)
    x[1] = 1
    bits = N.bit_length() - 1
    expect = [pow(psi, 2 * ntt.bitrev(k, bits) + 1, q) for k in range(N)]
    assert ntt.ntt_naive(x, q, psi).tolist() == expect
    # the evaluation points are exactly the N roots of X^N + 1
    assert sorted(expect) == sorted(pow(psi, e, q) for e in range(1, 2 * N, 2))


@pytest.mark.parametrize("N,bound", [(16, 1 << 14), (64, 1 << 16), (1024, 1 << 28),
                                     (2048, 1 << 28), (4096, 1 << 28)])
def test_fast_ntt_equals_definition(N, bound):
    for q in params.ntt_primes(N, 2, bound=bound):
        psi = params.psi_min(N, q)
        a = rng.integers(0, q, size=(2, N)).astype(np.uint64)
        A = ntt.ntt(a, q, psi)
        assert np.array_equal(A, ntt.ntt_naive(a, q, psi))
        assert np.array_equal(ntt.intt(A, q, psi), a)
        assert np.array_equal(ntt.intt(A, q, psi), ntt.intt_naive(A, q, psi))


def test_fast_ntt_batched_leading_axes():
    N = 64
    q = params.ntt_primes(N, 1, bound=1 << 16)[0]
    psi = params.psi_min(N, q)
    a = rng.integers(0, q, size=(3, 4, N)).astype(np.uint64)
    A = ntt.ntt(a, q, psi)
    for i in range(3):
        for j in range(4):
            assert np.array_equal(A[i, j], ntt.ntt_naive(a[i, j], q, psi))


def test_negacyclic_mul_matches_schoolbook():
    N = 32
    q = params.ntt_primes(N, 1, bound=1 << 16)[0]
    psi = params.psi_min(N, q)
    a = rng.integers(0, q, N).astype(np.uint64)
    b = rng.integers(0, q, N).astype(np.uint64)
    assert ntt.negacyclic_mul(a, b, q, psi).tolist() == ntt.negacyclic_schoolbook(a, b, q)
