"""Pins for oracle.modswitch (Sec. 4.3 fusion target; App. D.5 error analysis).

* brute force on tiny moduli: the switched value is the integer z (taken
  mod 2^t) that minimises |z Q - x 2^t| over every candidate z, for every x;
* negation: switching Q - x gives 2^t minus the switch of x (mod 2^t),
  exactly (fails for floor or ceiling rounding);
* App. D.5's bound: the rounding error is at most half a new unit, i.e.
  |y Q - x 2^t| <= Q / 2 for the representative y of the switched value;
* the NTT round trip: switching NTT-form answers after the oracle's inverse
  NTT equals switching the coefficient form directly;
* decryption: fresh ciphertexts of random messages, switched to 2^29 (and
  2^24), decrypt to the messages; with zero encryption error the remaining
  noise is rounding only and stays within (N + 1) / 2 units of the phase;
* the ternary negacyclic product used by decryption vs the schoolbook one.
"""

import numpy as np
import pytest

import synth
from oracle import modswitch as ms
from oracle import ntt, params, rlwe
from oracle import scan as osc

rng = np.random.default_rng(2606)


@pytest.mark.parametrize("primes,bits", [([17, 97], 3), ([17, 97], 6), ([97], 8), ([5, 13], 2)])
def test_brute_force_nearest(primes, bits):
    Q = params.modulus(primes)
    T = 1 << bits
    xs = list(range(Q))
    res = np.array([[x % q for x in xs] for q in primes], dtype=np.uint64)   # [K][n]
    got = ms.switch(res, primes, bits)
    for x, g in zip(xs, got):
        best = min(range(T + 1), key=lambda z: abs(z * Q - x * T))
        assert int(g) == best % T, (x, int(g), best)


def _residues(x, qs):
    return np.array([[v % q for v in x] for q in qs], dtype=np.uint64)


def test_negation_identity():
    qs = params.ntt_primes(2048, 2)
    Q = params.modulus(qs)
    x = [int(v) for v in rng.integers(1, Q, 2000, dtype=np.int64)] + [1, Q - 1, Q // 2, Q // 2 + 1]
    a = ms.switch(_residues(x, qs), qs, 29)
    b = ms.switch(_residues([Q - v for v in x], qs), qs, 29)
    assert all((int(u) + int(v)) % (1 << 29) == 0 for u, v in zip(a, b))


@pytest.mark.parametrize("bits", [29, 20, 32])
def test_rounding_error_bound(bits):
    qs = params.ntt_primes(4096, 2)
    Q = params.modulus(qs)
    T = 1 << bits
    x = [int(v) for v in rng.integers(0, Q, 3000, dtype=np.int64)] + [0, 1, Q - 1, Q - 2]
    y = ms.switch(_residues(x, qs), qs, bits)
    for v, g in zip(x, y):
        err = min(abs(int(g) * Q - v * T), abs((int(g) + T) * Q - v * T))
        assert 2 * err <= Q


@pytest.mark.parametrize("N,K", [(1024, 1), (1024, 2), (2048, 2)])
def test_ntt_round_trip(N, K):
    qs = params.ntt_primes(N, K)
    psis = [params.psi_min(N, q) for q in qs]
    coeff = np.stack([rng.integers(0, q, (3, N), dtype=np.int64) for q in qs], axis=1).astype(np.uint64)
    hat = osc.query_ntt(coeff[:, None, None], qs, psis)[:, 0, 0]          # [3][K][N]
    assert np.array_equal(ms.intt_switch(hat, qs, psis), ms.switch(coeff, qs))


@pytest.mark.parametrize("bits", [29, 24])
@pytest.mark.parametrize("zero_error", [False, True])
def test_switched_ciphertexts_decrypt(bits, zero_error):
    N, p = 1024, 256
    qs = params.ntt_primes(N, 2)
    psis = [params.psi_min(N, q) for q in qs]
    delta = params.scale(qs, p)
    m = rng.integers(0, p, (4, N), dtype=np.int64)
    s = synth.secret(11, 0, N)
    a = np.stack([synth.mask_row(11, 0, i, qs, N) for i in range(4)])
    e = np.zeros((4, N), dtype=np.int64) if zero_error else \
        np.stack([synth.error_row(11, 0, i, N) for i in range(4)])
    ct = rlwe.encrypt(m, s, a, e, qs, psis, delta)                       # [4][2][K][N]
    sw = ms.switch(ct, qs, bits)                                          # [4][2][N]
    got, noise_num = ms.decrypt_switched(sw, s, p, bits)
    assert np.array_equal(got, m)
    worst = max(abs(int(v)) for v in noise_num.ravel()) / p               # in units of the phase
    if zero_error:
        assert worst <= (N + 1) / 2
    assert worst < (1 << bits) / (4 * p)


def test_ternary_product_vs_schoolbook():
    q = 257
    for N in (4, 8, 16):
        a = rng.integers(0, 1 << 29, N, dtype=np.int64)
        s = rng.integers(-1, 2, N, dtype=np.int64)
        got = ms.negacyclic_ternary(a, s) % q
        ref = ntt.negacyclic_schoolbook([int(v) % q for v in a], [int(v) % q for v in s], q)
        assert [int(v) for v in got] == [int(v) for v in ref]
