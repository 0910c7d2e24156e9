"""Pins of oracle/expand.py (query expansion and RGSW folding) against things
other than itself:

* the automorphism by its evaluation definition (a(X^g) at psi^e is a at
  psi^(e g)), by the ring-homomorphism identity over schoolbook products and by
  composition of exponents; the monomial product by schoolbook;
* the gadget digits by exact recomposition to the centred CRT value (Python
  integers), with extreme values;
* key switching by the exact phase identity
  phase_s(ks(ct)) = phase_s'(ct) + sum_d D_d e_d, with the digit-error products
  taken by schoolbook, and by the trivial ciphertext (0, b), which no key
  changes;
* expansion by its closed form on trivial ciphertexts -- output k of (0, b) is
  exactly (0, sum_{i = k mod 2^l} b_i X^(i - k)) -- and by decryption of real
  encryptions to the constant coefficient k;
* the external product by m * ct exactly for a noiseless RGSW(m), by the exact
  phase identity for a real one, and folding by selection of ct[index] exactly
  (noiseless) and by decryption (real);
* planted mistakes in the oracle (a wrong automorphism exponent, no
  pre-scaling) fail these pins.
"""

import functools

import numpy as np
import pytest

import synth
from oracle import expand as ex
from oracle import ntt as on
from oracle import params as op
from oracle import rlwe
from oracle.params import modulus

BASE_LOG, N_DIGITS = 14, 4        # 2^56 >= Q for two primes below 2^28


@functools.lru_cache(maxsize=None)
def _ring(N, K):
    qs = op.ntt_primes(N, K)
    return tuple(qs), tuple(op.psi_min(N, q) for q in qs)   # psi_min scans ~q/N candidates


def ring(N, K=2):
    qs, psis = _ring(N, K)
    return list(qs), list(psis)


def rand_res(rng, lead, qs, N):
    return np.stack([rng.integers(0, q, size=lead + (N,), dtype=np.uint64) for q in qs], axis=-2)


def schoolbook_signed(a, b, q):
    """negacyclic product of integer lists, reduced mod q"""
    return np.array(on.negacyclic_schoolbook([int(x) % q for x in a], [int(x) % q for x in b], q),
                    dtype=np.uint64)


@pytest.mark.parametrize("N,g", [(16, 3), (16, 17), (32, 31), (64, 5), (64, 65)])
def test_automorphism_by_evaluation(N, g):
    qs, psis = ring(N)
    rng = np.random.default_rng(N + g)
    a = rand_res(rng, (), qs, N)
    t = ex.automorphism(a, g, qs)
    for k, (q, psi) in enumerate(zip(qs, psis)):
        got = on.ntt_naive(t[k], q, psi)
        exps = on.slot_exponents(N)
        want = [sum(int(a[k, n]) * pow(psi, int(e) * g * n, q) for n in range(N)) % q for e in exps]
        assert [int(x) for x in got] == want


def test_automorphism_homomorphism_and_composition():
    N = 32
    qs, _ = ring(N)
    rng = np.random.default_rng(3)
    a, b = rand_res(rng, (), qs, N), rand_res(rng, (), qs, N)
    for g in (3, 33, 63):
        for k, q in enumerate(qs):
            ab = schoolbook_signed(a[k], b[k], q)
            lhs = ex.automorphism(np.stack([ab, ab]), g, [q, q])[0]
            ta, tb = ex.automorphism(a, g, qs)[k], ex.automorphism(b, g, qs)[k]
            assert np.array_equal(lhs, schoolbook_signed(ta, tb, q))
    for g, h in [(3, 5), (17, 33), (63, 63)]:
        assert np.array_equal(ex.automorphism(ex.automorphism(a, h, qs), g, qs),
                              ex.automorphism(a, g * h % (2 * N), qs))
    assert np.array_equal(ex.automorphism(a, 1, qs), a)


@pytest.mark.parametrize("e", [1, 5, 15, 16, -1, -4, 33])
def test_monomial_matches_schoolbook(e):
    N = 16
    qs, _ = ring(N)
    a = rand_res(np.random.default_rng(e + 100), (), qs, N)
    got = ex.monomial(a, e, qs)
    for k, q in enumerate(qs):
        ee = e % (2 * N)
        xe = [0] * N
        xe[ee % N] = 1 if ee < N else q - 1
        assert np.array_equal(got[k], schoolbook_signed(a[k], xe, q))


def test_ring_mul_matches_schoolbook():
    N = 16
    qs, psis = ring(N)
    rng = np.random.default_rng(8)
    a, b = rand_res(rng, (), qs, N), rand_res(rng, (), qs, N)
    got = ex.ring_mul(a, b, qs, psis)
    for k, q in enumerate(qs):
        assert np.array_equal(got[k], schoolbook_signed(a[k], b[k], q))


def test_digits_recompose_exactly():
    N = 16
    qs, _ = ring(N)
    Q = modulus(qs)
    rng = np.random.default_rng(11)
    a = rand_res(rng, (3,), qs, N)
    xs = [0, 1, Q - 1, (Q - 1) // 2, (Q + 1) // 2, Q // 2, 2 ** 55, Q - 2 ** 55]
    for i, x in enumerate(xs):
        for k, q in enumerate(qs):
            a[0, k, i] = x % q
    D = ex.digits(a, qs, BASE_LOG, N_DIGITS)
    assert D.shape == (N_DIGITS, 3, N)
    half = 1 << (BASE_LOG - 1)
    assert D[:-1].min() >= -half and D[:-1].max() < half
    assert D[-1].min() >= -half and D[-1].max() <= half
    for r in range(3):
        for j in range(N):
            x = int(rlwe.crt(a[r][:, j:j + 1], qs)[0])
            xc = x - Q if x > Q // 2 else x
            assert sum(int(D[d, r, j]) << (BASE_LOG * d) for d in range(N_DIGITS)) == xc
    with pytest.raises(ValueError):
        ex.digits(a, qs, BASE_LOG, 3)          # 2^42 < Q


def _keys(seed, s, N, qs, psis, levels, n_digits=N_DIGITS):
    out = []
    for j in range(levels):
        g = ex.expansion_exponent(N, j)
        sg = ex.automorphism(ex.to_residues(s, qs), g, qs)
        s_from = rlwe.crt(sg, qs)
        Q = modulus(qs)
        s_from = np.array([int(v) - Q if int(v) > Q // 2 else int(v) for v in s_from])
        out.append(ex.ksk(s_from, s, synth.key_masks(seed, "ksk", 0, j, n_digits, qs, N),
                          synth.key_errors(seed, "ksk", 0, j, n_digits, N), qs, psis, BASE_LOG))
    return np.stack(out)


def test_keyswitch_exact_phase_identity():
    N = 32
    qs, psis = ring(N)
    s = synth.secret(4, 0, N)
    s_from = synth.secret(4, 1, N)
    masks = synth.key_masks(4, "ksk", 0, 0, N_DIGITS, qs, N)
    errs = synth.key_errors(4, "ksk", 0, 0, N_DIGITS, N)
    key = ex.ksk(s_from, s, masks, errs, qs, psis, BASE_LOG)
    rng = np.random.default_rng(5)
    ct = rand_res(rng, (2,), qs, N)
    out = ex.keyswitch(ct, key, qs, psis, BASE_LOG)
    D = ex.digits(ct[0], qs, BASE_LOG, N_DIGITS)
    ph_new = rlwe.phase_residues(out, s, qs, psis)
    ph_old = rlwe.phase_residues(ct, s_from, qs, psis)
    for k, q in enumerate(qs):
        extra = np.zeros(N, dtype=np.uint64)
        for d in range(N_DIGITS):
            extra = (extra + schoolbook_signed(D[d], errs[d], q)) % np.uint64(q)
        assert np.array_equal(ph_new[k], (ph_old[k] + extra) % np.uint64(q))
    trivial = ct.copy()
    trivial[0] = 0
    assert np.array_equal(ex.keyswitch(trivial, key, qs, psis, BASE_LOG), trivial)


def _closed_form(b, n, qs):
    """expansion of (0, b): output k = (0, sum_{i = k mod 2^l} b_i X^(i - k))"""
    N = b.shape[-1]
    l = ex.levels(n)
    out = np.zeros((n, 2, len(qs), N), dtype=np.uint64)
    for k in range(n):
        for i in range(k, N, 1 << l):
            out[k, 1, :, i - k] = b[:, i]
    return out


@pytest.mark.parametrize("N,n", [(16, 5), (16, 16), (32, 3), (64, 20), (64, 1)])
def test_expand_trivial_closed_form(N, n):
    qs, psis = ring(N)
    s = synth.secret(9, 0, N)
    keys = _keys(9, s, N, qs, psis, ex.levels(n))
    b = rand_res(np.random.default_rng(N * n), (), qs, N)
    ct = np.stack([np.zeros_like(b), b])
    assert np.array_equal(ex.expand(ct, keys, n, qs, psis, BASE_LOG), _closed_form(b, n, qs))


@pytest.mark.parametrize("N,n,p", [(16, 5, 256), (64, 20, 1 << 18), (64, 64, 256)])
def test_expand_decrypts_to_each_coefficient(N, n, p):
    qs, psis = ring(N)
    s = synth.secret(21, 0, N)
    keys = _keys(21, s, N, qs, psis, ex.levels(n))
    rng = np.random.default_rng(N + n)
    m = np.zeros(N, dtype=np.int64)
    m[:n] = rng.integers(0, p, size=n)
    delta = op.scale(qs, p)
    ct = rlwe.encrypt(m, s, synth.mask_row(21, 0, 0, qs, N), synth.error_row(21, 0, 0, N), qs,
                      psis, delta)
    out = ex.expand(ct, keys, n, qs, psis, BASE_LOG)
    got, noise = rlwe.decrypt(out, s, qs, psis, delta, p)
    want = np.zeros((n, N), dtype=np.int64)
    want[:, 0] = m[:n]
    assert np.array_equal(got, want)
    assert max(abs(int(v)) for v in noise.ravel()) < delta // 2


def _rgsw(seed, level, m, s, N, qs, psis, noiseless=False):
    rows = 2 * N_DIGITS
    masks = synth.key_masks(seed, "rgsw", 0, level, rows, qs, N)
    errs = synth.key_errors(seed, "rgsw", 0, level, rows, N)
    if noiseless:
        masks, errs = np.zeros_like(masks), np.zeros_like(errs)
    return ex.rgsw(m, s, masks, errs, qs, psis, BASE_LOG), errs


@pytest.mark.parametrize("m", [0, 1, 3])
def test_external_product_noiseless_is_scalar_multiple(m):
    N = 16
    qs, psis = ring(N)
    s = synth.secret(30, 0, N)
    C, _ = _rgsw(30, 0, m, s, N, qs, psis, noiseless=True)
    ct = rand_res(np.random.default_rng(m), (2,), qs, N)
    Q = np.array(qs, dtype=np.uint64)[:, None]
    assert np.array_equal(ex.external_product(C, ct, qs, psis, BASE_LOG), ct * np.uint64(m) % Q)


def test_external_product_exact_phase_identity():
    N = 32
    qs, psis = ring(N)
    s = synth.secret(31, 0, N)
    C, errs = _rgsw(31, 0, 1, s, N, qs, psis)
    ct = rand_res(np.random.default_rng(6), (2,), qs, N)
    out = ex.external_product(C, ct, qs, psis, BASE_LOG)
    Da = ex.digits(ct[0], qs, BASE_LOG, N_DIGITS)
    Db = ex.digits(ct[1], qs, BASE_LOG, N_DIGITS)
    ph_new = rlwe.phase_residues(out, s, qs, psis)
    ph_old = rlwe.phase_residues(ct, s, qs, psis)
    for k, q in enumerate(qs):
        extra = np.zeros(N, dtype=np.uint64)
        for d in range(N_DIGITS):
            extra = (extra + schoolbook_signed(Da[d], errs[d], q)
                     + schoolbook_signed(Db[d], errs[N_DIGITS + d], q)) % np.uint64(q)
        assert np.array_equal(ph_new[k], (ph_old[k] + extra) % np.uint64(q))


@pytest.mark.parametrize("index", [0, 5, 7])
def test_fold_selects_the_indexed_ciphertext(index):
    N, L = 16, 3
    qs, psis = ring(N)
    s = synth.secret(40, 0, N)
    rng = np.random.default_rng(index)
    cts = rand_res(rng, (1 << L, 2), qs, N)
    Cs = np.stack([_rgsw(40, j, (index >> j) & 1, s, N, qs, psis, noiseless=True)[0]
                   for j in range(L)])
    assert np.array_equal(ex.fold(cts, Cs, qs, psis, BASE_LOG), cts[index])
    # real encryptions of messages and of the index bits: decrypts to the message
    p, delta = 256, op.scale(qs, 256)
    msgs = rng.integers(0, p, size=(1 << L, N))
    cts = np.stack([rlwe.encrypt(msgs[i], s, synth.mask_row(41, i, 0, qs, N),
                                 synth.error_row(41, i, 0, N), qs, psis, delta)
                    for i in range(1 << L)])
    Cs = np.stack([_rgsw(42, j, (index >> j) & 1, s, N, qs, psis)[0] for j in range(L)])
    got, _ = rlwe.decrypt(ex.fold(cts, Cs, qs, psis, BASE_LOG), s, qs, psis, delta, p)
    assert np.array_equal(got, msgs[index])


def test_planted_mistakes_fail_the_pins(monkeypatch):
    N, n = 16, 5
    qs, psis = ring(N)
    s = synth.secret(9, 0, N)
    keys = _keys(9, s, N, qs, psis, ex.levels(n) + 1)
    b = rand_res(np.random.default_rng(1), (), qs, N)
    ct = np.stack([np.zeros_like(b), b])
    want = _closed_form(b, n, qs)
    with monkeypatch.context() as mp:
        mp.setattr(ex, "expansion_exponent", lambda N, j: N // (1 << j) - 1)
        assert not np.array_equal(ex.expand(ct, keys, n, qs, psis, BASE_LOG), want)
    with monkeypatch.context() as mp:
        mp.setattr(ex, "levels", lambda n: max(1, (n - 1).bit_length()) + 1)
        assert not np.array_equal(ex.expand(ct, keys, n, qs, psis, BASE_LOG)[:n], want)
    with monkeypatch.context() as mp:
        real_monomial = ex.monomial
        mp.setattr(ex, "monomial", lambda a, e, q: real_monomial(a, -e, q))
        assert not np.array_equal(ex.expand(ct, keys, n, qs, psis, BASE_LOG), want)
