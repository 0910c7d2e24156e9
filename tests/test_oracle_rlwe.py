"""Pins for oracle.rlwe (App. A.2).

* CRT vs sympy's ``crt``;
* a fresh ciphertext's decryption noise equals the error drawn, exactly
  (the phase is Delta*m + e by App. A.2's defining equation), less the one
  that App. A's plaintext wrap-around predicts;
* the phase is linear under ciphertext addition and plaintext products
  (App. A, RNS prime selection, phase identities);
* the NTT-based mask product inside ``encrypt`` vs schoolbook at tiny N.
"""

import numpy as np
import pytest
from sympy.ntheory.modular import crt as sympy_crt

import synth
from oracle import ntt, params, rlwe

rng = np.random.default_rng(99)


def test_crt_matches_sympy():
    qs = params.ntt_primes(2048, 2)
    x = [int(v) for v in rng.integers(0, params.modulus(qs), 50, dtype=np.int64)]
    res = np.array([[v % q for v in x] for q in qs], dtype=np.uint64)  # [K][n]
    got = rlwe.crt(res, qs)
    for v, g, i in zip(x, got, range(len(x))):
        assert g == v == int(sympy_crt(qs, [int(res[0, i]), int(res[1, i])])[0])


def _keys(N, K, seed=7):
    qs = params.ntt_primes(N, K)
    psis = [params.psi_min(N, q) for q in qs]
    delta = params.scale(qs, 256)
    return qs, psis, delta


@pytest.mark.parametrize("N,K", [(1024, 1), (2048, 2), (4096, 2)])
def test_fresh_ciphertext_noise_is_the_drawn_error(N, K):
    qs, psis, delta = _keys(N, K)
    s = synth.secret(3, 0, N)
    m = rng.integers(0, 256, size=(2, N))
    a = np.stack([synth.mask_row(3, 0, i, qs, N) for i in range(2)])
    e = np.stack([synth.error_row(3, 0, i, N) for i in range(2)])
    ct = rlwe.encrypt(m, s, a, e, qs, psis, delta)
    assert ct.shape == (2, 2, K, N)
    assert np.array_equal(ct[:, 0], a)
    dec, noise = rlwe.decrypt(ct, s, qs, psis, delta, 256)
    assert np.array_equal(dec, m)
    # App. A: with Delta*p + 1 = Q a plaintext past p/2 centres to Delta*(m - p) - 1, so the
    # observed noise is the drawn error, less one exactly where Delta*m + e wraps past (Q-1)/2
    Q = params.modulus(qs)
    wraps = np.array([[delta * int(mm) + int(ee) > (Q - 1) // 2 for mm, ee in zip(r1, r2)]
                      for r1, r2 in zip(m, e)])
    assert wraps.any() and (~wraps).any()
    assert np.array_equal(np.asarray(noise, dtype=np.int64), e - wraps.astype(np.int64))


def test_encrypt_matches_schoolbook_mask_product():
    N = 16
    q = params.ntt_primes(N, 1, bound=1 << 20)[0]
    psi = params.psi_min(N, q)
    delta = q // 256
    s = synth.secret(5, 0, N)
    a = synth.mask_row(5, 0, 0, [q], N)[None]          # [1][K=1][N]
    e = synth.error_row(5, 0, 0, N)[None]
    m = np.arange(N)[None] % 256
    ct = rlwe.encrypt(m, s, a, e, [q], [psi], delta)
    a_s = ntt.negacyclic_schoolbook(a[0, 0], [int(v) % q for v in s], q)
    b = [(delta * int(mm) + int(ee) - x) % q for mm, ee, x in zip(m[0], e[0], a_s)]
    assert ct[0, 1, 0].tolist() == b


def test_phase_is_linear():
    N, K = 1024, 2
    qs, psis, delta = _keys(N, K)
    s = synth.secret(11, 0, N)
    a = np.stack([synth.mask_row(11, 0, i, qs, N) for i in range(2)])
    e = np.stack([synth.error_row(11, 0, i, N) for i in range(2)])
    m = rng.integers(0, 256, size=(2, N))
    ct = rlwe.encrypt(m, s, a, e, qs, psis, delta)
    ph = rlwe.phase_residues(ct, s, qs, psis)                # [2][K][N]
    tot = np.empty_like(ct[0])
    for k, q in enumerate(qs):
        tot[:, k] = (ct[0, :, k] + ct[1, :, k]) % np.uint64(q)
    ph_sum = rlwe.phase_residues(tot, s, qs, psis)
    for k, q in enumerate(qs):
        assert np.array_equal(ph_sum[k], (ph[0, k] + ph[1, k]) % np.uint64(q))
    # plaintext product: phase(c*ct) = c*phase(ct) in R_q
    c = rng.integers(0, 256, N).astype(np.uint64)
    prod = np.empty_like(ct[0])
    for k, (q, psi) in enumerate(zip(qs, psis)):
        for comp in range(2):
            prod[comp, k] = ntt.negacyclic_mul(c, ct[0, comp, k], q, psi)
    ph_prod = rlwe.phase_residues(prod, s, qs, psis)
    for k, (q, psi) in enumerate(zip(qs, psis)):
        assert np.array_equal(ph_prod[k], ntt.negacyclic_mul(c, ph[0, k], q, psi))


def test_error_sampler_respects_clip_and_sigma():
    e = np.concatenate([synth.error_row(1, 0, i, 4096) for i in range(16)])
    assert np.abs(e).max() <= 19
    assert 3.0 < e.std() < 3.4
