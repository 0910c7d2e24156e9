"""Pins of the ring-packing oracle (oracle/pack.py) against what the paper fixes.

* the NTT-form evaluation (Sec. 3.5, H C + (0|G) per slot) equals Eq.
  tiptoe-rp evaluated by the ring definition (schoolbook negacyclic
  products), with a ragged last chunk;
* closed form for trivial special ciphertexts (0, Delta s_i): the packed
  result is exactly (0, Delta * iota(b + A s)) in R_Q, computed here with an
  integer matrix-vector product and no ring arithmetic at all;
* end to end (App. C.1): with real RLWE encryptions of the LWE secret, the
  packed ciphertext decrypts, coefficient by coefficient, to the LWE phases
  b + A s mod p of every chunk, and to zero in the padding past D1;
* the paper's sizes: 1280 special ciphertexts at N = 4096 with three 28-bit
  primes take 120 MiB per client (Sec. 3.5).
Planted mistakes (a dropped offset, transposed mask chunks, the offset on
the wrong component) are shown to fail the closed form.
"""

import numpy as np
import pytest

import synth
from oracle import pack, params, rlwe


def _ring(N, K):
    qs = params.ntt_primes(N, K)
    return qs, [params.psi_min(N, q) for q in qs]


def _inputs(seed, D1, n, B, N, qs, p):
    A = synth.lwe_matrix(seed, D1, n, p)
    b = synth.lwe_offsets(seed, B, D1, p)
    rng = np.random.default_rng(seed)
    ct = np.stack([rng.integers(0, q, size=(B, n, 2, N), dtype=np.uint64) for q in qs], axis=3)
    return A, b, ct


@pytest.mark.parametrize("N,D1,n", [(256, 300, 3), (256, 256, 2), (256, 7, 2)])
def test_ntt_form_equals_ring_definition(N, D1, n):
    qs, psis = _ring(N, 2)
    p = 1 << 18
    A, b, ct = _inputs(N + D1, D1, n, 2, N, qs, p)
    got = pack.pack(A, b, ct, qs, psis, p)
    assert got.shape == (2, pack.n_chunks(D1, N), 2, 2, N)
    assert np.array_equal(got, pack.pack_coeff(A, b, ct, qs, p))


def _trivial(s, qs, delta, N):
    """Trivial encryptions (a = 0, b = Delta s_i) of the secret entries: [B][n][2][K][N]."""
    B, n = s.shape
    ct = np.zeros((B, n, 2, len(qs), N), dtype=np.uint64)
    for k, q in enumerate(qs):
        ct[:, :, 1, k, 0] = (delta * s) % q
    return ct


def _closed_form(A, b, s, qs, delta, N):
    """(0, Delta * iota(b + A s)) per chunk, from an integer product: [B][C'][2][K][N]."""
    x = b.astype(np.int64) + (A.astype(np.int64) @ s.T).T          # [B][D1], no reduction
    B, D1 = x.shape
    Cp = pack.n_chunks(D1, N)
    xp = np.zeros((B, Cp * N), dtype=object)
    xp[:, :D1] = x
    out = np.zeros((B, Cp, 2, len(qs), N), dtype=np.uint64)
    for k, q in enumerate(qs):
        out[:, :, 1, k] = ((delta * xp) % q).reshape(B, Cp, N).astype(np.uint64)
    return out


@pytest.mark.parametrize("N,D1,n,p_log2", [(256, 600, 9, 18), (256, 512, 12, 32), (512, 20, 6, 8)])
def test_trivial_special_ciphertexts_closed_form(N, D1, n, p_log2):
    qs, psis = _ring(N, 2)
    p = 1 << p_log2
    delta = params.scale(qs, p)
    B = 3
    A = synth.lwe_matrix(7, D1, n, p)
    b = synth.lwe_offsets(7, B, D1, p)
    s = np.stack([synth.lwe_secret(7, beta, n) for beta in range(B)])
    ct = _trivial(s, qs, delta, N)
    exp = _closed_form(A, b, s, qs, delta, N)
    assert np.array_equal(pack.pack(A, b, ct, qs, psis, p), exp)
    # planted mistakes, each caught by the closed form
    assert not np.array_equal(pack.pack(A, 0 * b, ct, qs, psis, p), exp)
    At = np.ascontiguousarray(A.reshape(-1)[::-1].reshape(A.shape))
    assert not np.array_equal(pack.pack(At, b, ct, qs, psis, p), exp)
    y = pack.pack_ntt_form(A, b, ct, qs, psis, p)
    g = pack.offset_ntt(b, N, qs, psis, p)
    wrong = y.copy()
    for k, q in enumerate(qs):                                       # offset on component 0 too
        wrong[:, :, 0, k] = (wrong[:, :, 0, k] + g[:, :, k]) % np.uint64(q)
    from oracle import scan
    assert not np.array_equal(scan.answer_intt(wrong, qs, psis), exp)


@pytest.mark.parametrize("N,D1,n", [(256, 600, 40), (1024, 1024, 64)])
def test_packed_ciphertext_decrypts_to_lwe_phases(N, D1, n):
    qs, psis = _ring(N, 2)
    p = 1 << 18
    delta = params.scale(qs, p)
    B, seed = 2, 21
    A = synth.lwe_matrix(seed, D1, n, p)
    b = synth.lwe_offsets(seed, B, D1, p)
    s_lwe = np.stack([synth.lwe_secret(seed, beta, n) for beta in range(B)])
    cts, keys = [], []
    for beta in range(B):
        key = synth.secret(seed, beta, N)
        m = np.zeros((n, N), dtype=np.int64)
        # the constant polynomials s_i, encrypted as the signed integers they
        # are: Delta * (-1), not Delta * (p - 1), which would add
        # -(Q mod p) * iota(A_i) to the phase when p does not divide Q - 1
        m[:, 0] = s_lwe[beta]
        a = np.stack([synth.mask_row(seed, beta, i, qs, N) for i in range(n)])
        e = np.stack([synth.error_row(seed, beta, i, N) for i in range(n)])
        cts.append(rlwe.encrypt(m, key, a, e, qs, psis, delta))
        keys.append(key)
    res = pack.pack(A, b, np.stack(cts), qs, psis, p)                 # [B][C'][2][K][N]
    phase = pack.lwe_phase(A, b, s_lwe, p)                            # [B][D1]
    Cp = pack.n_chunks(D1, N)
    for beta in range(B):
        m, noise = rlwe.decrypt(res[beta], keys[beta], qs, psis, delta, p)   # [C'][N]
        flat = m.reshape(Cp * N)
        assert np.array_equal(flat[:D1], phase[beta])
        assert not flat[D1:].any()
        assert max(abs(int(v)) for v in noise.ravel()) < delta // 2


def test_paper_special_ciphertext_size():
    # Sec. 3.5: n = 1280 special ciphertexts of two polynomials, N = 4096,
    # #RNS = 3 residues of 4 bytes, make 120 MiB per client
    n, N, rns = 1280, 4096, 3
    assert n * 2 * rns * N * 4 == 120 * 2**20
