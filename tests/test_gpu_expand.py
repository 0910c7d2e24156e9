"""GPU parity of query expansion (pir_expand) and RGSW folding (pir_fold)
against oracle/expand.

* expansion, every output word: N in {1024, 2048}, n in {1, 5, 64, 100}, B up
  to 3 clients with their own keys, two gadgets;
* expansion at the benchmark's size (N = 4096, two primes, n = 1280): sampled
  outputs (always 0, 1 and n - 1) word-exact against the oracle's recursion
  along their path, and every output of a real encryption of the client's
  ternary secret decrypts to its coefficient;
* ExpPack end to end: the expanded ciphertexts are the special ciphertexts of
  ring packing (pir_pack) and the packed RLWE ciphertexts decrypt to the LWE
  phases b + A s mod p;
* folding, every output word: D = 8 at N = 1024 (B = 2) and D = 256 at
  N = 4096 (the paper's log2 D_r = 8 rounds), with real RGSW encryptions of the
  index bits; the folded ciphertext decrypts to the indexed message;
* argument checks (host side).
"""

import numpy as np
import pytest

import synth
from oracle import expand as ex
from oracle import pack as opk
from oracle import params as op
from oracle import rlwe
from oracle.params import modulus

from pirtest import empty_dev, ring, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_11536_amd import pir
    c = pir.Context(0)
    yield c
    c.close()
    torch.cuda.empty_cache()


def _params(rg, p_log2=8):
    from paper_2606_11536_amd import pir
    return pir.Params(rg.log2n, list(rg.primes), p_log2)


def _signed(res, qs):
    Q = modulus(qs)
    x = rlwe.crt(res, qs)
    return np.array([int(v) - Q if int(v) > Q // 2 else int(v) for v in x], dtype=np.int64)


def _keys(seed, B, levels, rg, base_log, n_digits):
    """[B][levels][n_digits][2][K][N]: client b's key j switches s(X^(N/2^j+1)) -> s."""
    out, secrets = [], []
    for b in range(B):
        s = synth.secret(seed, b, rg.N)
        secrets.append(s)
        per = []
        for j in range(levels):
            g = ex.expansion_exponent(rg.N, j)
            s_from = _signed(ex.automorphism(ex.to_residues(s, rg.primes), g, rg.primes),
                             rg.primes)
            per.append(ex.ksk(s_from, s,
                              synth.key_masks(seed, "ksk", b, j, n_digits, rg.primes, rg.N),
                              synth.key_errors(seed, "ksk", b, j, n_digits, rg.N),
                              rg.primes, rg.psis, base_log))
        out.append(np.stack(per))
    return np.stack(out), secrets


def _uniform_ct(seed, B, rg):
    rng = np.random.default_rng(seed)
    return np.stack([np.stack([np.stack([rng.integers(0, q, rg.N, dtype=np.uint64)
                                         for q in rg.primes]) for _ in range(2)])
                     for _ in range(B)])


@pytest.mark.parametrize("log2n,n,B,base_log,n_digits", [(10, 5, 2, 14, 4), (10, 64, 1, 8, 7),
                                                         (10, 100, 3, 14, 4), (11, 1, 1, 14, 4)])
def test_expand_matches_oracle(ctx, log2n, n, B, base_log, n_digits):
    rg = ring(log2n, 2)
    l = ex.levels(n)
    keys, _ = _keys(log2n + n, B, l, rg, base_log, n_digits)
    ct = _uniform_ct(n, B, rg)
    K = ctx.load_expand_keys(_params(rg), keys, B, l, base_log, n_digits)
    out = empty_dev((B, n, 2, rg.K, rg.N))
    ctx.expand(K, to_dev(ct), n, out)
    got = to_host(out)
    for b in range(B):
        want = ex.expand(ct[b], keys[b], n, rg.primes, rg.psis, base_log)
        assert np.array_equal(got[b], want), f"client {b}"
    K.free()


def _path(ct, keys, n, m, qs, psis, base_log):
    """Output m of the expansion of ct, by the oracle's recursion along its path only."""
    l = ex.levels(n)
    N = ct.shape[-1]
    Q = np.array(qs, dtype=np.uint64)[:, None]
    inv = np.array([pow(2, -l, q) for q in qs], dtype=np.uint64)[:, None]
    c = np.asarray(ct, dtype=np.uint64) % Q * inv % Q
    for j in range(l):
        if (m >> j) & 1:
            c = ex.monomial(c, -(1 << j), qs)
        c = (c + ex.subs(c, ex.expansion_exponent(N, j), keys[j], qs, psis, base_log)) % Q
    return c


def test_expand_full_size(ctx):
    rg, n, B, base_log, n_digits = ring(12, 2), 1280, 2, 14, 4
    l = ex.levels(n)
    keys, secrets = _keys(77, B, l, rg, base_log, n_digits)
    # client b encrypts its own ternary LWE secret as coefficients 0 .. n-1
    p = 256
    delta = op.scale(rg.primes, p)
    msgs, cts = [], []
    for b in range(B):
        m = np.zeros(rg.N, dtype=np.int64)
        m[:n] = synth.lwe_secret(77, b, n)
        msgs.append(m)
        cts.append(rlwe.encrypt(m, secrets[b], synth.mask_row(77, b, 0, rg.primes, rg.N),
                                synth.error_row(77, b, 0, rg.N), rg.primes, rg.psis, delta))
    cts = np.stack(cts)
    K = ctx.load_expand_keys(_params(rg), keys, B, l, base_log, n_digits)
    out = empty_dev((B, n, 2, rg.K, rg.N))
    ctx.expand(K, to_dev(cts), n, out)
    got = to_host(out)
    for b in range(B):
        for m in [0, 1, n - 1, 517 + b]:
            assert np.array_equal(got[b, m], _path(cts[b], keys[b], n, m, rg.primes, rg.psis,
                                                   base_log)), f"client {b} output {m}"
        dec, _ = rlwe.decrypt(got[b], secrets[b], rg.primes, rg.psis, delta, p)
        want = np.zeros((n, rg.N), dtype=np.int64)
        want[:, 0] = msgs[b][:n] % p
        assert np.array_equal(dec, want), f"client {b}"
    K.free()


def test_exppack_end_to_end(ctx):
    # one ciphertext of the LWE secret, expanded into the n special ciphertexts of
    # ring packing, packs LWE ciphertexts into RLWE ones that decrypt to the phases
    rg, n, B, D1, p_log2, base_log, n_digits = ring(12, 2), 64, 2, 5000, 8, 8, 7
    p = 1 << p_log2
    l = ex.levels(n)
    keys, secrets = _keys(88, B, l, rg, base_log, n_digits)
    delta = op.scale(rg.primes, p)
    s_lwe = np.stack([synth.lwe_secret(88, b, n) for b in range(B)])
    cts = []
    for b in range(B):
        m = np.zeros(rg.N, dtype=np.int64)
        m[:n] = s_lwe[b]
        cts.append(rlwe.encrypt(m, secrets[b], synth.mask_row(88, b, 0, rg.primes, rg.N),
                                synth.error_row(88, b, 0, rg.N), rg.primes, rg.psis, delta))
    K = ctx.load_expand_keys(_params(rg, p_log2), keys, B, l, base_log, n_digits)
    special = empty_dev((B, n, 2, rg.K, rg.N))
    ctx.expand(K, to_dev(np.stack(cts)), n, special)
    A = synth.lwe_matrix(88, D1, n, p)
    bb = synth.lwe_offsets(88, B, D1, p)
    H = ctx.load_pack(_params(rg, p_log2), A, D1, n)
    Cp = opk.n_chunks(D1, rg.N)
    packed = empty_dev((B, Cp, 2, rg.K, rg.N))
    ctx.pack(H, B, special, to_dev(bb), packed)
    got = to_host(packed)
    phase = opk.lwe_phase(A, bb, s_lwe, p)
    for b in range(B):
        dec, _ = rlwe.decrypt(got[b], secrets[b], rg.primes, rg.psis, delta, p)
        want = np.zeros((Cp, rg.N), dtype=np.int64)
        want.reshape(-1)[:D1] = phase[b]
        assert np.array_equal(dec, want), f"client {b}"
    H.free()
    K.free()


def _rgsws(seed, B, L, index, rg, base_log, n_digits):
    out, secrets = [], []
    for b in range(B):
        s = synth.secret(seed, b, rg.N)
        secrets.append(s)
        out.append(np.stack([ex.rgsw((int(index[b]) >> j) & 1, s,
                                     synth.key_masks(seed, "rgsw", b, j, 2 * n_digits,
                                                     rg.primes, rg.N),
                                     synth.key_errors(seed, "rgsw", b, j, 2 * n_digits, rg.N),
                                     rg.primes, rg.psis, base_log) for j in range(L)]))
    return np.stack(out), secrets


@pytest.mark.parametrize("log2n,L,B", [(10, 3, 2), (12, 8, 1)])
def test_fold_matches_oracle(ctx, log2n, L, B):
    rg, base_log, n_digits, p = ring(log2n, 2), 14, 4, 256
    D = 1 << L
    index = synth.indices(L + 3, B, D)
    rg_s, secrets = _rgsws(L + 3, B, L, index, rg, base_log, n_digits)
    delta = op.scale(rg.primes, p)
    rng = np.random.default_rng(L)
    msgs = rng.integers(0, p, size=(B, D, rg.N))
    cts = np.stack([np.stack([rlwe.encrypt(msgs[b, i], secrets[b],
                                           synth.mask_row(L + 4, b, i, rg.primes, rg.N),
                                           synth.error_row(L + 4, b, i, rg.N), rg.primes,
                                           rg.psis, delta) for i in range(D)])
                    for b in range(B)])
    out = empty_dev((B, 2, rg.K, rg.N))
    ctx.fold(_params(rg), to_dev(cts), D, to_dev(rg_s), base_log, n_digits, B, out)
    got = to_host(out)
    for b in range(B):
        want = ex.fold(cts[b], rg_s[b], rg.primes, rg.psis, base_log)
        assert np.array_equal(got[b], want), f"client {b}"
        dec, _ = rlwe.decrypt(got[b], secrets[b], rg.primes, rg.psis, delta, p)
        assert np.array_equal(dec, msgs[b, int(index[b])])


def _small_ring(log2n=10):
    # two small NTT primes (= 1 mod 2N, Q ~ 2^29): gadget digits of 2^16 exceed
    # both, so the digit residues need a true reduction, not one added q
    from pirtest import Ring
    N = 1 << log2n
    qs = [12289, 40961]
    assert all(q % (2 * N) == 1 for q in qs)
    return Ring(log2n, qs, [op.psi_min(N, q) for q in qs], op.scale(qs, 256))


def test_expand_small_primes(ctx):
    rg, n, B, base_log, n_digits = _small_ring(), 12, 2, 16, 2
    l = ex.levels(n)
    keys, _ = _keys(91, B, l, rg, base_log, n_digits)
    ct = _uniform_ct(91, B, rg)
    K = ctx.load_expand_keys(_params(rg), keys, B, l, base_log, n_digits)
    out = empty_dev((B, n, 2, rg.K, rg.N))
    ctx.expand(K, to_dev(ct), n, out)
    got = to_host(out)
    for b in range(B):
        assert np.array_equal(got[b], ex.expand(ct[b], keys[b], n, rg.primes, rg.psis, base_log))
    K.free()


def test_fold_small_primes(ctx):
    rg, L, B, base_log, n_digits = _small_ring(), 3, 2, 16, 2
    D = 1 << L
    index = synth.indices(93, B, D)
    rg_s, _ = _rgsws(93, B, L, index, rg, base_log, n_digits)
    cts = np.stack([_uniform_ct(94 + b, D, rg) for b in range(B)])
    out = empty_dev((B, 2, rg.K, rg.N))
    ctx.fold(_params(rg), to_dev(cts), D, to_dev(rg_s), base_log, n_digits, B, out)
    got = to_host(out)
    for b in range(B):
        assert np.array_equal(got[b], ex.fold(cts[b], rg_s[b], rg.primes, rg.psis, base_log))


def test_arguments(ctx):
    from paper_2606_11536_amd import pir
    rg = ring(10, 2)
    keys, _ = _keys(5, 1, 2, rg, 14, 4)
    with pytest.raises(pir.PirError):                     # 2^(10*4) does not cover Q
        ctx.load_expand_keys(_params(rg), keys, 1, 2, 10, 4)
    K = ctx.load_expand_keys(_params(rg), keys, 1, 2, 14, 4)
    out = empty_dev((1, 8, 2, rg.K, rg.N))
    ct = to_dev(_uniform_ct(1, 1, rg))
    with pytest.raises(pir.PirError):                     # n = 8 needs 3 levels of keys
        ctx.expand(K, ct, 8, out)
    with pytest.raises(pir.PirError):
        ctx.expand(K, ct, 0, out)
    K.free()
    three = ring(10, 3)
    with pytest.raises(pir.PirError) as e:                # one or two primes only
        ctx.fold(_params(three), ct, 2, ct, 20, 4, 1, out)
    assert e.value.status == 2
    with pytest.raises(pir.PirError):                     # D not a power of two
        ctx.fold(_params(rg), ct, 3, ct, 14, 4, 1, out)
