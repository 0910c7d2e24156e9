"""GPU parity of ring packing (pir_pack_load + pir_pack) against oracle/pack.

* every output word, coefficient form and switched to 2^29, for ragged D1
  (the last chunk partial), n in {100, 1280}, B in {1, 3, 17}, N in {1024,
  2048}, p = 2^18 and p = 2^32;
* end to end: real RLWE encryptions of two clients' LWE secrets, packed on
  the GPU, decrypt to the LWE phases b + A s mod p (n = 1280, the paper's
  LWE dimension);
* the bench's size (D1 = 2^18, n = 1280, N = 4096, two primes, B = 32): four
  chunks of every client, exactly;
* argument checks: an ordinary database is refused, as are B = 0 and switching
  with more than two primes.
"""

import numpy as np
import pytest

import synth
from oracle import modswitch as oms
from oracle import pack as opk
from oracle import rlwe

from bigcheck import query_ntt
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


def _params(rg, p_log2):
    from paper_2606_11536_amd import pir
    return pir.Params(rg.log2n, list(rg.primes), p_log2)


def _special(seed, B, n, rg):
    return np.stack([synth.uniform_query(seed, beta, n, rg.primes, rg.N) for beta in range(B)]
                    ).astype(np.uint64)                               # [B][n][2][K][N]


@pytest.mark.parametrize("log2n,D1,n,B,p_log2", [(10, 2500, 100, 3, 18), (10, 1024, 100, 1, 18),
                                                 (11, 5000, 1280, 17, 18), (11, 777, 64, 3, 32)])
def test_pack_matches_oracle(ctx, log2n, D1, n, B, p_log2):
    rg = ring(log2n, 2)
    p = 1 << p_log2
    seed = D1 + n + B
    A = synth.lwe_matrix(seed, D1, n, p)
    b = synth.lwe_offsets(seed, B, D1, p)
    ct = _special(seed, B, n, rg)
    H = ctx.load_pack(_params(rg, p_log2), A, D1, n)
    Cp = opk.n_chunks(D1, rg.N)
    assert (H.R, H.C) == (n, Cp)
    out = empty_dev((B, Cp, 2, rg.K, rg.N))
    ctx.pack(H, B, to_dev(ct), to_dev(b), out)
    exp = opk.pack(A, b, ct, rg.primes, rg.psis, p)
    assert np.array_equal(to_host(out), exp)
    sw = empty_dev((B, Cp, 2, rg.N))
    ctx.pack(H, B, to_dev(ct), to_dev(b), sw, switch_bits=29)
    assert np.array_equal(to_host(sw), oms.switch(exp, rg.primes, 29))
    H.free()


def test_packed_ciphertexts_decrypt_to_lwe_phases(ctx):
    rg = ring(11, 2)
    p, D1, n, B, seed = 1 << 18, 3000, 1280, 2, 5
    A = synth.lwe_matrix(seed, D1, n, p)
    b = synth.lwe_offsets(seed, B, D1, p)
    s_lwe = np.stack([synth.lwe_secret(seed, beta, n) for beta in range(B)])
    from oracle import params as op
    delta = op.scale(rg.primes, p)                                     # floor(Q / p)
    cts, keys = [], []
    for beta in range(B):
        key = synth.secret(seed, beta, rg.N)
        m = np.zeros((n, rg.N), dtype=np.int64)
        m[:, 0] = s_lwe[beta]                                          # Delta * s_i, signed
        a = np.stack([synth.mask_row(seed, beta, i, rg.primes, rg.N) for i in range(n)])
        e = np.stack([synth.error_row(seed, beta, i, rg.N) for i in range(n)])
        cts.append(rlwe.encrypt(m, key, a, e, rg.primes, rg.psis, delta))
        keys.append(key)
    H = ctx.load_pack(_params(rg, 18), A, D1, n)
    Cp = opk.n_chunks(D1, rg.N)
    out = empty_dev((B, Cp, 2, rg.K, rg.N))
    ctx.pack(H, B, to_dev(np.stack(cts)), to_dev(b), out)
    got = to_host(out)
    phase = opk.lwe_phase(A, b, s_lwe, p)
    for beta in range(B):
        m, noise = rlwe.decrypt(got[beta], keys[beta], rg.primes, rg.psis, delta, p)
        flat = m.reshape(-1)
        assert np.array_equal(flat[:D1], phase[beta])
        assert not flat[D1:].any()
    H.free()


def test_pack_bench_size_sampled_chunks(ctx):
    import torch
    rg = ring(12, 2)
    p, D1, n, B, seed = 1 << 18, 1 << 18, 1280, 32, 9
    A = synth.lwe_matrix(seed, D1, n, p)
    b = synth.lwe_offsets(seed, B, D1, p)
    pool = _special(seed, 2, n, rg)                                   # two distinct clients' keys
    H = ctx.load_pack(_params(rg, 18), to_dev(A), D1, n)
    Cp = D1 // rg.N
    sp = torch.empty((B, n, 2, rg.K, rg.N), dtype=torch.int32, device="cuda")
    dev_pool = [to_dev(x) for x in pool]
    for beta in range(B):
        sp[beta].copy_(dev_pool[beta % 2])
    out = empty_dev((B, Cp, 2, rg.K, rg.N))
    ctx.pack(H, B, sp, to_dev(b), out)
    torch.cuda.synchronize()
    q_hat = query_ntt(pool, rg.primes, rg.psis)
    from oracle import scan as osc
    for r in (0, 1, 37, Cp - 1):
        rows = slice(r * rg.N, (r + 1) * rg.N)
        h_hat = opk.hint_ntt(A[rows], rg.N, rg.primes, rg.psis)      # [K][n][1][N]
        y = osc.db_mul(h_hat, q_hat, rg.primes)                      # [2][1][2][K][N]
        g = opk.offset_ntt(b[:, rows], rg.N, rg.primes, rg.psis, p)   # [B][1][K][N]
        got = to_host(out[:, r])
        for beta in range(B):
            yb = y[beta % 2, 0].copy()
            for k, q in enumerate(rg.primes):
                yb[1, k] = (yb[1, k] + g[beta, 0, k]) % np.uint64(q)
            exp = osc.answer_intt(yb, rg.primes, rg.psis)
            assert np.array_equal(got[beta], exp), f"chunk {r} client {beta}"
    H.free()


def test_pack_arguments(ctx):
    from paper_2606_11536_amd import pir
    rg = ring(10, 2)
    raw = synth.db_bytes(1, 4, 4, rg.N)
    db = ctx.load_db(rg.pir_params(), raw, 4, 4)
    q = empty_dev((1, 4, 2, rg.K, rg.N))
    bb = empty_dev((1, 4 * rg.N))
    out = empty_dev((1, 4, 2, rg.K, rg.N))
    with pytest.raises(pir.PirError) as e:
        ctx.pack(db, 1, q, bb, out)
    assert e.value.status == 1
    A = synth.lwe_matrix(2, 100, 4, 1 << 18)
    H = ctx.load_pack(_params(rg, 18), A, 100, 4)
    with pytest.raises(pir.PirError) as e:
        ctx.pack(H, 0, q, bb, out)
    assert e.value.status == 1
    db.free()
    H.free()
    rg3 = ring(10, 3)
    H3 = ctx.load_pack(_params(rg3, 18), A, 100, 4)
    with pytest.raises(pir.PirError) as e:
        ctx.pack(H3, 1, q, bb, out, switch_bits=29)
    assert e.value.status == 2
    H3.free()
