"""GPU parity of the answer drain with modulus switching (pir_intt_modswitch).

The fused kernel (inverse NTT per prime, CRT, nearest integer to x 2^bits / Q
mod 2^bits) is compared word for word with the oracle:
* uniform NTT-form residues, N in {1024, 2048, 4096}, one and two primes,
  bits in {29, 20, 32, 1}, a ragged polynomial count;
* at the size of a config-3 batch (32 queries x 1024 columns x 2 = 65536
  polynomials, N = 2048, two primes: 1 GiB in, 512 MiB out) on sampled
  polynomials;
* end to end: one-hot queries scanned by the library, drained through the
  fused kernel, decrypt at 2^29 to the selected database row;
* argument checks: no polynomials is a no-op; bits outside [1, 32] and more
  than two primes are refused; the input is left unchanged.
"""

import numpy as np
import pytest

import synth
from oracle import modswitch as oms
from oracle import params as op
from oracle import query as oq
from oracle import scan as osc

from pirtest import empty_dev, residues, ring, to_dev, to_host

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


@pytest.mark.parametrize("log2n,K,bits", [(10, 1, 29), (10, 2, 29), (11, 2, 29), (12, 2, 29),
                                          (11, 2, 20), (11, 2, 32), (11, 2, 1), (12, 1, 32)])
def test_matches_oracle(ctx, log2n, K, bits):
    rg = ring(log2n, K)
    P = 37
    hat = residues(np.random.default_rng(log2n * 10 + K + bits), (P,), rg)   # [P][K][N]
    src = to_dev(hat)
    out = empty_dev((P, rg.N))
    ctx.intt_modswitch(rg.pir_params(), src, out, bits)
    assert np.array_equal(to_host(out), oms.intt_switch(hat, rg.primes, rg.psis, bits))
    assert np.array_equal(to_host(src), hat)


def test_full_batch_sampled(ctx):
    import torch
    rg = ring(11, 2)
    P = 32 * 1024 * 2
    gen = torch.Generator(device="cuda").manual_seed(9)
    src = torch.empty((P, 2, rg.N), dtype=torch.int32, device="cuda")
    for k, q in enumerate(rg.primes):
        src[:, k].copy_(torch.randint(0, q, (P, rg.N), generator=gen, device="cuda",
                                      dtype=torch.int64).to(torch.int32))
    out = empty_dev((P, rg.N))
    ctx.intt_modswitch(rg.pir_params(), src, out)
    torch.cuda.synchronize()
    pick = np.random.default_rng(4).choice(P, 8, replace=False).tolist() + [0, P - 1]
    hat = to_host(src[pick])
    assert np.array_equal(to_host(out[pick]), oms.intt_switch(hat, rg.primes, rg.psis, 29))


def test_end_to_end_decrypts_at_2_29(ctx):
    rg = ring(11, 2)
    R, C = 24, 40
    raw = synth.db_bytes(77, R, C, rg.N)
    i_star = 13
    ct, s = oq.onehot_query(77, 0, i_star, R, rg.primes, rg.psis, rg.delta, rg.N)
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    q_hat = osc.query_ntt(ct[None], rg.primes, rg.psis)
    ans = empty_dev((1, C, 2, rg.K, rg.N))
    ctx.db_mul(db, to_dev(q_hat), 1, ans)
    out = empty_dev((C, 2, rg.N))
    ctx.intt_modswitch(rg.pir_params(), ans, out)
    got = to_host(out)
    want = oms.intt_switch(to_host(ans)[0], rg.primes, rg.psis)
    assert np.array_equal(got, want)
    m, noise_num = oms.decrypt_switched(got, s, rg.p)
    assert np.array_equal(m, raw[i_star].astype(np.int64))
    assert max(abs(int(v)) for v in noise_num.ravel()) < (1 << 29) // 4
    db.free()


def test_arguments(ctx):
    from paper_2606_11536_amd import pir
    rg = ring(10, 2)
    src = to_dev(np.zeros((2, 2, rg.N), dtype=np.uint64))
    out = empty_dev((2, rg.N))
    ctx.intt_modswitch(rg.pir_params(), src, out, 29, n_polys=0)
    for bits in (0, 33):
        with pytest.raises(pir.PirError):
            ctx.intt_modswitch(rg.pir_params(), src, out, bits)
    q3 = op.ntt_primes(rg.N, 3)
    with pytest.raises(pir.PirError):
        ctx.intt_modswitch(pir.Params(10, q3, 8), src, out, 29, n_polys=1)
