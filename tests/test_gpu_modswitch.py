"""GPU parity of the answer drain with modulus switching (pir_intt_modswitch).

The fused kernel (inverse NTT per prime, CRT, nearest integer to x 2^bits / Q
mod 2^bits) is compared word for word with the oracle:
* uniform NTT-form residues, N in {1024, 2048, 4096}, one and two primes,
  bits in {29, 20, 32, 1}, a ragged polynomial count;
* two primes of very different size (28 and 14 bits), in both orders;
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


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("bits", [29, 32, 7])
def test_unequal_primes_match_oracle(ctx, order, bits):
    """A 28-bit prime beside a 14-bit one (both = 1 mod 2N at N = 1024): the CRT
    step must not assume the primes are of similar size."""
    from oracle import params as op
    from pirtest import Ring
    qs = [op.ntt_primes(1024, 1)[0], 12289]
    qs = qs if order == 0 else qs[::-1]
    rg = Ring(10, qs, [op.psi_min(1024, q) for q in qs], op.scale(qs, 256))
    P = 29
    hat = residues(np.random.default_rng(100 + order * 10 + bits), (P,), rg)
    hat[0, :, :5] = np.array(qs, dtype=np.uint64)[:, None] - 1          # largest residues
    out = empty_dev((P, rg.N))
    ctx.intt_modswitch(rg.pir_params(), to_dev(hat), out, bits)
    assert np.array_equal(to_host(out), oms.intt_switch(hat, rg.primes, rg.psis, bits))


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


JOBS = [(11, 2, 40, 20, 1, 29), (11, 2, 40, 20, 3, 29), (10, 1, 33, 9, 2, 0),
        (11, 2, 64, 17, 5, 24), (10, 2, 70, 12, 1, 0)]


def _batch(ctx, seed):
    rng = np.random.default_rng(seed)
    jobs, checks = [], []
    for n, (log2n, K, R, C, B, bits) in enumerate(JOBS):
        rg = ring(log2n, K)
        raw = synth.db_bytes(seed + n, R, C, rg.N)
        db = ctx.load_db(rg.pir_params(), raw, R, C)
        qc = residues(rng, (B, R, 2), rg)
        out = empty_dev((B, C, 2, rg.N) if bits else (B, C, 2, K, rg.N))
        jobs.append((db, B, to_dev(qc), out, bits))
        y = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), osc.query_ntt(qc, rg.primes, rg.psis),
                       rg.primes)
        checks.append(oms.intt_switch(y, rg.primes, rg.psis, bits) if bits
                      else osc.answer_intt(y, rg.primes, rg.psis))
    return jobs, checks


def test_answer_batch_with_switching(ctx):
    """Batch-1 and batched jobs, with and without a modulus switch, in one call:
    switched answers are [B][C][2][N] words equal to the oracle's switch of the
    oracle's answers; the others are unchanged coefficient-form answers."""
    from paper_2606_11536_amd import pir
    jobs, checks = _batch(ctx, 300)
    ctx.answer_batch(jobs)
    for (db, B, qd, out, bits), exp in zip(jobs, checks):
        assert np.array_equal(to_host(out), exp), (B, bits)
    bad = [(jobs[0][0], 1, jobs[0][2], jobs[0][3], 33)]
    with pytest.raises(pir.PirError):
        ctx.answer_batch(bad)
    for j in jobs:
        j[0].free()


def test_plan_replays_with_switching(ctx):
    """The same job list captured in a HIP graph: three replays, with eager work
    and synchronisation between them, each equal to the oracle."""
    import torch
    jobs, checks = _batch(ctx, 400)
    pl = ctx.plan(jobs)
    scratch = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
    for r in range(3):
        for j in jobs:
            j[3].zero_()
        pl.launch()
        torch.cuda.synchronize()
        for (db, B, qd, out, bits), exp in zip(jobs, checks):
            assert np.array_equal(to_host(out), exp), (r, B, bits)
        scratch.add_(1)
        torch.cuda.synchronize()
    pl.close()
    for j in jobs:
        j[0].free()
